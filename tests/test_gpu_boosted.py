"""GPU parity of rrf_randutv_boosted (Alg. 2) against the FP64 oracle
(oracle/randutv_boosted.py) on the same input and sketch seed.

Gates, as for Alg. 3: U and V orthogonal and A = U T V^T to 1e-13, T
upper trapezoidal with diagonal, non-negative, descending b x b blocks,
|T_kk| equal to the oracle's to 1e-10 relative plus 10 n u ||A||, and every
entry of |T| within 1e-9 ||A|| of the oracle's, where the singular vectors
that fix V_i are well conditioned. On the 2048 x 2048 case with 256-wide
samples of a slowly decaying spectrum they are not, and both bounds widen by
4 x the oracle's own movement under backward-error-sized perturbations of A.
The recycled samples are checked on an exact-rank input where they make
every block exact, and the accuracy gain over Alg. 3 on graded spectra.
"""
import numpy as np
import pytest

import oracle
from oracle import metrics as M
from oracle.randutv_boosted import randutv_boosted as boosted_ref
from synthetic import gaussian_matrix, spectral_matrix, spectrum

from test_gpu_factorizations import (_check_blocks, _check_factorization, _diag_parity, _host,
                                     _to_dev, U64)

pytestmark = pytest.mark.gpu


def _run(A, b, q, p, seed, gpu, **kw):
    from paper_2106_13402_amd import randutv_boosted
    out = randutv_boosted(_to_dev(A, gpu), b, q, p, seed, **kw)
    return tuple(_host(x) if x is not None else None for x in out)


def _oracle_spread(A, b, q, p, seed, To, nsamp=2):
    """Elementwise max over backward-error-sized perturbations of A
    (||E|| = n eps ||A||) of how far the oracle's |T| moves: the conditioning
    of the output itself. V_i is built from individual singular vectors of
    the sample matrix, so where its singular values lie close together (a
    slowly decaying spectrum sampled 256 wide) rounding moves T more than in
    Alg. 3; any two correct FP64 runs then differ by about this much."""
    m, n = A.shape
    nA = M.spec(A)
    spread = np.zeros_like(To)
    for t in range(nsamp):
        E = gaussian_matrix(m, n, seed=900 + t)
        E *= n * np.finfo(np.float64).eps * nA / M.spec(E)
        _, Tp, _ = boosted_ref(A + E, b, q, p, seed, want_u=False, want_v=False)
        spread = np.maximum(spread, np.abs(np.abs(Tp) - np.abs(To)))
    return spread


def _parity(A, b, q, p, seed, gpu, derived=False):
    U, T, V = _run(A, b, q, p, seed, gpu)
    _check_factorization(A, U, T, V)
    _check_blocks(T, b)
    _, To, _ = boosted_ref(A, b, q, p, seed, want_u=False, want_v=False)
    nA = M.spec(A)
    if not derived:
        _diag_parity(T, To, nA, A.shape[1])
        np.testing.assert_allclose(np.abs(T), np.abs(To), rtol=0, atol=1e-9 * nA)
        return U, T, V
    spread = _oracle_spread(A, b, q, p, seed, To)
    n = A.shape[1]
    dg, do, ds = np.abs(np.diag(T)), np.abs(np.diag(To)), np.diag(spread)
    tol = 1e-10 * do + 10 * n * U64 * nA + 4 * ds
    bad = np.abs(dg - do) > tol
    print(f"  oracle spread: max {spread.max() / nA:.2e} ||A||, diagonal {ds.max() / nA:.2e}; "
          f"GPU - oracle: diagonal {np.abs(dg - do).max() / nA:.2e}", flush=True)
    assert not bad.any(), (np.flatnonzero(bad)[:5], (dg - do)[bad][:5], ds[bad][:5])
    # elementwise, against the spread's maximum over each b x b tile (two
    # perturbations estimate the conditioning of single entries only roughly)
    m_, n_ = T.shape
    tiles = spread.copy()
    for r0 in range(0, m_, b):
        for c0 in range(0, n_, b):
            tiles[r0:r0 + b, c0:c0 + b] = spread[r0:r0 + b, c0:c0 + b].max()
    dev = np.abs(np.abs(T) - np.abs(To))
    ratio = dev / (1e-9 * nA + 4 * tiles)
    print(f"  elementwise: worst (GPU - oracle) / bound = {ratio.max():.3f}", flush=True)
    assert np.all(ratio <= 1.0)
    return U, T, V


@pytest.mark.parametrize("m,n,b,q,p", [
    (600, 400, 32, 1, 32),   # p = b, several steps, ragged last block
    (513, 300, 64, 2, 16),   # tall, odd m
    (256, 256, 32, 0, 32),   # q = 0: later steps sample X = G
    (300, 120, 16, 1, 100),  # p clipped to N_i - b as the blocks shrink
    (64, 64, 8, 1, 0),       # p = 0
    (200, 200, 100, 1, 100), # b + p = 200 in one panel, two steps
])
def test_boosted_parity_gaussian(gpu, m, n, b, q, p):
    print(f"case: boosted gaussian m={m} n={n} b={b} q={q} p={p}", flush=True)
    A = gaussian_matrix(m, n, seed=m + n + p)
    _parity(A, b, q, p, 11, gpu)


@pytest.mark.parametrize("q", [1, 2])
def test_boosted_parity_graded(gpu, q):
    """512 x 512, s_j = 10^(-6 (j-1)/511), b = p = 32."""
    print(f"case: boosted graded q={q}", flush=True)
    n = 512
    A = spectral_matrix(n, n, spectrum("geometric", n, decades=6.0), seed=0)
    _parity(A, 32, q, 32, 1, gpu)


def test_boosted_parity_b128_p128(gpu):
    """2048 x 2048, b = p = 128, q = 2: 256-wide samples (panels split by
    columns) and 256 x 256 SVDs of R_Y."""
    print("case: boosted n=2048 b=128 p=128 q=2", flush=True)
    n = 2048
    A = spectral_matrix(n, n, spectrum("exp", n, scale=800.0), seed=0)
    _parity(A, 128, 2, 128, 1, gpu, derived=True)


@pytest.mark.parametrize("square", [False, True])
def test_boosted_recycled_samples_exact_on_low_rank(gpu, square):
    """Rank 12, b = 4, p = 12, q = 0: every later block takes the exact top-b
    singular values of its trailing block (the oracle pin, on the GPU)."""
    print(f"case: boosted exact rank square={square}", flush=True)
    n = 40
    m = n if square else 60
    s = np.zeros(n)
    s[:12] = 2.0 ** -np.arange(12) * (1 + 0.1 * np.arange(12) / 12)
    A = spectral_matrix(m, n, s, seed=3)
    _, T, _ = _run(A, 4, 0, 12, 7, gpu, want_u=False, want_v=False)
    for c0 in (4, 8):
        sv = np.linalg.svd(T[c0:, c0:], compute_uv=False)[:4]
        np.testing.assert_allclose(np.diag(T)[c0:c0 + 4], sv, rtol=1e-10)
    assert np.abs(T[12:, 12:]).max() < 1e-14


def test_boosted_beats_basic_at_block_edges(gpu):
    """1024 x 1024, s_j = 1e-5^((j-1)/1023), b = p = 64, q = 1: the largest
    e_k / sigma_{k+1} of Alg. 2 is below 0.9 x that of Alg. 3 (same seed)."""
    from paper_2106_13402_amd import randutv
    print("case: boosted vs basic accuracy", flush=True)
    n, b = 1024, 64
    s = spectrum("fast", n)
    A = spectral_matrix(n, n, s, seed=2)
    _, Tb, _ = _run(A, b, 1, b, 1, gpu, want_u=False, want_v=False)
    T3 = _host(randutv(_to_dev(A, gpu), b, 1, 1, want_u=False, want_v=False)[1])
    ks = np.arange(0, n - 1, 4)
    rb = np.max(M.trailing_norms(Tb, ks) / s[ks])
    r3 = np.max(M.trailing_norms(T3, ks) / s[ks])
    print(f"  max e_k/sigma: boosted {rb:.3f}, basic {r3:.3f}", flush=True)
    assert rb < 0.9 * r3


@pytest.mark.parametrize("m,n,b,q,p", [(300, 500, 32, 1, 32), (120, 257, 16, 2, 8)])
def test_boosted_wide_through_transpose(gpu, m, n, b, q, p):
    """m < n through the transpose (Sec. 3.2, as for Alg. 3): T = T'^T lower
    trapezoidal with diagonal blocks, |T| equal to the oracle's."""
    print(f"case: boosted wide m={m} n={n} b={b} q={q} p={p}", flush=True)
    A = gaussian_matrix(n, m, seed=m + n + p).T.copy(order="F")
    U, T, V = _run(A, b, q, p, 11, gpu)
    assert U.shape == (m, m) and T.shape == (m, n) and V.shape == (n, n)
    _check_factorization(A.T, V, T.T, U)
    _check_blocks(T.T, b)
    _, To, _ = boosted_ref(A, b, q, p, 11, want_u=False, want_v=False)
    nA = M.spec(A)
    _diag_parity(T, To, nA, n)
    np.testing.assert_allclose(np.abs(T), np.abs(To), rtol=0, atol=1e-9 * nA)
