"""End-to-end GPU parity of rrf_randutv / rrf_powerurv against the FP64
oracle on the same input and the same sketch seed.

Gates (FP64 path):
* ||U^T U - I||, ||V^T V - I|| <= 1e-13 and ||A - U T V^T|| / ||A|| <= 1e-13
  (2-norms), T exactly upper trapezoidal;
* randUTV: every b x b diagonal block diagonal, non-negative, descending;
* |T_kk| agrees with the oracle to 1e-10 relative, plus an absolute floor of
  10 n u ||A||: two backward-stable FP64 runs differ by perturbations of
  order n u ||A||, which dominate once T_kk sinks towards that level;
* |T| elementwise within 1e-9 ||A|| on well-conditioned inputs (|T| does not
  depend on the sign rule of the small SVDs).
"""
import numpy as np
import pytest

import oracle
from oracle import metrics as M
from synthetic import gaussian_matrix, spectral_matrix, spectrum

pytestmark = pytest.mark.gpu
U64 = np.finfo(np.float64).eps / 2


def _to_dev(x, gpu):
    import torch
    from paper_2106_13402_amd import colmajor
    return colmajor(torch.as_tensor(np.asfortranarray(x), device=gpu))


def _host(x):
    return None if x is None else x.detach().cpu().numpy()


def _check_factorization(A, U, T, V, tol=1e-13):
    assert M.orth_error(U) <= tol, M.orth_error(U)
    assert M.orth_error(V) <= tol, M.orth_error(V)
    assert M.recon_error(A, U, T, V) <= tol, M.recon_error(A, U, T, V)
    assert np.all(np.tril(T, -1) == 0.0)


def _check_blocks(T, b):
    n = T.shape[1]
    for c0 in range(0, n, b):
        c1 = min(c0 + b, n)
        blk = T[c0:c1, c0:c1]
        assert np.all(blk - np.diag(np.diag(blk)) == 0.0)
        d = np.diag(blk)
        assert np.all(d >= 0) and np.all(np.diff(d) <= 0)


def _diag_parity(T, To, nA, n):
    dg, do = np.abs(np.diag(T)), np.abs(np.diag(To))
    tol = 1e-10 * do + 10 * n * U64 * nA
    bad = np.abs(dg - do) > tol
    assert not bad.any(), (np.flatnonzero(bad)[:5], dg[bad][:5], do[bad][:5])


def _oracle_spread(A, b, q, seed, nsamp=3):
    """|T_kk| of the oracle and how far it moves under backward-error-sized
    perturbations of A (||E|| = n eps ||A||, 3 random draws).

    Where the sketch is numerically rank deficient inside a block the
    trailing sketch directions are fixed by rounding, so T_kk there is not a
    well-posed function of A; any correct FP64 run lands within this envelope.
    """
    n = A.shape[1]
    _, To, _ = oracle.randutv(A, b, q, seed, want_u=False, want_v=False)
    do = np.abs(np.diag(To))
    nA = M.spec(A)
    spread = np.zeros_like(do)
    rng = np.random.default_rng(12345)
    for _ in range(nsamp):
        E = rng.standard_normal(A.shape)
        E *= n * 2 * U64 * nA / np.linalg.norm(E, 2)
        _, Tp, _ = oracle.randutv(A + E, b, q, seed, want_u=False, want_v=False)
        spread = np.maximum(spread, np.abs(np.abs(np.diag(Tp)) - do))
    return To, do, spread


def _diag_parity_derived(T, A, b, q, seed):
    """Strict gate on the well-posed diagonal, magnitude check on the rest.

    Entries whose oracle value moves by less than a tenth of the strict
    tolerance under backward-error-sized perturbations are well-posed and
    must agree to 1e-10 relative (+ 10 n u ||A||). Where the oracle itself
    moves by more, the value is fixed by rounding inside a numerically rank
    deficient sketch and differs between any two correct FP64 runs; there the
    GPU must match the oracle's rank-revealing magnitude (within a factor 2).
    """
    To, do, spread = _oracle_spread(A, b, q, seed)
    n = A.shape[1]
    nA = M.spec(A)
    dg = np.abs(np.diag(T))
    strict = 1e-10 * do + 10 * n * U64 * nA
    posed = spread <= 0.1 * strict
    bad = posed & (np.abs(dg - do) > strict)
    assert not bad.any(), (np.flatnonzero(bad)[:5], dg[bad][:5], do[bad][:5])
    floor = 10 * n * U64 * nA
    ill = ~posed & (do > floor)
    ratio = dg[ill] / do[ill]
    assert np.all((ratio >= 0.5) & (ratio <= 2.0)), (np.flatnonzero(ill)[:5], ratio.min(), ratio.max())
    return To, float(spread.max() / nA)


def run_randutv(A, b, q, seed, gpu, **kw):
    from paper_2106_13402_amd import randutv
    U, T, V = randutv(_to_dev(A, gpu), b, q, seed, **kw)
    return _host(U), _host(T), _host(V)


def test_config1_512_geometric(gpu):
    """512 x 512, s_j = 10^(-12 (j-1)/511), b = 32, q = 1, sketch seed 1."""
    n = 512
    s = spectrum("geometric", n, decades=12.0)
    A = spectral_matrix(n, n, s, seed=0)
    print(f"case: randutv 512x512 geometric b=32 q=1", flush=True)
    U, T, V = run_randutv(A, 32, 1, 1, gpu)
    Uo, To, Vo = oracle.randutv(A, 32, 1, 1)
    nA = s[0]
    _check_factorization(A, U, T, V)
    _check_blocks(T, 32)
    _diag_parity(T, To, nA, n)
    # rank-revealing quality matches the oracle on the k-grid
    ks = np.arange(0, n, 32)
    eg, eo = M.trailing_norms(T, ks), M.trailing_norms(To, ks)
    assert np.all(np.abs(eg - eo) <= 1e-10 * eo + 10 * n * U64 * nA)
    assert np.all(eg >= s[ks] * (1 - 1e-8) - 1e-14)


GRID = [(11, 8, 3), (9, 4, 4), (40, 30, 7), (100, 64, 16), (257, 200, 32), (300, 300, 64),
        (130, 129, 128), (1000, 10, 4), (64, 64, 1)]


@pytest.mark.parametrize("m,n,b", GRID)
@pytest.mark.parametrize("q", [0, 1, 2])
def test_randutv_grid_gaussian(gpu, m, n, b, q):
    print(f"case: randutv gaussian m={m} n={n} b={b} q={q}", flush=True)
    A = gaussian_matrix(m, n, seed=m + n + b)
    U, T, V = run_randutv(A, b, q, 7, gpu)
    nA = M.spec(A)
    _check_factorization(A, U, T, V)
    _check_blocks(T, b)
    To, rel_spread = _diag_parity_derived(T, A, b, q, 7)
    if rel_spread < 1e-12:  # well-posed: the whole of |T| is determined
        np.testing.assert_allclose(np.abs(T), np.abs(To), atol=1e-9 * nA)


@pytest.mark.parametrize("q", [0, 1, 2])
def test_randutv_power_decay_1024(gpu, q):
    """s_j = j^-2 on 1024 x 1024, b = 128 (the second config's spectrum).

    With q >= 1 the sketch (T22^T T22)^q T22^T G spans a range of
    (s_1/s_128)^(2q+1) >= 4e12 inside one block, so its trailing directions
    are set by rounding and T_kk there is not a well-posed function of the
    input: the oracle itself moves by up to 1e-5 (q=1) / 1e-1 (q=2) relative
    when A is perturbed by ||E|| = n eps ||A||, the size of a backward error.
    Such entries are held to the oracle's rank-revealing magnitude (factor 2);
    the well-posed ones, and all of q = 0, to the strict 1e-10 gate.
    """
    n = 1024
    s = spectrum("power", n, p=2.0)
    A = spectral_matrix(n, n, s, seed=0)
    U, T, V = run_randutv(A, 128, q, 1, gpu)
    _check_factorization(A, U, T, V)
    _check_blocks(T, 128)
    if q == 0:
        _, To, _ = oracle.randutv(A, 128, q, 1, want_u=False, want_v=False)
        _diag_parity(T, To, s[0], n)
        return
    _diag_parity_derived(T, A, 128, q, 1)


def _gpu_orth_error(Q, iters=40):
    """||Q^T Q - I||_2 on the device by power iteration on the symmetric
    error matrix (for factors too large to bring to the host)."""
    import torch
    E = Q.T @ Q
    E.diagonal().sub_(1.0)
    x = torch.randn(E.shape[0], 1, dtype=E.dtype, device=E.device,
                    generator=torch.Generator(device=E.device).manual_seed(0))
    lam = 0.0
    for _ in range(iters):
        y = E @ x
        lam = float(torch.linalg.vector_norm(y))
        if lam == 0.0:
            return 0.0
        x = y / lam
    return lam


def test_randutv_tall_panel_split(gpu):
    """m = 20000, n = 384, b = 256 (the shape class of the 32768 x 8192,
    b = 256 configuration): the 20000 x 256 panel of step 1 is taller than
    one panel launch takes and is factored by the column split."""
    from paper_2106_13402_amd import randutv
    m, n, b, q = 20000, 384, 256, 1
    s = spectrum("geometric", n, decades=8.0)
    A = spectral_matrix(m, n, s, seed=0)
    print(f"case: randutv tall split m={m} n={n} b={b} q={q}", flush=True)
    dA = _to_dev(A, gpu)
    U, T, V = randutv(dA, b, q, 1)
    assert _gpu_orth_error(U) <= 1e-13
    Th, Vh = _host(T), _host(V)
    assert M.orth_error(Vh) <= 1e-13
    R = dA - U @ T @ V.T
    assert float(R.norm()) <= 1e-13 * np.linalg.norm(A)  # Frobenius >= spectral
    assert np.all(np.tril(Th, -1) == 0.0)
    _check_blocks(Th, b)
    _diag_parity_derived(Th, A, b, q, 1)


def test_randutv_edge_cases(gpu):
    # zero matrix: T = 0 exactly, U and V orthogonal
    A = np.zeros((50, 40))
    U, T, V = run_randutv(A, 8, 1, 1, gpu)
    assert np.all(T == 0.0)
    assert M.orth_error(U) < 1e-13 and M.orth_error(V) < 1e-13
    # b >= n: one SVD, T = diag(sigma(A))
    A = gaussian_matrix(30, 20, seed=2)
    U, T, V = run_randutv(A, 32, 1, 1, gpu)
    np.testing.assert_allclose(np.diag(T), np.linalg.svd(A, compute_uv=False), rtol=1e-13)
    _check_factorization(A, U, T, V)
    # n = 1
    A = gaussian_matrix(17, 1, seed=3)
    U, T, V = run_randutv(A, 4, 2, 1, gpu)
    assert abs(T[0, 0] - np.linalg.norm(A)) < 1e-14 * np.linalg.norm(A)
    _check_factorization(A, U, T, V)
    # exact rank r
    rng = np.random.default_rng(5)
    A = rng.standard_normal((96, 12)) @ rng.standard_normal((12, 80))
    U, T, V = run_randutv(A, 8, 1, 1, gpu)
    assert M.spec(T[12:, 12:]) < 1e-12 * M.spec(A)
    _check_factorization(A, U, T, V)
    # orthogonal input: T = I
    from synthetic import haar
    A = haar(64, 64, seed=1)
    U, T, V = run_randutv(A, 16, 2, 1, gpu)
    np.testing.assert_allclose(T, np.eye(64), atol=1e-13)


def test_randutv_options_and_layouts(gpu):
    import torch
    from paper_2106_13402_amd import randutv
    A = gaussian_matrix(200, 150, seed=9)
    Uo, To, Vo = oracle.randutv(A, 32, 1, 3)
    # U and V not requested
    _, T, _ = randutv(_to_dev(A, gpu), 32, 1, 3, want_u=False, want_v=False)
    np.testing.assert_allclose(np.abs(_host(T)), np.abs(To), atol=1e-9 * M.spec(A))
    # A a strided sub-block (lda > m)
    big = np.zeros((260, 170))
    big[10:210, 5:155] = A
    dbig = _to_dev(big, gpu)
    U, T, V = randutv(dbig[10:210, 5:155], 32, 1, 3)
    np.testing.assert_allclose(np.abs(_host(T)), np.abs(To), atol=1e-9 * M.spec(A))
    # in place
    dA = _to_dev(A, gpu)
    U, T, V = randutv(dA, 32, 1, 3, inplace=True)
    assert T.data_ptr() == dA.data_ptr()
    np.testing.assert_allclose(np.abs(_host(dA)), np.abs(To), atol=1e-9 * M.spec(A))
    # bitwise determinism
    _, T1, _ = randutv(_to_dev(A, gpu), 32, 1, 3)
    _, T2, _ = randutv(_to_dev(A, gpu), 32, 1, 3)
    assert torch.equal(T1, T2)


@pytest.mark.parametrize("p", [600, -600, 300, -300, 100])
def test_randutv_extreme_scale(gpu, p):
    """Entries near 2^600 (or 2^-600): squared column norms would overflow
    (underflow) binary64; near 2^300 the q = 1 sketch, which grows like
    |A|^3, would. T is then factored from 2^-e A, max|2^-e A| in [0.5, 1),
    and scaled back; 2^100 stays inside the unscaled range (2^150 at q = 1).
    |T_kk| 2^-p matches the oracle on the unscaled A, and U, V and
    A = U T V^T hold to binary64 accuracy."""
    print(f"case: randutv extreme scale 2^{p}", flush=True)
    A = gaussian_matrix(200, 150, seed=11)
    As = A * 2.0 ** p
    U, T, V = run_randutv(As, 32, 1, 3, gpu)
    assert np.all(np.isfinite(T)) and np.all(np.isfinite(U)) and np.all(np.isfinite(V))
    assert M.orth_error(U) <= 1e-13 and M.orth_error(V) <= 1e-13
    R = A - U @ (T * 2.0 ** -p) @ V.T
    assert M.spec(R) <= 1e-13 * M.spec(A)
    _, To, _ = oracle.randutv(A, 32, 1, 3, want_u=False, want_v=False)
    _diag_parity(T * 2.0 ** -p, To, M.spec(A), 150)


def test_randutv_rejects_nonfinite(gpu):
    from paper_2106_13402_amd import RRFError, randutv
    A = gaussian_matrix(40, 30, seed=1)
    A[3, 4] = np.nan
    with pytest.raises(RRFError) as e:
        randutv(_to_dev(A, gpu), 8, 1, 1, check_finite=True)
    assert e.value.status == 4


# ---------------------------------------------------------------- powerURV
@pytest.mark.parametrize("m,n,b", [(40, 30, 8), (300, 256, 64), (512, 512, 128), (700, 300, 32)])
@pytest.mark.parametrize("q", [0, 1, 2])
def test_powerurv_parity(gpu, m, n, b, q):
    from paper_2106_13402_amd import powerurv
    print(f"case: powerurv m={m} n={n} b={b} q={q}", flush=True)
    s = np.linspace(2.0, 1.0, n)
    A = spectral_matrix(m, n, s, seed=m + n)
    U, T, V = (_host(x) for x in powerurv(_to_dev(A, gpu), q, 1, b=b))
    Uo, To, Vo = oracle.powerurv(A, q, 1)
    _check_factorization(A, U, T, V)
    _diag_parity(T, To, 2.0, n)
    np.testing.assert_allclose(np.abs(T), np.abs(To), atol=1e-9 * 2.0)


def _powerurv_spread(A, q, seed, nsamp=3):
    """|T_kk| of the powerURV oracle and its largest change under three
    backward-error-sized perturbations of A (||E||_2 = n eps ||A||_2)."""
    n = A.shape[1]
    _, To, _ = oracle.powerurv(A, q, seed)
    do = np.abs(np.diag(To))
    nA = M.spec(A)
    spread = np.zeros_like(do)
    rng = np.random.default_rng(12345)
    for _ in range(nsamp):
        E = rng.standard_normal(A.shape)
        E *= n * 2 * U64 * nA / np.linalg.norm(E, 2)
        _, Tp, _ = oracle.powerurv(A + E, q, seed)
        spread = np.maximum(spread, np.abs(np.abs(np.diag(Tp)) - do))
    return To, do, spread


@pytest.mark.parametrize("kind", ["power", "geometric"])
@pytest.mark.parametrize("q", [0, 1, 2])
def test_powerurv_decaying_1024(gpu, kind, q):
    """powerURV (Alg. 1) in FP64 at 1024 x 1024 on decaying spectra, s_j = j^-2
    and s_j = 10^(-12 (j-1)/1023), where the QRs of the power products are
    ill-conditioned: |T_kk| equal to the oracle's to 1e-10 relative plus
    10 n u ||A|| where the value is well posed (the oracle's own spread under
    backward-error-sized perturbations is below a tenth of that), within a
    factor 2 elsewhere; e_k equal to the oracle's on a k-grid to the same
    tolerance when every |T_kk| is well posed, and never below s_{k+1}."""
    from paper_2106_13402_amd import powerurv
    n = 1024
    s = spectrum("power", n, p=2.0) if kind == "power" else spectrum("geometric", n, decades=12.0)
    A = spectral_matrix(n, n, s, seed=0)
    print(f"case: powerurv FP64 {kind} n={n} q={q}", flush=True)
    U, T, V = (_host(x) for x in powerurv(_to_dev(A, gpu), q, 1, b=128))
    _check_factorization(A, U, T, V)
    To, do, spread = _powerurv_spread(A, q, 1)
    nA = s[0]
    dg = np.abs(np.diag(T))
    strict = 1e-10 * do + 10 * n * U64 * nA
    posed = spread <= 0.1 * strict
    bad = posed & (np.abs(dg - do) > strict)
    assert not bad.any(), (np.flatnonzero(bad)[:5], dg[bad][:5], do[bad][:5])
    ill = ~posed & (do > 10 * n * U64 * nA)
    if ill.any():
        r = dg[ill] / do[ill]
        assert np.all((r >= 0.5) & (r <= 2.0)), (r.min(), r.max())
    ks = [0, 1, 16, 64, 127, 128, 256, 512, 900]
    eg, eo = M.trailing_norms(T, ks), M.trailing_norms(To, ks)
    if posed.all():
        assert np.all(np.abs(eg - eo) <= 1e-10 * eo + 10 * n * U64 * nA), (eg, eo)
    else:
        assert np.all((eg >= eo / 1.5) & (eg <= 1.5 * eo)), (eg, eo)
    assert np.all(eg >= s[ks] * (1 - 1e-8) - 10 * n * U64 * nA)


@pytest.mark.parametrize("m,n,b,q", [(200, 330, 64, 1), (129, 300, 32, 2)])
def test_powerurv_wide_through_transpose(gpu, m, n, b, q):
    """m < n through the transpose (the Sec. 3.2 reading, as for randUTV):
    T = T'^T lower trapezoidal, U m x m, V n x n, and |T| equal to the
    oracle's, which takes the same route."""
    from paper_2106_13402_amd import powerurv
    print(f"case: powerurv wide m={m} n={n} b={b} q={q}", flush=True)
    s = np.linspace(2.0, 1.0, m)
    A = spectral_matrix(n, m, s, seed=m + n).T.copy(order="F")
    U, T, V = (_host(x) for x in powerurv(_to_dev(A, gpu), q, 1, b=b))
    assert U.shape == (m, m) and T.shape == (m, n) and V.shape == (n, n)
    _check_factorization(A.T, V, T.T, U)
    _, To, _ = oracle.powerurv(A, q, 1)
    _diag_parity(T, To, 2.0, n)
    np.testing.assert_allclose(np.abs(T), np.abs(To), atol=1e-9 * 2.0)


# ------------------------------------------------ powerURV, bfloat16 power products
POWER_MIXED = [(300, 256, 32, 1, 64.0), (400, 256, 64, 2, 40.0), (256, 256, 16, 2, 1e9),
               (520, 300, 128, 1, 75.0)]


@pytest.mark.parametrize("m,n,b,q,scale", POWER_MIXED)
def test_powerurv_bf16_parity(gpu, m, n, b, q, scale):
    """GPU against the oracle's mixed mode (same rounded operands; the GPU
    accumulates in FP32, the oracle in FP64): |T_kk| agree to a median of
    1e-5 ||A|| and at most 2e-4 ||A|| (FP32 accumulation over K <= 520
    terms: ~K 2^-24 relative in the worst case, far less typically; an FP32
    emulation on the CPU gives medians 3e-8 to 2.4e-6), while the FP64 path
    sits 6e-5 to 7e-5 away in the median, which the first bound excludes. U, V orthogonal and A = U T V^T to FP64 accuracy (the QRs,
    the Q factors and A V are FP64). scale = 1e9 is the linear spectrum."""
    from paper_2106_13402_amd import powerurv
    print(f"case: powerurv bf16 m={m} n={n} b={b} q={q}", flush=True)
    j = np.arange(n, dtype=float)
    s = 1.0 - j / (2 * n) if scale > 1e8 else np.exp(-j / scale)
    A = spectral_matrix(m, n, s, seed=m + n + q)
    U, T, V = (_host(x) for x in powerurv(_to_dev(A, gpu), q, 1, b=b, precision="bf16_sketch"))
    _check_factorization(A, U, T, V)
    _, To, _ = oracle.powerurv(A, q, 1, precision="bf16")
    _, T64, _ = oracle.powerurv(A, q, 1)
    d = np.abs(np.abs(np.diag(T)) - np.abs(np.diag(To))) / s[0]
    d64 = np.abs(np.abs(np.diag(T64)) - np.abs(np.diag(To))) / s[0]
    assert np.median(d) <= 1e-5 and d.max() <= 2e-4, (np.median(d), d.max())
    assert np.median(d64) > 4 * np.median(d)  # the bound tells the modes apart


def test_powerurv_bf16_gate_1024(gpu):
    """1024 x 1024, s_j = exp(-j/200), q = 2: e_k of the mixed mode within
    max(1.5 sigma_{k+1}, 1.1 x the FP64 oracle envelope over 5 sketch seeds)."""
    from paper_2106_13402_amd import powerurv
    n = 1024
    s = np.exp(-np.arange(n) / 200.0)
    A = spectral_matrix(n, n, s, seed=9)
    U, T, V = (_host(x) for x in powerurv(_to_dev(A, gpu), 2, 1, b=128,
                                          precision="bf16_sketch"))
    _check_factorization(A, U, T, V)
    ks = list(range(0, n, 64))
    env = np.zeros(len(ks))
    for seed in range(5):
        _, To, _ = oracle.powerurv(A, 2, 100 + seed)
        env = np.maximum(env, [M.spec(To[k:, k:]) for k in ks])
    ek = [M.spec(T[k:, k:]) for k in ks]
    bad = [k for i, k in enumerate(ks) if ek[i] > max(1.5 * s[k], 1.1 * env[i])]
    assert not bad, bad


def test_powerurv_bf16_resolution_limit(gpu):
    """1024 x 1024, s_j = exp(-j/80) (down to 3e-6), q = 2: the gate holds
    where sigma_{k+1} >= 1e-3 sigma_1; below, where the bfloat16 power
    products no longer separate directions, e_k stays within 10x the FP64
    envelope (a bounded, documented limit, not a pass of the gate)."""
    from paper_2106_13402_amd import powerurv
    n = 1024
    s = np.exp(-np.arange(n) / 80.0)
    A = spectral_matrix(n, n, s, seed=10)
    U, T, V = (_host(x) for x in powerurv(_to_dev(A, gpu), 2, 1, b=128,
                                          precision="bf16_sketch"))
    _check_factorization(A, U, T, V)
    ks = list(range(0, n, 64))
    env = np.zeros(len(ks))
    for seed in range(3):
        _, To, _ = oracle.powerurv(A, 2, 100 + seed)
        env = np.maximum(env, [M.spec(To[k:, k:]) for k in ks])
    ek = np.array([M.spec(T[k:, k:]) for k in ks])
    hi = [i for i, k in enumerate(ks) if s[k] >= 1e-3]
    assert all(ek[i] <= max(1.5 * s[ks[i]], 1.1 * env[i]) for i in hi)
    assert np.all(ek <= 10 * env), (ek / env).max()


# ------------------------------------------------------- mixed-precision sketch
_ENVELOPES = {}


def _oracle_envelope(A, b, q, seeds, ks):
    """Largest e_k = ||T(k:, k:)||_2 over FP64 oracle runs with several sketch
    seeds: the spread of the randomized algorithm itself. Computed once per
    (input, b, q, seeds) on the grid k = 0, n/64, ... and kept for the
    session (the mixed-mode tests of every precision share it)."""
    import hashlib
    n = A.shape[1]
    grid = list(range(0, n, max(1, n // 64)))
    key = (hashlib.sha1(np.ascontiguousarray(A).tobytes()).hexdigest(), A.shape, b, q,
           tuple(seeds))
    if key not in _ENVELOPES:
        env = np.zeros(len(grid))
        for sd in seeds:
            _, To, _ = oracle.randutv(A, b, q, sd, want_u=False, want_v=False)
            env = np.maximum(env, M.trailing_norms(To, grid))
        _ENVELOPES[key] = dict(zip(grid, env))
    table = _ENVELOPES[key]
    return np.array([table[k] for k in ks])


def _mixed_gate(T, A, b, q, seed, s, rec_err, factor=1.1):
    """e_k <= max(1.5 sigma_{k+1}, factor * e_k^FP64) for every k on the grid
    with sigma_{k+1} >= 100 rec_err ||A||, e_k = ||T(k:, k:)||_2.

    The mixed sketch perturbs each step's subspace at the bfloat16 level, so
    the run follows a different (equally valid) random trajectory from the
    oracle's; e_k^FP64 is therefore the envelope of FP64 oracle runs over the
    same seed and others (12 in all up to n = 1024, 5 above). At q = 0 the
    FP64 runs themselves spread from 1.5 to 1.95 sigma_{k+1} at block edges,
    and the mixed mode's distribution is the same (checked over 12 seeds with
    the CPU reference of the mixed sketch)."""
    n = T.shape[1]
    ks = [k for k in range(0, n, max(1, n // 64)) if s[k] >= 100 * rec_err * s[0]]
    eg = M.trailing_norms(T, ks)
    nseeds = 12 if n <= 1024 else 5
    eo = _oracle_envelope(A, b, q, [seed + 101 * t for t in range(nseeds)], ks)
    bad = [(k, g, o, s[k]) for k, g, o in zip(ks, eg, eo) if g > max(1.5 * s[k], factor * o)]
    assert not bad, bad[:5]
    return max(g / o for g, o in zip(eg, eo))


def _run_mixed(A, b, q, seed, gpu):
    from paper_2106_13402_amd import randutv
    U, T, V = (_host(x) for x in randutv(_to_dev(A, gpu), b, q, seed, precision="bf16_sketch"))
    _check_factorization(A, U, T, V)
    _check_blocks(T, b)
    return U, T, V


@pytest.mark.parametrize("q", [0, 1, 2])
def test_randutv_bf16_sketch_headline_spectrum(gpu, q):
    """The headline input class, s_j = exp(-j/800), at 2048 x 2048 and b = 128:
    the spectrum falls by a factor 0.85 across a block, far above what the
    bfloat16 sketch resolves, and the FP64 parts keep the factorization exact
    (orthogonal U, V; backward error ~ u)."""
    n, b = 2048, 128
    s = spectrum("exp", n, scale=800.0)
    A = spectral_matrix(n, n, s, seed=0)
    print(f"case: randutv bf16 sketch exp(-j/800) n={n} q={q}", flush=True)
    U, T, V = _run_mixed(A, b, q, 1, gpu)
    _mixed_gate(T, A, b, q, 1, s, M.recon_error(A, U, T, V))


@pytest.mark.parametrize("q", [0, 1, 2])
def test_randutv_bf16_sketch_geometric(gpu, q):
    """512 x 512, s_j = 10^(-12 (j-1)/511), b = 32: 0.75 decades per block."""
    n = 512
    s = spectrum("geometric", n, decades=12.0)
    A = spectral_matrix(n, n, s, seed=0)
    print(f"case: randutv bf16 sketch 512 geometric q={q}", flush=True)
    U, T, V = _run_mixed(A, 32, q, 1, gpu)
    _mixed_gate(T, A, 32, q, 1, s, M.recon_error(A, U, T, V))


@pytest.mark.parametrize("m,n,b,q", [(1000, 700, 64, 1), (64, 64, 1, 1), (600, 600, 96, 2)])
def test_randutv_bf16_sketch_shapes(gpu, m, n, b, q):
    s = spectrum("exp", n, scale=n / 2.0)
    A = spectral_matrix(m, n, s, seed=1)
    print(f"case: randutv bf16 sketch m={m} n={n} b={b} q={q}", flush=True)
    U, T, V = _run_mixed(A, b, q, 3, gpu)
    _mixed_gate(T, A, b, q, 3, s, M.recon_error(A, U, T, V))


def test_randutv_bf16_sketch_steep_block_limit(gpu):
    """Known limit of the bfloat16 power iteration: with q power steps the
    sketch cannot separate directions whose singular values fall below about
    (2^-8)^(1/(2q+1)) of the block's leading one (0.33 at q = 2). With
    s_j = exp(-j/30) and b = 100 the spectrum falls 27x inside a block, so the
    mixed mode's e_k at block edges is up to ~1.5x the FP64 value; the
    factorization itself stays exact and the loss stays bounded (2x)."""
    m, n, b, q = 513, 300, 100, 2
    s = spectrum("exp", n, scale=30.0)
    A = spectral_matrix(m, n, s, seed=1)
    U, T, V = _run_mixed(A, b, q, 3, gpu)
    worst = _mixed_gate(T, A, b, q, 3, s, M.recon_error(A, U, T, V), factor=2.0)
    print(f"steep spectrum: worst e_k(mixed) / e_k(FP64 envelope) = {worst:.2f}", flush=True)


@pytest.mark.parametrize("m,n,b,q,precision", [(300, 500, 64, 1, "fp64"), (129, 1000, 32, 2, "fp64"),
                                               (400, 640, 64, 1, "bf16_sketch")])
def test_randutv_wide_through_transpose(gpu, m, n, b, q, precision):
    """m < n (Sec. 3.2): the factorization of A^T, transposed back: T lower
    trapezoidal and |T| equal to the oracle's (which takes the same route)."""
    from paper_2106_13402_amd import randutv
    print(f"case: randutv wide m={m} n={n} b={b} q={q} {precision}", flush=True)
    A = gaussian_matrix(n, m, seed=m + n).T.copy(order="F")
    U, T, V = (_host(x) for x in randutv(_to_dev(A, gpu), b, q, 5, precision=precision))
    assert U.shape == (m, m) and T.shape == (m, n) and V.shape == (n, n)
    assert np.all(np.triu(T, 1) == 0.0)
    assert M.orth_error(U) <= 1e-13 and M.orth_error(V) <= 1e-13
    assert M.recon_error(A, U, T, V) <= 1e-13
    if precision == "fp64":
        _, To, _ = oracle.randutv(A, b, q, 5, want_u=False, want_v=False)
        np.testing.assert_allclose(np.abs(T), np.abs(To), rtol=0, atol=1e-9 * M.spec(A))
