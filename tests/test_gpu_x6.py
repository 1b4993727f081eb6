"""GPU checks of the split-bfloat16 six-term product (rrf_gemm_x6) and of
randUTV with it in every update of T, U and V (RRF_PREC_BF16_X6).

Kernel: the GPU result against the oracle's definition of the product
(oracle.bf16.gemm_x6: the same three-part split, the six exact terms summed in
FP64); the two differ only by the binary32 sums of each K slice
(fp32_x6_bound) and the FP64 rounding of alpha v + beta C. A closed form pins
the split and the six terms to the last bit.

Factorization: the x6 products carry about 1e-8 relative error (of
|A| |B|), which the accumulation of U and V from Householder transforms
amplifies about a thousandfold (the same accumulation with binary64
products stays orthogonal to 1e-14): U and V hold to about 1e-5 and
A = U T V^T to a few 1e-6 up to n = 2048, about 20x closer than the x3
mode. The gate on e_k is the mixed gate (e_k within max(1.5 sigma_{k+1},
1.1 x the FP64 oracle envelope) wherever sigma_{k+1} is above 100 x the
reconstruction error).
"""
import numpy as np
import pytest

from oracle import metrics as M
from oracle.bf16 import fp32_x6_bound, gemm_x6 as gemm_x6_ref
from synthetic import spectral_matrix, spectrum

from test_gpu_factorizations import _check_blocks, _host, _mixed_gate, _to_dev

pytestmark = pytest.mark.gpu
U64 = np.finfo(np.float64).eps / 2

CASES = [
    (1, 1, 1), (17, 33, 5), (64, 64, 64), (130, 70, 300), (257, 129, 1000),
    (200, 128, 5000),   # skinny: split-K path
    (3000, 128, 4100),  # update-like, split-K, ragged K and M
    (1000, 1100, 256),  # rank-2b update shape
]


@pytest.mark.parametrize("M,N,K", CASES)
@pytest.mark.parametrize("ta,tb", [(False, False), (True, False), (False, True), (True, True)])
def test_gemm_x6_matches_oracle(gpu, M, N, K, ta, tb):
    from paper_2106_13402_amd import gemm_x6
    print(f"case: gemm_x6 M={M} N={N} K={K} ta={ta} tb={tb}", flush=True)
    rng = np.random.default_rng(M * 7 + N * 3 + K + 2 * ta + tb)
    A = rng.standard_normal((K, M) if ta else (M, K)) * 2.0 ** rng.integers(-6, 6, (K, M) if ta else (M, K))
    B = rng.standard_normal((N, K) if tb else (K, N))
    C0 = rng.standard_normal((M, N))
    alpha, beta = -0.75, 1.25
    Cd = _to_dev(C0, gpu)
    gemm_x6(_to_dev(A, gpu), _to_dev(B, gpu), transa=ta, transb=tb, alpha=alpha, beta=beta,
            C_out=Cd)
    opA = A.T if ta else A
    opB = B.T if tb else B
    ref = alpha * gemm_x6_ref(opA, opB) + beta * C0
    bound = abs(alpha) * fp32_x6_bound(opA, opB) + 4 * U64 * (np.abs(ref) + abs(beta) * np.abs(C0))
    err = np.abs(_host(Cd) - ref)
    assert np.all(err <= bound), float((err / bound).max())
    # and about 2^-22 of |A| |B| from the binary64 product
    exact = alpha * (opA @ opB) + beta * C0
    scale = np.abs(opA) @ np.abs(opB)
    assert np.all(np.abs(_host(Cd) - exact) <= 2.0 ** -21 * scale + 1e-15 * np.abs(exact))


def test_gemm_x6_closed_form(gpu):
    """a = 1 + 2^-9 + 2^-18 splits as hi = 1, mid = 2^-9, lo = 2^-18; the six
    terms of a a give exactly 1 + 2^-8 + 2^-17 + 2^-18 (mid lo, lo mid and
    lo lo dropped)."""
    from paper_2106_13402_amd import gemm_x6
    print("case: gemm_x6 closed form", flush=True)
    a = np.array([[1.0 + 2.0 ** -9 + 2.0 ** -18]])
    c = _host(gemm_x6(_to_dev(a, gpu), _to_dev(a, gpu)))
    assert c[0, 0] == 1.0 + 2.0 ** -8 + 2.0 ** -17 + 2.0 ** -18


def test_gemm_x6_strided_and_unaligned(gpu):
    from paper_2106_13402_amd import gemm_x6
    print("case: gemm_x6 strided", flush=True)
    rng = np.random.default_rng(5)
    big = rng.standard_normal((701, 650))
    Bm = rng.standard_normal((601, 40))
    sub = _to_dev(big, gpu)[51:651, 31:621]
    Bs = _to_dev(Bm, gpu)[1:601]
    Cd = gemm_x6(sub, Bs, transa=True)
    opA = big[51:651, 31:621].T
    ref = gemm_x6_ref(opA, Bm[1:601])
    err = np.abs(_host(Cd) - ref)
    assert np.all(err <= fp32_x6_bound(opA, Bm[1:601]) + 4 * U64 * np.abs(ref))


# ------------------------------------------------------------ factorization
def _factor_x6(A, b, q, seed, gpu):
    from paper_2106_13402_amd import randutv
    return tuple(_host(x) for x in randutv(_to_dev(A, gpu), b, q, seed, precision="bf16_x6"))


def _check_x6(A, U, T, V, b, orth_tol=2e-5, rec_tol=5e-6):
    eo = max(M.orth_error(U), M.orth_error(V))
    rec = M.recon_error(A, U, T, V)
    print(f"  x6: orthogonality {eo:.2e}, ||A - U T V^T|| / ||A|| = {rec:.2e}", flush=True)
    assert eo <= orth_tol and rec <= rec_tol
    assert np.all(np.tril(T, -1) == 0.0)
    _check_blocks(T, b)
    return rec


@pytest.mark.parametrize("q", [1, 2])
def test_randutv_x6_headline_spectrum(gpu, q):
    """2048 x 2048, s_j = exp(-j/800), b = 128."""
    n, b = 2048, 128
    s = spectrum("exp", n, scale=800.0)
    A = spectral_matrix(n, n, s, seed=0)
    print(f"case: randutv x6 exp(-j/800) n={n} q={q}", flush=True)
    U, T, V = _factor_x6(A, b, q, 1, gpu)
    rec = _check_x6(A, U, T, V, b)
    _mixed_gate(T, A, b, q, 1, s, rec)


@pytest.mark.parametrize("m,n,b,q", [(1000, 700, 64, 1), (600, 600, 96, 2), (64, 64, 1, 1)])
def test_randutv_x6_shapes(gpu, m, n, b, q):
    s = spectrum("exp", n, scale=n / 2.0)
    A = spectral_matrix(m, n, s, seed=1)
    print(f"case: randutv x6 m={m} n={n} b={b} q={q}", flush=True)
    U, T, V = _factor_x6(A, b, q, 3, gpu)
    rec = _check_x6(A, U, T, V, b)
    _mixed_gate(T, A, b, q, 3, s, rec)


def test_randutv_x6_vs_x3_and_scaling(gpu):
    """The x6 updates are in use: at least 30x more accurate than x3 on the
    same input; inputs that differ by a power of two give the same U, V and
    T scaled exactly; repeated runs are bitwise identical."""
    from paper_2106_13402_amd import randutv
    n, b = 512, 64
    A = spectral_matrix(n, n, spectrum("exp", n, scale=200.0), seed=4)
    print("case: randutv x6 vs x3", flush=True)
    U3, T3, V3 = (_host(x) for x in randutv(_to_dev(A, gpu), b, 1, 7, precision="bf16_x3"))
    U6, T6, V6 = _factor_x6(A, b, 1, 7, gpu)
    r3, r6 = M.recon_error(A, U3, T3, V3), M.recon_error(A, U6, T6, V6)
    assert r6 * 30 <= r3, (r6, r3)
    U7, T7, V7 = _factor_x6(A * 2.0 ** 300, b, 1, 7, gpu)
    np.testing.assert_array_equal(U7, U6)
    np.testing.assert_array_equal(V7, V6)
    np.testing.assert_array_equal(T7, T6 * 2.0 ** 300)


def test_randutv_x6_wide(gpu):
    m, n, b, q = 300, 520, 64, 1
    s = spectrum("exp", m, scale=m / 2.0)
    A = spectral_matrix(n, m, s, seed=2).T.copy(order="F")
    print(f"case: randutv x6 wide m={m} n={n} b={b} q={q}", flush=True)
    U, T, V = _factor_x6(A, b, q, 3, gpu)
    assert U.shape == (m, m) and T.shape == (m, n) and V.shape == (n, n)
    rec = _check_x6(A.T, V, T.T, U, b)
    _mixed_gate(T.T, A.T, b, q, 3, s, rec)
