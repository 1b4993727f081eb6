"""GPU checks of the split-bfloat16 three-pass product (rrf_gemm_x3) and of
randUTV with it in every update of T, U and V (RRF_PREC_BF16_X3).

Kernel: the GPU result against the oracle's definition of the product
(oracle.bf16.gemm_x3: the same split, exact terms summed in FP64); the two
differ only by the binary32 summation of the 3K exact terms
(fp32_x3_bound) and the FP64 rounding of alpha v + beta C. Closed-form
cases pin the split itself (the binary32 rounding comes before the
bfloat16 one) and the three passes (lo_a lo_b is dropped).

Factorization: the x3 updates carry about 2^-16 relative error per product,
so U, V and A = U T V^T hold to about 1e-5 instead of binary64 level; the
gate on e_k is the mixed gate of the bfloat16 sketch (e_k within
max(1.5 sigma_{k+1}, 1.1 x the FP64 oracle envelope) wherever sigma_{k+1}
is above 100 x the reconstruction error).
"""
import numpy as np
import pytest

from oracle import metrics as M
from oracle.bf16 import fp32_x3_bound, gemm_x3 as gemm_x3_ref
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
def test_gemm_x3_matches_oracle(gpu, M, N, K, ta, tb):
    from paper_2106_13402_amd import gemm_x3
    print(f"case: gemm_x3 M={M} N={N} K={K} ta={ta} tb={tb}", flush=True)
    rng = np.random.default_rng(M * 7 + N * 3 + K + 2 * ta + tb)
    A = rng.standard_normal((K, M) if ta else (M, K)) * 2.0 ** rng.integers(-6, 6, (K, M) if ta else (M, K))
    B = rng.standard_normal((N, K) if tb else (K, N))
    C0 = rng.standard_normal((M, N))
    alpha, beta = -0.75, 1.25
    Cd = _to_dev(C0, gpu)
    gemm_x3(_to_dev(A, gpu), _to_dev(B, gpu), transa=ta, transb=tb, alpha=alpha, beta=beta,
            C_out=Cd)
    opA = A.T if ta else A
    opB = B.T if tb else B
    ref = alpha * gemm_x3_ref(opA, opB) + beta * C0
    bound = abs(alpha) * fp32_x3_bound(opA, opB) + 4 * U64 * (np.abs(ref) + abs(beta) * np.abs(C0))
    err = np.abs(_host(Cd) - ref)
    assert np.all(err <= bound), float((err / bound).max())


def test_gemm_x3_closed_forms(gpu):
    """Entries whose split and product are exact in binary32: the result is
    known to the last bit."""
    from paper_2106_13402_amd import gemm_x3
    print("case: gemm_x3 closed forms", flush=True)
    e = 2.0 ** -10
    # hi = 1, lo = 2^-10: three passes give 1 + 2^-9, missing lo lo = 2^-20
    a = np.array([[1.0 + e]])
    c = _host(gemm_x3(_to_dev(a, gpu), _to_dev(a, gpu)))
    assert c[0, 0] == 1.0 + 2.0 ** -9
    # a = 1 + 2^-8 + 2^-30 rounds to the binary32 tie 1 + 2^-8, so hi = 1 and
    # lo = 2^-8; with b = 1 + 2^-12 (hi = 1, lo = 2^-12) the product is
    # 1 + 2^-8 + 2^-12. Rounding a to bfloat16 directly from binary64 would
    # give hi = 1 + 2^-7, lo = -2^-8 and an extra 2^-19.
    a = np.array([[1.0 + 2.0 ** -8 + 2.0 ** -30]])
    b = np.array([[1.0 + 2.0 ** -12]])
    c = _host(gemm_x3(_to_dev(a, gpu), _to_dev(b, gpu)))
    assert c[0, 0] == 1.0 + 2.0 ** -8 + 2.0 ** -12


def test_gemm_x3_strided_and_unaligned(gpu):
    """Operands as sub-blocks with odd leading dimensions (8-byte loads)."""
    from paper_2106_13402_amd import gemm_x3
    print("case: gemm_x3 strided", flush=True)
    rng = np.random.default_rng(5)
    big = rng.standard_normal((701, 650))
    Bm = rng.standard_normal((601, 40))
    dbig = _to_dev(big, gpu)
    sub = dbig[51:651, 31:621]     # 600 x 590, lda 701, odd start
    Bs = _to_dev(Bm, gpu)[1:601]  # 600 x 40, ldb 601
    Cd = gemm_x3(sub, Bs, transa=True)
    opA = big[51:651, 31:621].T
    ref = gemm_x3_ref(opA, Bm[1:601])
    err = np.abs(_host(Cd) - ref)
    assert np.all(err <= fp32_x3_bound(opA, Bm[1:601]) + 4 * U64 * np.abs(ref))


# ------------------------------------------------------------ factorization
def _factor_x3(A, b, q, seed, gpu):
    from paper_2106_13402_amd import randutv
    U, T, V = (_host(x) for x in randutv(_to_dev(A, gpu), b, q, seed, precision="bf16_x3"))
    return U, T, V


def _check_x3(A, U, T, V, b, tol):
    m, n = A.shape
    eo = max(M.orth_error(U), M.orth_error(V))
    rec = M.recon_error(A, U, T, V)
    print(f"  x3: ||U^T U - I||, ||V^T V - I|| <= {eo:.2e}, ||A - U T V^T|| / ||A|| = {rec:.2e}",
          flush=True)
    assert eo <= tol and rec <= tol
    assert np.all(np.tril(T, -1) == 0.0)
    _check_blocks(T, b)
    return rec


@pytest.mark.parametrize("q", [1, 2])
def test_randutv_x3_headline_spectrum(gpu, q):
    """2048 x 2048, s_j = exp(-j/800), b = 128."""
    n, b = 2048, 128
    s = spectrum("exp", n, scale=800.0)
    A = spectral_matrix(n, n, s, seed=0)
    print(f"case: randutv x3 exp(-j/800) n={n} q={q}", flush=True)
    U, T, V = _factor_x3(A, b, q, 1, gpu)
    rec = _check_x3(A, U, T, V, b, 1e-4)
    _mixed_gate(T, A, b, q, 1, s, rec)


@pytest.mark.parametrize("m,n,b,q", [(1000, 700, 64, 1), (600, 600, 96, 2), (513, 300, 100, 2),
                                     (64, 64, 1, 1)])
def test_randutv_x3_shapes(gpu, m, n, b, q):
    s = spectrum("exp", n, scale=n / 2.0)
    A = spectral_matrix(m, n, s, seed=1)
    print(f"case: randutv x3 m={m} n={n} b={b} q={q}", flush=True)
    U, T, V = _factor_x3(A, b, q, 3, gpu)
    rec = _check_x3(A, U, T, V, b, 1e-4)
    _mixed_gate(T, A, b, q, 3, s, rec, factor=1.5 if b == 100 else 1.1)


def test_randutv_x3_power_of_two_invariance(gpu):
    """T is formed from 2^-e A with max|2^-e A| in [0.5, 1): inputs that
    differ by a power of two give the same U and V and T scaled exactly,
    also where A itself is beyond the binary32 range."""
    n, b = 300, 32
    s = spectrum("geometric", n, decades=6.0)
    A = spectral_matrix(n, n, s, seed=2)
    print("case: randutv x3 power-of-two invariance", flush=True)
    U0, T0, V0 = _factor_x3(A, b, 1, 5, gpu)
    for p in (200, -200):
        U1, T1, V1 = _factor_x3(A * 2.0 ** p, b, 1, 5, gpu)
        np.testing.assert_array_equal(U1, U0)
        np.testing.assert_array_equal(V1, V0)
        np.testing.assert_array_equal(T1, T0 * 2.0 ** p)
    _check_x3(A, U0, T0, V0, b, 1e-4)


def test_randutv_x3_differs_from_bf16_sketch(gpu):
    """The x3 updates are in use: the result differs from the bfloat16
    sketch mode (binary64 updates) by far more than binary64 rounding, and
    repeated runs are bitwise identical."""
    from paper_2106_13402_amd import randutv
    n, b = 512, 64
    A = spectral_matrix(n, n, spectrum("exp", n, scale=200.0), seed=4)
    print("case: randutv x3 vs bf16 sketch", flush=True)
    _, T1, _ = (_host(x) for x in randutv(_to_dev(A, gpu), b, 1, 7, precision="bf16_sketch"))
    _, T3, _ = _factor_x3(A, b, 1, 7, gpu)
    _, T3b, _ = _factor_x3(A, b, 1, 7, gpu)
    np.testing.assert_array_equal(T3, T3b)
    assert np.abs(T3 - T1).max() > 1e-9 * np.abs(A).max()


def test_randutv_x3_wide(gpu):
    """m < n in the x3 mode: the transpose's factorization (U and V
    exchanged, T lower trapezoidal) to the same x3 accuracy and e_k gate as a
    tall input."""
    m, n, b, q = 300, 520, 64, 1
    s = spectrum("exp", m, scale=m / 2.0)
    A = spectral_matrix(n, m, s, seed=2).T.copy(order="F")
    print(f"case: randutv x3 wide m={m} n={n} b={b} q={q}", flush=True)
    U, T, V = _factor_x3(A, b, q, 3, gpu)
    assert U.shape == (m, m) and T.shape == (m, n) and V.shape == (n, n)
    rec = _check_x3(A.T, V, T.T, U, b, 1e-4)
    _mixed_gate(T.T, A.T, b, q, 3, s, rec)
