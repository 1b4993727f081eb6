"""GPU component parity: the sketch generator, the FP64 MFMA GEMM, the
Householder panel and the block SVD, each called through the C-ABI and
compared with an independent CPU computation (the oracle's generator, numpy
products, LAPACK dgeqrf, numpy's SVD).

Tolerances come from the arithmetic: a K-term FP64 dot product is within
gamma_K |a|^T |b| of the exact value (gamma_K ~ K u); Householder QR and
one-sided Jacobi are backward stable, so factors agree to a small multiple of
n u relative to the input's norm when the problem is well conditioned.
"""
import numpy as np
import pytest

import oracle
from oracle.hqr import form_q, hqr

pytestmark = pytest.mark.gpu
U64 = np.finfo(np.float64).eps / 2


def _to_dev(x, gpu):
    import torch
    from paper_2106_13402_amd import colmajor
    return colmajor(torch.as_tensor(np.asfortranarray(x), device=gpu))


def _host(x):
    return x.detach().cpu().numpy()


# ------------------------------------------------------------- generator
@pytest.mark.parametrize("seed,stream,rows,cols", [
    (1, 1, 37, 11), (0, 0, 4, 1), (1, 7, 4096, 128), (2**40 + 3, 2**32 + 5, 1001, 3)])
def test_gaussian_matches_oracle(gpu, seed, stream, rows, cols):
    from paper_2106_13402_amd import gaussian
    g = _host(gaussian(seed, stream, rows, cols, gpu))
    ref = oracle.gaussian(seed, stream, rows, cols)
    # same uniforms bit for bit; log/sqrt/cos/sin may differ by a few ulp
    np.testing.assert_allclose(g, ref, rtol=0, atol=16 * U64 * np.maximum(1.0, np.abs(ref)).max())


@pytest.mark.parametrize("seed,stream,rows,cols", [
    (1, 1, 37, 11), (0, 0, 4, 1), (1, 7, 4096, 128), (2**64 - 1, 2**63 + 5, 1001, 3)])
def test_sketch_uniforms_bit_exact(gpu, seed, stream, rows, cols):
    """The Philox words and their 53-bit uniforms agree with the oracle's bit
    for bit (the Gaussians built from them may differ by a few ulp)."""
    from paper_2106_13402_amd import sketch_uniforms
    u = _host(sketch_uniforms(seed, stream, rows, cols, gpu))
    groups = (rows + 3) // 4
    g = np.arange(groups, dtype=np.uint64)[:, None]
    c = np.arange(cols, dtype=np.uint64)[None, :]
    z = np.zeros((1, 1), dtype=np.uint64)
    w = oracle.philox.philox4x64_10((g, c, z, z), (np.uint64(seed), np.uint64(stream)))
    ref = np.empty((4 * groups, cols))
    for i, (word, open0) in enumerate(zip(w, (True, False, True, False))):
        ref[i::4] = oracle.philox.uniforms_from_words(word, open0)
    np.testing.assert_array_equal(u, ref[:rows])
    assert np.all(u[0::4] > 0.0) and np.all(u[1::4] < 1.0)


# ------------------------------------------------------------------ GEMM
GEMM_CASES = [
    (1, 1, 1), (17, 33, 5), (64, 64, 64), (130, 70, 300), (257, 129, 1000),
    (200, 128, 5000),   # skinny: split-K path
    (3000, 128, 8192),  # sketch-like, split-K, several tiles and a ragged tail
    (1000, 1100, 128),  # rank-b update shape
]


@pytest.mark.parametrize("M,N,K", GEMM_CASES)
@pytest.mark.parametrize("ta,tb", [(False, False), (True, False), (False, True), (True, True)])
def test_dgemm(gpu, M, N, K, ta, tb):
    from paper_2106_13402_amd import dgemm
    rng = np.random.default_rng(M * 7 + N * 3 + K)
    A = rng.standard_normal((K, M) if ta else (M, K))
    B = rng.standard_normal((N, K) if tb else (K, N))
    C0 = rng.standard_normal((M, N))
    alpha, beta = 0.75, -1.25
    Cd = _to_dev(C0, gpu)
    dgemm(_to_dev(A, gpu), _to_dev(B, gpu), transa=ta, transb=tb, alpha=alpha, beta=beta, C_out=Cd)
    opA = A.T if ta else A
    opB = B.T if tb else B
    ref = alpha * (opA @ opB) + beta * C0
    bound = (K + 2) * 2 * U64 * (abs(alpha) * (np.abs(opA) @ np.abs(opB)) + abs(beta) * np.abs(C0))
    err = np.abs(_host(Cd) - ref)
    assert np.all(err <= 4 * bound + 1e-300), float((err / (bound + 1e-300)).max())


def test_dgemm_strided_views(gpu):
    """Operands are sub-blocks of larger matrices (lda > rows), as in T22."""
    import torch
    from paper_2106_13402_amd import colmajor, dgemm
    rng = np.random.default_rng(5)
    big = rng.standard_normal((700, 650))
    Bm = rng.standard_normal((600, 40))
    dbig = _to_dev(big, gpu)
    sub = dbig[50:650, 30:620]  # 600 x 590, lda 700
    Cd = dgemm(sub, _to_dev(Bm, gpu), transa=True)
    ref = big[50:650, 30:620].T @ Bm
    np.testing.assert_allclose(_host(Cd), ref, atol=1e-11 * np.abs(ref).max())
    assert isinstance(sub, torch.Tensor) and sub.stride(0) == 1 and colmajor(sub) is sub


def test_dgemm_k_zero_scales(gpu):
    import torch
    from paper_2106_13402_amd import dgemm
    A = torch.zeros((5, 0), dtype=torch.float64, device=gpu)
    B = torch.zeros((0, 3), dtype=torch.float64, device=gpu)
    C = _to_dev(np.ones((5, 3)), gpu)
    dgemm(A, B, beta=2.0, C_out=C)
    assert np.all(_host(C) == 2.0)


# ---------------------------------------------------------- panel QR
def _larft(W, tau):
    """Forward compact-WY factor from explicit reflectors (Schreiber-Van Loan)."""
    k = tau.size
    T = np.zeros((k, k))
    for i in range(k):
        T[:i, i] = -tau[i] * T[:i, :i] @ (W[:, :i].T @ W[:, i])
        T[i, i] = tau[i]
    return T


# (32768, 256) and (40000, 256) exceed one panel launch: one and two levels
# of the column split.
PANEL_CASES = [(5, 1), (64, 32), (1000, 7), (513, 32), (4096, 128), (16384, 128), (20000, 64),
               (32768, 128), (3000, 256), (32768, 256), (40000, 256)]


@pytest.mark.parametrize("kernel", ["cholqr", "column", "tree"])
@pytest.mark.parametrize("M,k", PANEL_CASES)
def test_householder_panel_matches_lapack(gpu, M, k, kernel):
    print(f"case: panel M={M} k={k} kernel={kernel}", flush=True)
    rng = np.random.default_rng(M + k)
    P = rng.standard_normal((M, k))
    _check_panel_lapack(P, *_panel(P, gpu, kernel))


def _panel(P, gpu, kernel="tree"):
    """rrf_householder_panel with the kernel chosen through the environment:
    "cholqr" (the default: CholeskyQR where it applies, else the column
    kernel), "column" (RRF_PANEL_COLUMN=1) or "tree" (RRF_PANEL_TREE=1).
    A bool picks the tree (True) or the column kernel (False)."""
    import os
    from paper_2106_13402_amd import householder_panel
    if isinstance(kernel, bool):
        kernel = "tree" if kernel else "column"
    env = {"RRF_PANEL_TREE": "1" if kernel == "tree" else "0",
           "RRF_PANEL_COLUMN": "1" if kernel == "column" else "0"}
    old = {key: os.environ.get(key) for key in env}
    os.environ.update(env)
    try:
        return tuple(_host(x) for x in householder_panel(_to_dev(P, gpu)))
    finally:
        for key, v in old.items():
            if v is None:
                del os.environ[key]
            else:
                os.environ[key] = v


def _check_panel_lapack(P, W, R, Tf, tau):
    M, k = P.shape
    qr, tau_ref = hqr(P)
    W_ref = np.tril(qr[:, :k], -1) + np.eye(M, k)
    np.testing.assert_allclose(tau, tau_ref, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(W, W_ref, atol=1e-11)
    np.testing.assert_allclose(R, np.triu(qr[:k, :k]), atol=1e-11 * np.abs(P).max() * np.sqrt(M))
    np.testing.assert_allclose(Tf, _larft(W_ref, tau_ref), atol=1e-10)
    assert np.all(np.tril(R, -1) == 0) and np.all(np.tril(Tf, -1) == 0)
    assert np.all(np.triu(W, 1) == 0) and np.all(np.diag(W) == 1.0)
    Q = np.eye(M, k) - W @ (Tf @ W[:k, :].T)
    np.testing.assert_allclose(Q, form_q(qr, tau_ref, k), atol=1e-11)


# The tree kernel (k <= 64, M <= 65536; wider panels split into halves it
# takes): one leaf, a leaf boundary, ragged last leaves, trees of every
# shape up to the 256-leaf maximum, and the column split above 64.
TREE_CASES = [(64, 64), (256, 17), (257, 1), (257, 64), (511, 2), (512, 63), (513, 64),
              (769, 40), (2049, 64), (16384, 64), (65536, 64), (5000, 65), (3000, 100),
              (65536, 128)]


@pytest.mark.parametrize("M,k", TREE_CASES)
def test_panel_tree_matches_lapack(gpu, M, k):
    print(f"case: tree panel M={M} k={k}", flush=True)
    rng = np.random.default_rng(7 * M + k)
    P = rng.standard_normal((M, k)) * 2.0 ** rng.integers(-3, 4, k)[None, :]
    _check_panel_lapack(P, *_panel(P, gpu))


@pytest.mark.parametrize("M,k", [(3000, 64), (16384, 128), (1000, 33)])
def test_panel_tree_matches_column_kernel(gpu, M, k):
    """Both kernels give the same reflectors (to rounding)."""
    print(f"case: tree vs column panel M={M} k={k}", flush=True)
    P = np.random.default_rng(M - k).standard_normal((M, k))
    a, b = _panel(P, gpu, True), _panel(P, gpu, False)
    for x, y, name in zip(a, b, ("W", "R", "Tf", "tau")):
        np.testing.assert_allclose(x, y, atol=1e-12 * max(1.0, np.abs(y).max()), err_msg=name)


def test_panel_tree_graded(gpu):
    """Columns spanning 14 decades (the sketch of a decaying spectrum): Q is
    orthogonal and Q R = P to rounding, and the well-separated leading
    reflectors match LAPACK's."""
    print("case: tree panel, graded columns", flush=True)
    M, k = 4000, 64
    from synthetic import haar
    P = haar(M, k, seed=5, stream=1) @ np.diag(10.0 ** -np.linspace(0, 14, k)) @ haar(k, k, seed=5, stream=2).T
    W, R, Tf, tau = _panel(P, gpu)
    Q = np.eye(M, k) - W @ (Tf @ W[:k, :].T)
    assert np.linalg.norm(Q.T @ Q - np.eye(k), 2) < 1e-14 * 20
    assert np.linalg.norm(Q @ R - P, 2) < 1e-15 * 20 * np.linalg.norm(P, 2)
    qr, tau_ref = hqr(P)
    np.testing.assert_allclose(np.abs(np.diag(R)), np.abs(np.diag(qr)[:k]), atol=1e-14 * 20)
    np.testing.assert_allclose(tau[:8], tau_ref[:8], atol=1e-9)


@pytest.mark.parametrize("M,k", [(1024, 16), (4096, 128), (16384, 128), (5000, 100), (33000, 128),
                                 (2048, 33), (3000, 97), (1500, 50)])
def test_panel_cholqr_matches_column_kernel(gpu, M, k):
    """CholeskyQR with reconstructed reflectors and the column kernel give the
    same W, R, Tf and tau to rounding on well-conditioned panels (k not a
    multiple of 4 leaves the last 4 x 4 block partly padding)."""
    print(f"case: cholqr vs column panel M={M} k={k}", flush=True)
    P = np.random.default_rng(M + 3 * k).standard_normal((M, k))
    a, b = _panel(P, gpu, "cholqr"), _panel(P, gpu, "column")
    for x, y, name in zip(a, b, ("W", "R", "Tf", "tau")):
        np.testing.assert_allclose(x, y, atol=1e-12 * max(1.0, np.abs(y).max()), err_msg=name)


@pytest.mark.parametrize("decades", [4, 7, 11])
def test_panel_cholqr_conditioning(gpu, decades):
    """Columns whose singular values span 4 to 11 decades (what the sketch of
    a decaying spectrum looks like): CholeskyQR2 keeps orthogonality to
    rounding up to about 8 decades (cond(P) = 1e8, u cond^2 ~ 1); beyond,
    its first Cholesky factorization breaks down and the column kernel
    takes the panel. Either way Q is orthogonal and Q R = P to rounding,
    and the leading, well-determined reflectors match LAPACK's."""
    print(f"case: cholqr panel, {decades} decades", flush=True)
    M, k = 4000, 64
    from synthetic import haar
    P = (haar(M, k, seed=6, stream=1) @ np.diag(10.0 ** -np.linspace(0, decades, k))
         @ haar(k, k, seed=6, stream=2).T)
    W, R, Tf, tau = _panel(P, gpu, "cholqr")
    Q = np.eye(M, k) - W @ (Tf @ W[:k, :].T)
    assert np.linalg.norm(Q.T @ Q - np.eye(k), 2) < 1e-14 * 20
    assert np.linalg.norm(Q @ R - P, 2) < 1e-15 * 20 * np.linalg.norm(P, 2)
    qr, tau_ref = hqr(P)
    np.testing.assert_allclose(np.abs(np.diag(R)), np.abs(np.diag(qr)[:k]),
                               atol=1e-14 * 20 * np.abs(P).max())
    np.testing.assert_allclose(tau[:8], tau_ref[:8], atol=1e-9)


@pytest.mark.parametrize("case", ["zero", "dependent", "graded14", "nan_free_zero_panel"])
def test_panel_cholqr_falls_back(gpu, case):
    """Ill-conditioned or rank-deficient panels raise the device flag in a
    Cholesky pass and the column kernel factors the untouched panel: the
    result is bitwise the column kernel's."""
    print(f"case: cholqr fallback {case}", flush=True)
    rng = np.random.default_rng(11)
    M, k = 2000, 32
    P = rng.standard_normal((M, k))
    if case == "zero":
        P[:, 7] = 0.0
    elif case == "dependent":
        P[:, 20] = P[:, 3] * 3.0 - P[:, 9]
    elif case == "graded14":
        from synthetic import haar
        P = (haar(M, k, seed=8, stream=1) @ np.diag(10.0 ** -np.linspace(0, 14, k))
             @ haar(k, k, seed=8, stream=2).T)
    else:
        P[:] = 0.0
    a, b = _panel(P, gpu, "cholqr"), _panel(P, gpu, "column")
    for x, y, name in zip(a, b, ("W", "R", "Tf", "tau")):
        assert np.array_equal(x, y), name


def test_panel_cholqr_triangular_input(gpu):
    """A panel that is already upper triangular ([R0; 0]): every sub-column
    is exactly zero, where dlarfg takes H = I; the reconstruction returns the
    reflection tau = 2, v = e_j with row j of R negated instead (the same
    convention as the tree kernel). Q R = P and Q is orthogonal."""
    print("case: cholqr panel, triangular input", flush=True)
    M, k = 2048, 32
    rng = np.random.default_rng(12)
    P = np.zeros((M, k))
    P[:k] = np.triu(rng.standard_normal((k, k))) + 4.0 * np.eye(k)
    W, R, Tf, tau = _panel(P, gpu, "cholqr")
    Q = np.eye(M, k) - W @ (Tf @ W[:k, :].T)
    assert np.linalg.norm(Q.T @ Q - np.eye(k), 2) < 1e-14 * 20
    np.testing.assert_allclose(Q @ R, P, atol=1e-13 * np.abs(P).max())
    np.testing.assert_allclose(np.abs(np.diag(R)), np.abs(np.diag(P[:k])), rtol=1e-13)
    assert np.all(np.abs(W[k:]) < 1e-13)


@pytest.mark.parametrize("tree", [False, True])
def test_householder_panel_zero_and_rank_deficient(gpu, tree):
    """A zero sub-column, a zero column and a dependent column. dlarfg leaves
    a reflector whose sub-column is exactly zero as H = I (tau = 0), and so
    does the column kernel. The tree kernel recovers its reflectors from the
    Q of a tree of QRs: a column that is exactly e_j comes back as the
    reflection I - 2 e_j e_j^T (tau = 2) with row j of R negated, and past
    the first rank drop (the zero column 2) Q's next column is any unit
    vector orthogonal to the earlier ones, so the reflectors from there on
    are a different, equally exact, choice. Both give P = Q R with Q
    orthogonal; LAPACK's reflectors are matched where P determines them."""
    rng = np.random.default_rng(1)
    P = rng.standard_normal((300, 8))
    P[:, 2] = 0.0                  # zero column
    P[:, 5] = P[:, 1] * 3.0        # dependent column
    P[1:, 0] = 0.0                 # zero sub-column below the diagonal
    W, R, Tf, tau = _panel(P, gpu, tree)
    qr, tau_ref = hqr(P)
    assert tau[0] == (2.0 if tree else 0.0) and np.all(W[1:, 0] == 0.0)
    assert abs(R[0, 0]) == abs(P[0, 0])
    np.testing.assert_allclose(tau[1], tau_ref[1], atol=1e-12)
    np.testing.assert_allclose(W[:, 1], np.tril(qr, -1)[:, 1] + np.eye(300, 8)[:, 1], atol=1e-12)
    np.testing.assert_allclose(abs(R[1, 1]), abs(qr[1, 1]), rtol=1e-13)
    amax = np.abs(P).max()
    assert np.abs(R[:3, 2]).max() < 1e-13 * amax * 20   # R(:, 2) = Q^T 0
    assert abs(R[5, 5]) < 1e-13 * amax * 20             # column 5 in span(Q(:, :2))
    if not tree:
        # columns 0..4 are determined by P in the dlarfg convention; column 5
        # lies in the span of the earlier ones, so its reflector (and every
        # later one) is fixed by rounding noise alone
        assert tau[2] == 0.0
        np.testing.assert_allclose(tau[:5], tau_ref[:5], atol=1e-12)
        np.testing.assert_allclose(np.abs(np.diag(R))[:5], np.abs(np.diag(qr))[:5], atol=1e-12 * 20)
    Q = np.eye(300) - W @ Tf @ W.T
    assert np.linalg.norm(Q.T @ Q - np.eye(300), 2) < 1e-13
    np.testing.assert_allclose(Q[:, :8] @ R, P, atol=1e-12 * 20)


def test_householder_panel_inplace(gpu):
    from paper_2106_13402_amd import householder_panel
    rng = np.random.default_rng(2)
    P = rng.standard_normal((2000, 16))
    dP = _to_dev(P, gpu)
    W, R, Tf, tau = householder_panel(dP, inplace=True)
    qr, tau_ref = hqr(P)
    np.testing.assert_allclose(_host(dP), np.tril(qr, -1) + np.eye(2000, 16), atol=1e-11)


# ------------------------------------------------------------- block SVD
@pytest.mark.parametrize("k", [1, 2, 7, 16, 32, 33, 63, 64, 65, 100, 128, 256])
def test_block_svd(gpu, k):
    from paper_2106_13402_amd import block_svd
    rng = np.random.default_rng(k)
    B = np.triu(rng.standard_normal((k, k)))  # shape of the panel's R
    Us, d, Vs = (_host(x) for x in block_svd(_to_dev(B, gpu)))
    Ur, dr, Vr = oracle.small_svd(B)
    nB = np.linalg.norm(B, 2)
    np.testing.assert_allclose(d, dr, atol=8 * k * U64 * nB)
    assert np.all(np.diff(d) <= 0)
    # Us and Vs come out of ~(sweeps * k) plane rotations per column, each
    # orthogonal to within a few eps: their departure from orthogonality is
    # bounded by a small multiple of k eps (the scale LAPACK's own SVD tests
    # measure it in), with a 1e-13 floor for the small blocks.
    orth = max(1e-13, 4 * k * np.finfo(float).eps)
    assert np.linalg.norm(Us.T @ Us - np.eye(k), 2) < orth
    assert np.linalg.norm(Vs.T @ Vs - np.eye(k), 2) < orth
    assert np.linalg.norm(Us @ np.diag(d) @ Vs.T - B, 2) < 8 * k * U64 * nB
    for j in range(k):
        assert Vs[np.argmax(np.abs(Vs[:, j])), j] > 0
    # singular vectors agree with the oracle where the gaps are large
    gaps = np.minimum(np.abs(np.diff(np.r_[np.inf, dr])), np.abs(np.diff(np.r_[dr, -np.inf])))
    ok = gaps > 1e-6 * nB
    np.testing.assert_allclose(Vs[:, ok], Vr[:, ok], atol=1e-8)


def test_block_svd_graded_and_degenerate(gpu):
    from paper_2106_13402_amd import block_svd
    from synthetic import haar
    k = 32
    s = 10.0 ** -np.arange(k, dtype=float) * 0.5  # 1 down to 1e-31: relative accuracy matters
    B = haar(k, k, seed=3, stream=1) @ np.diag(s) @ haar(k, k, seed=3, stream=2).T
    _, d, _ = (_host(x) for x in block_svd(_to_dev(np.triu(np.linalg.qr(B)[1]), gpu)))
    # forming B rounds at eps ||B||, so only values well above that are fixed
    np.testing.assert_allclose(d[:6], s[:6], rtol=1e-9)
    assert np.all(d[6:] < 1e-4)
    # zero block: d = 0, U and V orthogonal
    Us, d, Vs = (_host(x) for x in block_svd(_to_dev(np.zeros((16, 16)), gpu)))
    assert np.all(d == 0)
    assert np.linalg.norm(Us.T @ Us - np.eye(16)) < 1e-14
    assert np.linalg.norm(Vs.T @ Vs - np.eye(16)) < 1e-14
    # rank 3
    rng = np.random.default_rng(4)
    B = rng.standard_normal((24, 3)) @ rng.standard_normal((3, 24))
    Us, d, Vs = (_host(x) for x in block_svd(_to_dev(B, gpu)))
    assert np.all(d[3:] < 1e-13 * d[0])
    assert np.linalg.norm(Us.T @ Us - np.eye(24), 2) < 1e-13


# ------------------------------------------------- bfloat16 sketch building blocks
def _bf16_bits_to_f64(t16):
    u = t16.detach().cpu().numpy().astype(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


def _f64_to_bf16_bits(x):
    """Bit patterns of bfloat16-exact binary64 values."""
    return (np.asarray(x, np.float64).astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)


@pytest.mark.parametrize("aligned", [False, True])
@pytest.mark.parametrize("scaled", [False, True])
def test_to_bf16_bit_exact(gpu, scaled, aligned):
    """Strided (odd leading dimension: element loads) and 16-byte aligned
    (pairs of loads, a ragged last group of four rows) inputs."""
    from oracle.bf16 import bf16_round, pow2_scale
    from paper_2106_13402_amd import to_bf16
    rng = np.random.default_rng(11)
    M, N = (1002, 300) if aligned else (1000, 300)
    X = rng.standard_normal((M, N)) * 2.0 ** rng.integers(-60, 40, (M, N))
    X[0, :5] = [0.0, -0.0, 3e-41, -2.2e-39, 1.0 + 2.0 ** -8 + 2.0 ** -30]  # zeros, underflow, direct rounding
    X[1:17, 7] = (np.arange(256, 272) + 0.5) * 2.0 ** -9                     # exact ties
    r0, ldx = (0, M + 6) if aligned else (4, M + 9)
    big = np.zeros((ldx, N + 3))
    big[r0:r0 + M, 2:2 + N] = X
    dX = _to_dev(big, gpu)[r0:r0 + M, 2:2 + N]                              # strided view
    out, outT = to_bf16(dX, scaled=scaled, transpose=True)
    s = pow2_scale(X) if scaled else 1.0
    want = _f64_to_bf16_bits(bf16_round(X * s))
    got = out.detach().cpu().numpy().astype(np.uint16)
    np.testing.assert_array_equal(got[:M], want)
    assert np.all(got[M:] == 0)                                              # zero padding
    gotT = outT.detach().cpu().numpy().astype(np.uint16)
    np.testing.assert_array_equal(gotT[:N], want.T)
    assert np.all(gotT[N:] == 0)


BF16_GEMM_CASES = [(1, 1, 1), (130, 7, 1000), (300, 200, 77), (1000, 128, 16384),
                   (4097, 128, 3000), (128, 128, 0)]


@pytest.mark.parametrize("M,N,K", BF16_GEMM_CASES)
def test_gemm_bf16_tn_exact_products(gpu, M, N, K):
    from oracle.bf16 import bf16_round, fp32_gemm_bound, gemm_tn_reference, pow2_scale
    from paper_2106_13402_amd import gemm_bf16_tn, to_bf16
    rng = np.random.default_rng(M + N + K)
    A = rng.standard_normal((max(K, 1), M))[:K]
    B = rng.standard_normal((max(K, 1), N))[:K]
    if K == 0:
        import torch
        A16 = torch.zeros((M, 8), dtype=torch.int16, device=gpu).t()  # 8 x M, column-major
        B16 = torch.zeros((N, 8), dtype=torch.int16, device=gpu).t()
    else:
        A16, _ = to_bf16(_to_dev(A, gpu))
        B16, _ = to_bf16(_to_dev(B, gpu))
    Ar, Br = bf16_round(A), bf16_round(B)
    exact = gemm_tn_reference(Ar, Br)
    bound = fp32_gemm_bound(Ar, Br)
    C = _host(gemm_bf16_tn(A16, K, B16, out="f64"))
    assert np.all(np.abs(C - exact) <= bound), np.max(np.abs(C - exact) - bound)
    # column-rescaled bfloat16 output: each column's power of two puts its
    # max in [0.5, 1); values within one bfloat16 unit of the exact scaled ones
    C16 = gemm_bf16_tn(A16, K, B16, out="bf16")
    dec = _bf16_bits_to_f64(C16)
    assert np.all(dec[M:] == 0)
    for j in range(N):
        s = pow2_scale(exact[:, j])
        col = dec[:M, j]
        if K == 0:
            assert np.all(col == 0)
            continue
        ref = exact[:, j] * s
        assert 0.5 <= np.max(np.abs(col)) <= 1.0
        np.testing.assert_array_less(np.abs(col - ref), 2.0 ** -7 * np.abs(ref) + bound[:, j] * s + 1e-300)


def test_trace_records_only_the_selected_class(gpu):
    """rrf_trace_enable_class times one kernel class and leaves the other
    launches uninstrumented; rrf_trace_enable(1) times them all."""
    from paper_2106_13402_amd import dgemm, trace_enable, trace_enable_class, trace_read
    print("case: trace class filter", flush=True)
    rng = np.random.default_rng(3)
    A = _to_dev(rng.standard_normal((256, 256)), gpu)
    B = _to_dev(rng.standard_normal((256, 256)), gpu)
    try:
        trace_enable_class("dgemm_mfma_128x128_TN")
        dgemm(A, B, transa=True)
        dgemm(A, B)
        names = {e["name"]: e for e in trace_read()}
        assert set(names) == {"dgemm_mfma_128x128_TN"} and names["dgemm_mfma_128x128_TN"]["launches"] == 1
        assert names["dgemm_mfma_128x128_TN"]["ms"] > 0
        trace_enable(True)
        dgemm(A, B, transa=True)
        dgemm(A, B)
        assert {"dgemm_mfma_128x128_TN", "dgemm_mfma_128x128_NN"} <= {e["name"] for e in trace_read()}
    finally:
        trace_enable(False)
