"""GPU checks of rrf_randutv_batched with the bfloat16 sketch (Alg. 3 with
each step's power products Y = (T22^T T22)^q T22^T G formed from bfloat16
copies of T22 and G, FP32 accumulation, everything else FP64).

The mixed sketch perturbs each step's sampled subspace at the bfloat16
level, so matrix j follows another valid random trajectory than the FP64
oracle with seed + j; the gate is therefore the one of the single-matrix
mixed tests: per matrix, U and V orthogonal and A = U T V^T to FP64
accuracy, T upper trapezoidal with diagonal, descending b x b blocks, and
e_k = ||T(k:, k:)||_2 <= max(1.5 sigma_{k+1}, 1.1 x the largest e_k over
FP64 oracle runs with 12 sketch seeds) wherever sigma_{k+1} is resolved.
"""
import numpy as np
import pytest

from oracle import metrics as M
from synthetic import batch_gaussians, batch_shapes, gaussian_matrix, spectral_matrix, spectrum

from test_gpu_factorizations import (_check_blocks, _check_factorization, _host, _mixed_gate,
                                     _to_dev)

pytestmark = pytest.mark.gpu

SHAPES = [(40, 30), (64, 64), (33, 17), (100, 64), (9, 4), (70, 70), (1, 1), (5, 1), (130, 129),
          (250, 90)]


def _run(As_host, b, q, seed, gpu, **kw):
    from paper_2106_13402_amd import randutv_batched
    As = [_to_dev(A, gpu) for A in As_host]
    Us, Ts, Vs = randutv_batched(As, b, q, seed, precision="bf16_sketch", **kw)
    return ([_host(U) for U in Us] if Us is not None else None, [_host(T) for T in Ts],
            [_host(V) for V in Vs] if Vs is not None else None)


def _auto_b(n):
    from paper_2106_13402_amd import batched_block
    return batched_block(n, n)


def _gate_all(As, spectra, Us, Ts, Vs, b, q, seed):
    for j, A in enumerate(As):
        bj = b if b > 0 else _auto_b(A.shape[1])
        print(f"  matrix {j}: {A.shape[0]}x{A.shape[1]} b={bj}", flush=True)
        _check_factorization(A, Us[j], Ts[j], Vs[j])
        _check_blocks(Ts[j], bj)
        _mixed_gate(Ts[j], A, bj, q, seed + j, spectra[j], M.recon_error(A, Us[j], Ts[j], Vs[j]))


@pytest.mark.parametrize("b", [8, 16, 32])
@pytest.mark.parametrize("q", [1, 2])
def test_batched_bf16_ragged(gpu, b, q):
    """Ragged batch with decaying spectra (s_j = exp(-2j/n)): square, tall,
    n < b, n = 1 and a tail block of every width; bfloat16 copies whose
    leading dimension is padded to 8 on both operands."""
    print(f"case: batched bf16 ragged b={b} q={q}", flush=True)
    spectra = [spectrum("exp", n, scale=n / 2.0) for _, n in SHAPES]
    As = [spectral_matrix(m, n, s, seed=700 + j) for j, ((m, n), s) in enumerate(zip(SHAPES, spectra))]
    Us, Ts, Vs = _run(As, b, q, 13, gpu)
    _gate_all(As, spectra, Us, Ts, Vs, b, q, 13)


def test_batched_bf16_graded(gpu):
    """Graded spectra (10 decades across n), automatic b, split-free panels."""
    print("case: batched bf16 graded spectra", flush=True)
    shapes = [(200, 160), (256, 256), (300, 150), (400, 300)]
    spectra = [spectrum("geometric", n, decades=10.0) for _, n in shapes]
    As = [spectral_matrix(m, n, s, seed=800 + j) for j, ((m, n), s) in enumerate(zip(shapes, spectra))]
    Us, Ts, Vs = _run(As, 0, 1, 23, gpu)
    _gate_all(As, spectra, Us, Ts, Vs, 0, 1, 23)


def test_batched_bf16_differs_from_fp64(gpu):
    """The mixed mode runs its own sketch: its diagonal differs from the FP64
    batch by far more than FP64 rounding, while both factor A exactly."""
    from paper_2106_13402_amd import randutv_batched
    print("case: batched bf16 vs fp64", flush=True)
    As = [gaussian_matrix(m, n, seed=900 + j) for j, (m, n) in enumerate([(150, 120), (96, 96)])]
    dev = [_to_dev(A, gpu) for A in As]
    _, T64, _ = randutv_batched(dev, 16, 1, 31)
    _, T16, _ = randutv_batched(dev, 16, 1, 31, precision="bf16_sketch")
    for j, A in enumerate(As):
        d = np.abs(np.abs(np.diag(_host(T64[j]))) - np.abs(np.diag(_host(T16[j]))))
        assert d.max() > 1e-6 * M.spec(A), d.max()


def test_batched_bf16_edges(gpu):
    """Zero matrix (max|T22| = 0: scale 1, zero sketch), identity, no U / no V,
    and a second call on the same workspace giving the same result."""
    import torch
    from paper_2106_13402_amd import colmajor, randutv_batched
    print("case: batched bf16 edges", flush=True)
    A0 = gaussian_matrix(80, 60, seed=5)
    Z = torch.zeros((50, 40), dtype=torch.float64, device=gpu).t().contiguous().t()
    I = colmajor(torch.eye(64, dtype=torch.float64, device=gpu))
    Us, Ts, Vs = randutv_batched([_to_dev(A0, gpu), Z, I], 16, 1, 7, want_u=False,
                                 precision="bf16_sketch")
    assert Us is None
    assert np.all(_host(Ts[1]) == 0.0) and M.orth_error(_host(Vs[1])) < 1e-13
    np.testing.assert_allclose(_host(Ts[2]), np.eye(64), atol=1e-13)
    _, Ts2, _ = randutv_batched([_to_dev(A0, gpu), Z, I], 16, 1, 7, want_u=False, want_v=False,
                                precision="bf16_sketch")
    np.testing.assert_allclose(_host(Ts2[0]), _host(Ts[0]), rtol=0, atol=0)  # deterministic


def test_batched_bf16_full_size(gpu):
    """4096 matrices, n ~ U[64, 512], m ~ U[n, 2n], q = 1, automatic b: every
    matrix checked on the GPU (Frobenius-norm bounds), six against the gate."""
    import torch
    from paper_2106_13402_amd import randutv_batched
    shapes = batch_shapes(4096, seed=0)
    print(f"case: batched bf16 full size, {len(shapes)} matrices", flush=True)
    As = batch_gaussians(shapes, seed=0, device=gpu)
    Us, Ts, Vs = randutv_batched(As, 0, 1, 1000, precision="bf16_sketch")
    torch.cuda.synchronize()
    print("  factored", flush=True)
    worst_o, worst_r = 0.0, 0.0
    for j, (m, n) in enumerate(shapes):
        U, T, V, A = Us[j], Ts[j], Vs[j], As[j]
        eo = max(float(torch.linalg.norm(U.t() @ U - torch.eye(m, dtype=U.dtype, device=gpu))),
                 float(torch.linalg.norm(V.t() @ V - torch.eye(n, dtype=V.dtype, device=gpu))))
        er = float(torch.linalg.norm(A - U @ T @ V.t()) / torch.linalg.norm(A))
        worst_o, worst_r = max(worst_o, eo), max(worst_r, er)
        if n > 1:
            assert float(torch.tril(T, -1).abs().max()) == 0.0
    print(f"  worst ||U^T U - I||_F, ||V^T V - I||_F = {worst_o:.2e}, "
          f"||A - U T V^T||_F / ||A||_F = {worst_r:.2e}", flush=True)
    assert worst_o <= 1e-12 and worst_r <= 1e-13
    rng = np.random.default_rng(2)
    small = [j for j, (m, n) in enumerate(shapes) if n <= 160]
    for j in list(rng.choice(small, size=6, replace=False)):
        A = _host(As[j]).copy(order="F")
        bj = _auto_b(A.shape[1])
        T, U, V = _host(Ts[j]), _host(Us[j]), _host(Vs[j])
        _check_blocks(T, bj)
        s = np.linalg.svd(A, compute_uv=False)
        _mixed_gate(T, A, bj, 1, 1000 + int(j), s, M.recon_error(A, U, T, V))
