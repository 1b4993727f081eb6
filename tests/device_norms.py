"""Spectral norms of large device matrices for the GPU tests (torch, FP64).

Golub-Kahan-Lanczos bidiagonalisation with full (twice repeated)
reorthogonalisation, the bases kept as columns of preallocated matrices so
each step is a handful of device products. It runs on any torch device;
``tests/test_norm_estimators.py`` checks it on the CPU against exact norms.
"""
from __future__ import annotations


def gkl_norm(apply, apply_t, n: int, device, steps: int = 200, seed: int = 0) -> float:
    """Largest singular value of x -> apply(x) (n columns; apply_t is the
    transpose). Grows towards ||.||_2 from below, exact once the Krylov
    space is exhausted."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    v = torch.randn(n, 1, dtype=torch.float64, generator=g).to(device)
    v /= torch.linalg.vector_norm(v)
    k_max = min(steps, n)
    Vb = torch.zeros(n, k_max + 1, dtype=torch.float64, device=device)
    Vb[:, :1] = v
    u = apply(v)
    m = u.shape[0]
    Ub = torch.zeros(m, k_max, dtype=torch.float64, device=device)
    alpha, beta = [], []
    for j in range(k_max):
        for _ in range(2):
            u = u - Ub[:, :j] @ (Ub[:, :j].T @ u)
        a = float(torch.linalg.vector_norm(u))
        if a == 0.0:
            break
        u = u / a
        Ub[:, j:j + 1] = u
        alpha.append(a)
        v = apply_t(u) - a * Vb[:, j:j + 1]
        for _ in range(2):
            v = v - Vb[:, :j + 1] @ (Vb[:, :j + 1].T @ v)
        bt = float(torch.linalg.vector_norm(v))
        if bt <= 1e-300 or j + 1 >= n:
            break
        v = v / bt
        Vb[:, j + 1:j + 2] = v
        beta.append(bt)
        u = apply(v) - bt * u
    k = len(alpha)
    if k == 0:
        return 0.0
    B = torch.diag(torch.tensor(alpha, dtype=torch.float64))
    for i in range(min(len(beta), k - 1)):
        B[i, i + 1] = beta[i]
    return float(torch.linalg.matrix_norm(B, 2))


def spec(X, steps: int = 200) -> float:
    """||X||_2 of a device matrix."""
    if X.numel() == 0:
        return 0.0
    return gkl_norm(lambda x: X @ x, lambda y: X.T @ y, X.shape[1], X.device, steps)


def orth_error(Q, steps: int = 200) -> float:
    """||Q^T Q - I||_2 of a device matrix."""
    E = Q.T @ Q
    E.diagonal().sub_(1.0)
    return gkl_norm(lambda x: E @ x, lambda y: E @ y, E.shape[1], E.device, steps)


def recon_error(A, U, T, V, norm_a: float, steps: int = 200) -> float:
    """||A - U T V^T||_2 / norm_a without forming the product."""
    r = gkl_norm(lambda x: A @ x - U @ (T @ (V.T @ x)),
                 lambda y: A.T @ y - V @ (T.T @ (U.T @ y)), A.shape[1], A.device, steps)
    return r / norm_a if norm_a > 0 else r
