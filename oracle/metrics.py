"""Oracle-side accuracy measures for a UTV factorization (numpy, FP64).

TEST INFRASTRUCTURE: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import anything under ``oracle/``.

* ``e_k^T = ||T(k+1:m, k+1:n)||`` -- the low-rank error identity of Sec. 4.1
  (the error of the rank-k truncation equals the norm of the trailing block);
* ``e_k^A = ||A - U(:,1:k) T(1:k,:) V^T||`` -- the definition used in the
  numerical experiments (Sec. 5.2);
* the Frobenius recurrence ``e_i^2 = e_{i-1}^2 - ||T(I2, J2∪J3)||_F^2``
  (Sec. 4.1, the early-termination discussion).

The spectral norm (the paper's default norm) is used unless stated.
"""
from __future__ import annotations

import numpy as np


def spec(X: np.ndarray) -> float:
    if X.size == 0:
        return 0.0
    return float(np.linalg.norm(X, 2))


def orth_error(Q: np.ndarray) -> float:
    """||Q^T Q - I||_2."""
    k = Q.shape[1]
    return spec(Q.T @ Q - np.eye(k))


def recon_error(A: np.ndarray, U: np.ndarray, T: np.ndarray, V: np.ndarray) -> float:
    """||A - U T V^T||_2 / ||A||_2 (0 for the zero matrix)."""
    nA = spec(A)
    r = spec(A - U @ T @ V.T)
    return r / nA if nA > 0 else r


def trailing_norms(T: np.ndarray, ks) -> np.ndarray:
    """e_k^T for each k in ``ks`` (k = 0 gives ||T||)."""
    return np.array([spec(T[k:, k:]) for k in ks])


def truncation_errors(A, U, T, V, ks) -> np.ndarray:
    """e_k^A for each k in ``ks``."""
    out = []
    for k in ks:
        Ak = U[:, :k] @ T[:k, :] @ V.T
        out.append(spec(A - Ak))
    return np.array(out)


def strictly_lower_max(T: np.ndarray) -> float:
    return float(np.max(np.abs(np.tril(T, -1)))) if T.size else 0.0


def lanczos_norm(apply, apply_t, n: int, steps: int = 200, seed: int = 0) -> float:
    """Largest singular value of the operator x -> apply(x) (n columns, with
    its transpose apply_t), by Golub-Kahan-Lanczos bidiagonalisation with
    full (twice repeated) reorthogonalisation of both Krylov bases, started
    from a seeded Gaussian vector. The estimate grows towards ||.||_2 from
    below and is exact once the Krylov space is exhausted (steps >= n). Used
    for spectral norms of matrices too large for a full SVD on the host."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(n)
    v /= np.linalg.norm(v)
    vs, us, alpha, beta = [v], [], [], []
    u = apply(v)
    for _ in range(steps):
        for _rep in range(2):
            for w in us:
                u -= (w @ u) * w
        a = float(np.linalg.norm(u))
        if a == 0.0:
            break
        u = u / a
        us.append(u)
        alpha.append(a)
        v = apply_t(u) - a * vs[-1]
        for _rep in range(2):
            for w in vs:
                v -= (w @ v) * w
        bt = float(np.linalg.norm(v))
        if bt <= 1e-300 or len(vs) >= n:
            break
        v = v / bt
        vs.append(v)
        beta.append(bt)
        u = apply(v) - bt * u
    k = len(alpha)
    if k == 0:
        return 0.0
    B = np.diag(alpha)
    for i in range(min(len(beta), k - 1)):
        B[i, i + 1] = beta[i]
    return float(np.linalg.norm(B, 2))


def spec_lanczos(X: np.ndarray, steps: int = 200) -> float:
    """||X||_2 through ``lanczos_norm`` (exact ``spec`` when X is small)."""
    if X.size == 0:
        return 0.0
    if min(X.shape) <= 64:
        return spec(X)
    return lanczos_norm(lambda x: X @ x, lambda y: X.T @ y, X.shape[1], steps)
