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
