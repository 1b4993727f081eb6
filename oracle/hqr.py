"""Oracle Householder QR building blocks (LAPACK, FP64).

TEST INFRASTRUCTURE: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import anything under ``oracle/``.

Sec. 2.3 of the paper defines HQR_full / HQR_thin as unpivoted Householder QR
and the compact-WY form ``Q = I - Y T Y*`` of the reflector product. The
oracle takes those steps from reference LAPACK (through scipy):

* ``dgeqrf``  -- reflectors ``H_i = I - tau_i v_i v_i^T`` with the ``dlarfg``
  sign rule (beta = -sign(alpha) * norm), stored below the diagonal with an
  implicit unit diagonal, and R on and above it;
* ``dormqr``  -- apply ``Q`` or ``Q^T`` from the left or the right;
* ``dorgqr``  -- form the leading columns of ``Q`` explicitly.

These are library primitives serving as single steps; nothing is blocked or
fused beyond what LAPACK itself does.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import lapack


def _lwork(query) -> int:
    return max(1, int(query[-2][0]))


def hqr(X: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Householder QR of ``X`` (m x k): returns (packed factor, tau)."""
    X = np.asfortranarray(X, dtype=np.float64)
    m, k = X.shape
    if m == 0 or k == 0:
        return X.copy(order="F"), np.zeros(min(m, k))
    lw = _lwork(lapack.dgeqrf(X, lwork=-1))
    qr, tau, _, info = lapack.dgeqrf(X, lwork=lw)
    if info != 0:
        raise RuntimeError(f"dgeqrf info={info}")
    return qr, tau


def apply_q(qr: np.ndarray, tau: np.ndarray, C: np.ndarray, side: str, trans: str) -> np.ndarray:
    """Return ``op(Q) C`` (side 'L') or ``C op(Q)`` (side 'R'), op = N or T.

    ``Q`` is the full orthogonal matrix whose reflectors are packed in ``qr``.
    """
    C = np.asfortranarray(C, dtype=np.float64)
    if C.size == 0 or tau.size == 0:
        return C.copy(order="F")
    lw = _lwork(lapack.dormqr(side, trans, qr, tau, C, -1))
    out, _, info = lapack.dormqr(side, trans, qr, tau, C, lw)
    if info != 0:
        raise RuntimeError(f"dormqr info={info}")
    return out


def form_q(qr: np.ndarray, tau: np.ndarray, ncols: int) -> np.ndarray:
    """The leading ``ncols`` columns of ``Q`` (ncols may exceed len(tau))."""
    m = qr.shape[0]
    k = tau.size
    A = np.zeros((m, ncols), dtype=np.float64, order="F")
    A[:, : min(ncols, qr.shape[1])] = qr[:, : min(ncols, qr.shape[1])]
    if k == 0:
        return np.eye(m, ncols, order="F")
    lw = _lwork(lapack.dorgqr(A, tau, lwork=-1))
    q, _, info = lapack.dorgqr(A, tau, lwork=lw)
    if info != 0:
        raise RuntimeError(f"dorgqr info={info}")
    return q


def r_factor(qr: np.ndarray) -> np.ndarray:
    """Upper trapezoidal R stored on and above the diagonal of ``qr``."""
    return np.triu(qr)
