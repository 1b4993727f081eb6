"""Oracle for powerURV (Alg. 1 of the paper), FP64 on the CPU.

TEST INFRASTRUCTURE: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import anything under ``oracle/``.

Follows Alg. 1 (Sec. 3.2) in order: a Gaussian start V, q rounds of
``A V -> HQR_thin -> A^T (.) -> HQR_thin``, then ``A_hat = A V`` and
``[U, R] = HQR_full(A_hat)``. Readings of points the paper leaves open:

* the Gaussian is ``gaussian(seed, stream=0, n, n)``;
* for ``q = 0`` Alg. 1 would return the non-orthogonal Gaussian as V although
  its contract and the RURV it reduces to (Sec. 3.1, step 2) require
  ``V = Q`` of ``HQR_full(G)``; the oracle takes that RURV step;
* HQR uses LAPACK's ``dlarfg`` reflector signs; the returned ``T`` is the
  upper trapezoidal R of the final QR, so ``T(k,k)`` may be negative.
"""
from __future__ import annotations

import numpy as np

from .hqr import form_q, hqr
from .philox import gaussian


def powerurv(A: np.ndarray, q: int, seed: int, *, rounds: int | None = None):
    """Return ``(U, T, V)`` with ``A = U T V^T``.

    ``rounds`` (test/timing aid) stops the power loop after that many rounds
    and returns ``(None, None, V)``.
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if m < n:
        raise ValueError("powerurv oracle requires m >= n")
    if q < 0:
        raise ValueError("q must be non-negative")
    G = gaussian(seed, 0, n, n)
    if q == 0:
        W, tau = hqr(G)
        V = form_q(W, tau, n)
    else:
        V = G
    for j in range(q):
        if rounds is not None and j >= rounds:
            return None, None, V
        Y_hat = A @ V                      # m x n
        W, tau = hqr(Y_hat)
        V_hat = form_q(W, tau, n)          # HQR_thin: m x n orthonormal
        Y = A.T @ V_hat                    # n x n
        W, tau = hqr(Y)
        V = form_q(W, tau, n)              # n x n orthogonal
    A_hat = A @ V
    W, tau = hqr(A_hat)
    U = form_q(W, tau, m)                  # HQR_full: m x m orthogonal
    T = np.triu(W)                         # m x n upper trapezoidal R
    return U, T, V

