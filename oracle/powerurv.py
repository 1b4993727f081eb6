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

Mixed mode (``precision="bf16"``; the paper is FP64 throughout): the 2q
power products only have to carry the dominant right singular subspace of A
into V, so they are formed from bfloat16 values: A scaled by its
``pow2_scale`` and rounded once, V and V_hat rounded as they are (their
entries lie in [-1, 1]); the products of the rounded values are formed here
in FP64 (the GPU accumulates them in FP32, within ``fp32_gemm_bound``). A
positive scale of a product leaves its Householder Q unchanged. The QRs,
the explicit Q factors and the final ``A_hat = A V`` stay FP64.
"""
from __future__ import annotations

import numpy as np

from .bf16 import bf16_round, pow2_scale
from .hqr import form_q, hqr
from .philox import gaussian


def powerurv(A: np.ndarray, q: int, seed: int, *, rounds: int | None = None,
             precision: str = "fp64"):
    """Return ``(U, T, V)`` with ``A = U T V^T``.

    ``rounds`` (test/timing aid) stops the power loop after that many rounds
    and returns ``(None, None, V)``. ``precision="bf16"`` forms the power
    products from bfloat16 values (module docstring).
    """
    if precision not in ("fp64", "bf16"):
        raise ValueError("precision must be 'fp64' or 'bf16'")
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if m < n:
        # Sec. 3.2's reading for a wide matrix, as in randUTV: factor the
        # transpose, A^T = U' T' V'^T, so A = V' T'^T U'^T (T lower trapezoidal)
        if rounds is not None:
            raise ValueError("rounds needs m >= n")
        Ut, Tt, Vt = powerurv(A.T, q, seed, precision=precision)
        return Vt, np.asfortranarray(Tt.T), Ut
    if q < 0:
        raise ValueError("q must be non-negative")
    G = gaussian(seed, 0, n, n)
    if q == 0:
        W, tau = hqr(G)
        V = form_q(W, tau, n)
    else:
        V = G
    if precision == "bf16" and q > 0:
        Ap = bf16_round(A * pow2_scale(A))  # A scaled by a power of two, rounded once
        rnd = bf16_round
    else:
        Ap, rnd = A, (lambda X: X)
    for j in range(q):
        if rounds is not None and j >= rounds:
            return None, None, V
        Y_hat = Ap @ rnd(V)                # m x n
        W, tau = hqr(Y_hat)
        V_hat = form_q(W, tau, n)          # HQR_thin: m x n orthonormal
        Y = Ap.T @ rnd(V_hat)              # n x n
        W, tau = hqr(Y)
        V = form_q(W, tau, n)              # n x n orthogonal
    A_hat = A @ V
    W, tau = hqr(A_hat)
    U = form_q(W, tau, m)                  # HQR_full: m x m orthogonal
    T = np.triu(W)                         # m x n upper trapezoidal R
    return U, T, V

