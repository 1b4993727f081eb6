"""Oracle for randUTV_boosted (Alg. 2, Sec. 4.2-4.3 of the paper), FP64 on
the CPU.

TEST INFRASTRUCTURE: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import anything under ``oracle/``.

Alg. 2 is Alg. 3 with b + p samples per step, V_i built from the leading b
left singular vectors of the sample matrix Y (method b of Sec. 4.2: an
unpivoted QR of Y, the SVD of its square R factor, then HQR_full of
W_Y(:, 1:b)), and, after the first step, the p extra samples recycled from
the previous step instead of drawn and power-iterated again (Sec. 4.3).
This module executes the algorithm step by step in the paper's order, with
the readings of ``oracle/randutv.py`` (G of step i from stream i, dlarfg
reflectors, descending small SVDs with its sign rule, s = ceil(n / b), the
tall-thin final SVD) and these for the points Alg. 2 leaves open:

* ``W_next``. The text defines it as V_i(:, b+1:N_i)^T W_Y(:, b+1:b+p): the
  previous step's approximations of the right singular vectors b+1..b+p,
  written in the coordinates of the next trailing block's columns (N_{i+1}
  x p). The listing then uses it on the left of the trailing block
  (``X - W W^T X`` with X = T22 Y, and ``T22^T [Q, W]``), which needs
  M_{i+1} rows. Reading: W_next is kept as the text defines it, and at the
  next step its image T22 W_next, orthonormalised by an unpivoted QR (Wl,
  M_i x p), takes its place in those two lines. The recycled columns then
  cost one product of width p instead of 2q + 1.
* Oversampling width. Step i takes p_i = min(p, N_i - b) extra samples, so
  Y never has more columns than rows; a carried W_next keeps its first p_i
  columns.
* q = 0 after the first step. The listing's X = T22 Y(:, 1:b) would be a
  full power step; with q = 0 the left sample is X = G itself, so that the
  b fresh columns of Y = T22^T [Q, Wl] see T22 once, as in Alg. 3.
* G of step 1 has b + p_1 columns (stream 1); its first b columns are Alg.
  3's G_1.
"""
from __future__ import annotations

import math

import numpy as np

from .hqr import apply_q, form_q, hqr
from .philox import gaussian
from .small_svd import small_svd


def left_singular_vectors(Y: np.ndarray) -> np.ndarray:
    """The k = Y.shape[1] leading left singular vectors of a tall Y, by the
    tall-thin method of Sec. 4.2 (remark on Chan's method): Y = Q R, then
    W_Y = Q(:, 1:k) U_R with U_R the left singular vectors of R (descending)."""
    k = Y.shape[1]
    Wy, ty = hqr(Y)
    Uh, _, _ = small_svd(np.triu(Wy[:k, :k]))
    return form_q(Wy, ty, k) @ Uh


def randutv_boosted(A: np.ndarray, b: int, q: int, p: int, seed: int, *, want_u: bool = True,
                    want_v: bool = True):
    """Compute ``A = U T V^T`` by Alg. 2; returns ``(U, T, V)`` (None when
    not requested)."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if m < n:
        # a wide matrix through its transpose (Sec. 3.2), as for Alg. 3
        Ut, Tt, Vt = randutv_boosted(A.T, b, q, p, seed, want_u=want_v, want_v=want_u)
        return Vt, np.asfortranarray(Tt.T), Ut
    if b < 1 or q < 0 or p < 0:
        raise ValueError("need b >= 1, q >= 0 and p >= 0")
    T = np.array(A, order="F", copy=True)
    U = np.eye(m, order="F") if want_u else None
    V = np.eye(n, order="F") if want_v else None
    W_next = None
    for i in range(1, math.ceil(n / b) + 1):
        c0 = b * (i - 1)
        r2 = min(b * i, m)
        c2 = min(b * i, n)
        if r2 < m and c2 < n:
            T22 = T[c0:, c0:]
            Mi, Ni = T22.shape
            pi = min(p, Ni - b)
            # --- the sample matrix Y (N_i x (b + p_i))
            if i == 1:
                G = gaussian(seed, 1, Mi, b + pi)
                Y = T22.T @ G
                for _ in range(q):
                    Y = T22.T @ (T22 @ Y)
            else:
                G = gaussian(seed, i, Mi, b)
                if q >= 1:
                    Yb = T22.T @ G
                    for _ in range(q - 1):
                        Yb = T22.T @ (T22 @ Yb)
                    X = T22 @ Yb
                else:
                    X = G
                Wl = None
                if pi > 0:
                    Wz, tz = hqr(T22 @ W_next[:, :pi])
                    Wl = form_q(Wz, tz, pi)
                    X = X - Wl @ (Wl.T @ X)
                Wx, tx = hqr(X)
                S = form_q(Wx, tx, b)
                if Wl is not None:
                    S = np.hstack([S, Wl])
                Y = T22.T @ S
            # --- [W_Y, ~, ~] = SVD(Y);  [V_i, ~] = HQR_full(W_Y(:, 1:b))
            WY = left_singular_vectors(Y)
            Wv, tv = hqr(WY[:, :b])
            T[:, c0:] = apply_q(Wv, tv, T[:, c0:], "R", "N")
            if V is not None:
                V[:, c0:] = apply_q(Wv, tv, V[:, c0:], "R", "N")
            # --- W_next = V_i(:, b+1:N_i)^T W_Y(:, b+1:b+p_i)
            W_next = apply_q(Wv, tv, WY[:, b:], "L", "T")[b:, :]
            # --- the rest of the step as Alg. 3
            Wu, tu = hqr(T[c0:, c0:c2])
            R = np.triu(Wu[: c2 - c0, : c2 - c0])
            if U is not None:
                U[:, c0:] = apply_q(Wu, tu, U[:, c0:], "R", "N")
            T[c0:, c2:] = apply_q(Wu, tu, T[c0:, c2:], "L", "T")
            T[r2:, c0:c2] = 0.0
            Us, d, Vs = small_svd(R)
            if U is not None:
                U[:, c0:r2] = U[:, c0:r2] @ Us
            if V is not None:
                V[:, c0:c2] = V[:, c0:c2] @ Vs
            T[c0:r2, c0:c2] = np.diag(d)
            T[c0:r2, c2:] = Us.T @ T[c0:r2, c2:]
            T[:c0, c0:c2] = T[:c0, c0:c2] @ Vs
        else:
            B = np.array(T[c0:, c0:], order="F")
            M, N = B.shape
            if M > N:
                Wb, tb = hqr(B)
                if U is not None:
                    U[:, c0:] = apply_q(Wb, tb, U[:, c0:], "R", "N")
                B = np.triu(Wb[:N, :N])
            Us, d, Vs = small_svd(B)
            if U is not None:
                U[:, c0 : c0 + N] = U[:, c0 : c0 + N] @ Us
            if V is not None:
                V[:, c0:] = V[:, c0:] @ Vs
            T[c0:, c0:] = 0.0
            T[c0 : c0 + N, c0:] = np.diag(d)
            T[:c0, c0:] = T[:c0, c0:] @ Vs
    return U, T, V
