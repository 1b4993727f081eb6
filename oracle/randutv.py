"""Oracle for randUTV_basic (Alg. 3, Appendix B of the paper), FP64 on the CPU.

TEST INFRASTRUCTURE: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import anything under ``oracle/``.

The algorithm is randomized, so there is no closed-form output to write down;
this module executes Alg. 3 step by step in the paper's order and notation
(index sets I1, I2, I3 and J1, J2, J3; Sec. 4.1 explains each step), with
LAPACK Householder routines as the HQR_full steps and numpy's SVD for the
small blocks. Readings of points the paper leaves open:

* the Gaussian ``G`` of step i is ``gaussian(seed, stream=i)`` (1-based);
* ``HQR_full`` uses the LAPACK ``dlarfg`` reflector sign rule;
* the final (else) branch takes the SVD of a tall trailing block as an
  unpivoted QR followed by the SVD of its square R factor (the tall-thin SVD
  of Sec. 4.2, remark on Chan's method); for ``m == n`` with ``b | n`` it is a
  plain b x b SVD;
* small SVDs are ordered descending with the sign rule of ``small_svd``;
* the loop bound is ``s = ceil(n / b)`` for ``m >= n``;
* a wide A (m < n) is factored through its transpose (Sec. 3.2), which
  makes T lower trapezoidal.
"""
from __future__ import annotations

import math
from typing import Callable, Optional

import numpy as np

from .hqr import apply_q, hqr
from .philox import gaussian
from .small_svd import small_svd


def randutv(
    A: np.ndarray,
    b: int,
    q: int,
    seed: int,
    *,
    want_u: bool = True,
    want_v: bool = True,
    max_steps: Optional[int] = None,
    on_step: Optional[Callable[[int, np.ndarray], None]] = None,
    stop_before: Optional[Callable[[int, np.ndarray], bool]] = None,
):
    """Compute ``A = U T V^T`` by Alg. 3.

    Returns ``(U, T, V)``; U (m x m) and V (n x n) are ``None`` when not
    requested. ``max_steps`` stops after that many loop iterations (used to
    time a bounded sample); ``on_step(i, T)`` sees T after step i;
    ``stop_before(i, T)`` returning True ends the loop before step i.
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if m < n:
        # Sec. 3.2: a wide matrix is factored through its transpose,
        # A^T = U' T' V'^T, so A = V' T'^T U'^T with T'^T lower trapezoidal
        if stop_before is not None or max_steps is not None or on_step is not None:
            raise ValueError("the step hooks need m >= n")
        Ut, Tt, Vt = randutv(A.T, b, q, seed, want_u=want_v, want_v=want_u)
        return Vt, np.asfortranarray(Tt.T), Ut
    if b < 1 or q < 0:
        raise ValueError("need b >= 1 and q >= 0")
    T = np.array(A, order="F", copy=True)
    U = np.eye(m, order="F") if want_u else None
    V = np.eye(n, order="F") if want_v else None
    s = math.ceil(n / b)
    for i in range(1, s + 1):
        if max_steps is not None and i > max_steps:
            break
        if stop_before is not None and stop_before(i, T):
            break
        # Index sets (0-based, half-open): I1 = [0,c0), I2 = [c0,r2), I3 = [r2,m)
        c0 = b * (i - 1)
        r2 = min(b * i, m)
        c2 = min(b * i, n)
        if r2 < m and c2 < n:
            # --- sketch of Row(T22):  Y = (T22^T T22)^q T22^T G
            G = gaussian(seed, i, m - c0, b)
            T22 = T[c0:, c0:]
            Y = T22.T @ G
            for _ in range(q):
                Y = T22.T @ (T22 @ Y)
            # --- [V_i, ~] = HQR_full(Y)
            Wv, tv = hqr(Y)
            # --- T(:, J2∪J3) <- T(:, J2∪J3) V_i ;  V(:, J2∪J3) <- V(:, J2∪J3) V_i
            T[:, c0:] = apply_q(Wv, tv, T[:, c0:], "R", "N")
            if V is not None:
                V[:, c0:] = apply_q(Wv, tv, V[:, c0:], "R", "N")
            # --- [U_i, R] = HQR_full(T(I2∪I3, J2))
            Wu, tu = hqr(T[c0:, c0:c2])
            R = np.triu(Wu[: c2 - c0, : c2 - c0])
            # --- U(:, I2∪I3) <- U(:, I2∪I3) U_i ;  T(I2∪I3, J3) <- U_i^T T(I2∪I3, J3)
            if U is not None:
                U[:, c0:] = apply_q(Wu, tu, U[:, c0:], "R", "N")
            T[c0:, c2:] = apply_q(Wu, tu, T[c0:, c2:], "L", "T")
            # --- T(I3, J2) = 0
            T[r2:, c0:c2] = 0.0
            # --- small SVD of the b x b diagonal block and its updates
            Us, d, Vs = small_svd(R)
            if U is not None:
                U[:, c0:r2] = U[:, c0:r2] @ Us
            if V is not None:
                V[:, c0:c2] = V[:, c0:c2] @ Vs
            T[c0:r2, c0:c2] = np.diag(d)
            T[c0:r2, c2:] = Us.T @ T[c0:r2, c2:]
            T[:c0, c0:c2] = T[:c0, c0:c2] @ Vs
        else:
            # --- last block: SVD of T(I2∪I3, J2∪J3)
            B = np.array(T[c0:, c0:], order="F")
            M, N = B.shape
            if M > N:
                # tall-thin SVD: HQR_full, then SVD of the N x N R factor
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
        if on_step is not None:
            on_step(i, T)
    return U, T, V



def randutv_partial(A: np.ndarray, b: int, q: int, seed: int, tol: float, kmax: int, *,
                    want_u: bool = True, want_v: bool = True):
    """Alg. 3 halted early (Sec. 4.1, error of the rank-k approximation):
    before step i (0-based, c0 = i b) the loop stops when c0 >= kmax or when
    e_i = ||T(c0:, c0:)||_F <= tol ||A||_F. Returns ``(U, T, V, k)`` with
    k = the columns already reduced (T(k:, k:) is the unreduced remainder
    and A = U T V^T holds exactly as for the full factorization)."""
    A = np.asarray(A, dtype=np.float64)
    if A.shape[0] < A.shape[1]:
        # a wide matrix through its transpose (Sec. 3.2), k counting the
        # transpose's reduced columns
        Ut, Tt, Vt, k = randutv_partial(A.T, b, q, seed, tol, kmax, want_u=want_v, want_v=want_u)
        return Vt, np.asfortranarray(Tt.T), Ut, k
    e0 = float(np.linalg.norm(A))
    done = [0]

    def stop_before(i, T):
        c0 = b * (i - 1)
        if c0 >= kmax or float(np.linalg.norm(T[c0:, c0:])) <= tol * e0:
            return True
        done[0] = i
        return False

    U, T, V = randutv(A, b, q, seed, want_u=want_u, want_v=want_v, stop_before=stop_before)
    return U, T, V, min(b * done[0], A.shape[1])
