"""Oracle for the randomized SVD (RSVD, Sec. 3.3: the relationship with
powerURV), FP64 on the CPU.

TEST INFRASTRUCTURE: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import anything under ``oracle/``.

The plain definition, in the paper's order: Y = (A A^T)^q A G with
G = G_powerURV(:, 1:l) (the Gaussian of stream 0, so Theorem 1 compares the
two methods on the same draw), Q from a thin unpivoted QR of Y, the thin SVD
Q^T A = W Sigma V^T, and U = Q W. numpy's QR and SVD serve as the library
steps; singular values descend. m < n needs no transposition (every step is
defined for l <= min(m, n)).
"""
from __future__ import annotations

import numpy as np

from .philox import gaussian


def rsvd(A: np.ndarray, l: int, q: int, seed: int):
    """Return ``(U, s, V)``: U (m x l) and V (n x l) orthonormal, s (l)
    descending, with A ~ U diag(s) V^T."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if not 1 <= l <= min(m, n) or q < 0:
        raise ValueError("need 1 <= l <= min(m, n) and q >= 0")
    G = gaussian(seed, 0, n, l)
    Y = A @ G
    for _ in range(q):
        Y = A @ (A.T @ Y)
    Q, _ = np.linalg.qr(Y)
    W, s, Vt = np.linalg.svd(Q.T @ A, full_matrices=False)
    return Q @ W, s, Vt.T
