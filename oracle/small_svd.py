"""Oracle SVD of the small diagonal blocks, with a fixed order and sign rule.

TEST INFRASTRUCTURE: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import anything under ``oracle/``.

Alg. 3 (and Alg. 2) take ``svd(R(1:b,1:b))`` of each b x b diagonal block and
``svd`` of the last trailing block without fixing order or signs. Readings
used throughout this project:

* singular values in descending order, so that ``T(k,k)`` approximates
  ``sigma_k`` (Sec. 4.1, item 5 of the first-step goals);
* signs: each pair ``(u_k, v_k)`` is flipped so that the entry of ``v_k``
  of largest magnitude is positive (ties go to the lowest row index).

The signs only touch rows and columns that are already processed, so the
trailing block and every later diagonal value are independent of this rule.
"""
from __future__ import annotations

import numpy as np


def canonical_signs(Us: np.ndarray, Vs: np.ndarray) -> None:
    """Flip (u_k, v_k) pairs in place per the sign rule above."""
    k = min(Us.shape[1], Vs.shape[1])
    for j in range(k):
        col = Vs[:, j]
        if col.size == 0:
            continue
        idx = int(np.argmax(np.abs(col)))
        if col[idx] < 0:
            Vs[:, j] = -Vs[:, j]
            Us[:, j] = -Us[:, j]


def small_svd(B: np.ndarray) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Full SVD ``B = Us diag(d) Vs^T`` of a small matrix with rows >= cols.

    Returns ``Us`` (rows x rows), ``d`` (cols,), ``Vs`` (cols x cols).
    """
    B = np.asarray(B, dtype=np.float64)
    Us, d, VsT = np.linalg.svd(B, full_matrices=True)
    Us = np.array(Us, order="F")
    Vs = np.array(VsT.T, order="F")
    canonical_signs(Us, Vs)
    return Us, d, Vs
