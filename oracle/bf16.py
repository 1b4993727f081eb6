"""Reduced-precision sketch of randUTV's mixed mode, on the CPU.

TEST INFRASTRUCTURE: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import anything under ``oracle/``.

The paper computes everything in FP64. The sketch of Alg. 3,
Y = (T22^T T22)^q T22^T G, only has to capture the dominant right singular
subspace of T22, so the mixed mode forms it from bfloat16 copies of T22 and
G with FP32 accumulation; the QR of Y and every update of T, U and V stay in
FP64. The definitions the GPU path follows:

* ``bf16_round(x)``: round-to-nearest, ties-to-even, of a binary64 value to
  bfloat16 (8 significant bits, the exponent range of binary32), directly from
  binary64 (no intermediate binary32 rounding). Below 2^-126 the quantum is
  fixed at 2^-133 (gradual underflow); beyond the largest finite bfloat16
  value the result is +-inf.
* ``pow2_scale(x)``: the power of two 2^-e with max|x| 2^-e in [0.5, 1),
  e from frexp of max|x| (1 when x is all zero). Multiplying by it is exact.
* ``split_x3(x)`` and ``gemm_x3(A, B)``: the product of the x3 updates.
  x32 = x rounded to binary32 (nearest even), hi = x32 rounded to bfloat16,
  lo = (x32 - hi) rounded to bfloat16 (the subtraction is exact); the
  product keeps the three leading terms of (hi_a + lo_a)(hi_b + lo_b),
  hi_a hi_b + hi_a lo_b + lo_a hi_b, each exact, summed here in FP64 (the
  GPU sums them in FP32: ``fp32_x3_bound``). The split keeps about 17
  bits (|x - hi - lo| <= (2^-17 + 2^-24) |x|); per term the dropped part,
  mostly lo_a lo_b, is at most about 2^-15 |a| |b|.
* ``split_x6(x)`` and ``gemm_x6(A, B)``: the product of the x6 updates.
  x32 as above, hi = x32 rounded to bfloat16, mid = (x32 - hi) rounded to
  bfloat16, lo = (x32 - hi - mid) rounded to bfloat16 (nearest even, each
  subtraction exact in binary32), so hi + mid + lo = x32. The product keeps
  the six leading terms of (hi_a + mid_a + lo_a)(hi_b + mid_b + lo_b),
  hi hi + hi mid + mid hi + hi lo + lo hi + mid mid, each exact, summed here
  in FP64 (the GPU sums the terms of each K slice of 32 in binary32 and the
  slices in binary64: ``fp32_x6_bound``). The dropped mid lo + lo mid + lo lo
  is below about 2^-23 |a| |b| per term.
* ``sketch_bf16(T22, G, q)``: T22 is scaled by its pow2_scale and rounded
  to bfloat16, G (standard normal, in range) is rounded as it is;
  Y = T^T G; then q times: round Y column by column
  after scaling each column by its own pow2_scale, Z = T Y, the same for Z,
  Y = T^T Z. Positive column scalings commute with the products and leave
  the column space (hence the Householder Q of Y) unchanged; they only keep
  the FP32 range. This reference forms the products of the rounded values in
  FP64; the GPU accumulates them in FP32, so the two agree to within the FP32
  accumulation bound of ``fp32_gemm_bound`` per product.
"""
from __future__ import annotations

import numpy as np

_SIG = 8                    # significant bits of bfloat16
_EMIN = -126                # smallest normal exponent (value 2^-126)
_MAX = (2.0 - 2.0 ** -7) * 2.0 ** 127  # largest finite bfloat16
U32 = 2.0 ** -24            # unit roundoff of binary32


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round binary64 values to the nearest bfloat16 value (ties to even)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    fin = np.isfinite(x) & (x != 0.0)
    _, e = np.frexp(x[fin])           # x = f 2^e, 0.5 <= |f| < 1, so 2^(e-1) <= |x|
    # exponent of the leading bit is e - 1; the last kept bit is 2^(e-1-7),
    # never below the subnormal quantum 2^(-126-7)
    lead = np.maximum(e - 1, _EMIN)
    quantum_exp = lead - (_SIG - 1)
    q = np.rint(np.ldexp(x[fin], -quantum_exp))  # numpy rint: ties to even
    r = np.ldexp(q, quantum_exp)
    r[np.abs(r) > _MAX] = np.copysign(np.inf, r[np.abs(r) > _MAX])
    out[fin] = r
    out[~fin] = x[~fin]               # zeros (with sign), infs and NaNs pass through
    return out


def pow2_scale(x: np.ndarray) -> float:
    """2^-e with max|x| 2^-e in [0.5, 1); 1.0 for an all-zero input."""
    m = float(np.max(np.abs(x))) if x.size else 0.0
    if m == 0.0:
        return 1.0
    _, e = np.frexp(m)
    return float(np.ldexp(1.0, -int(e)))


def gemm_tn_reference(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """A^T B of bfloat16-exact inputs, formed in FP64 (the products are exact)."""
    return np.asarray(A, np.float64).T @ np.asarray(B, np.float64)


def fp32_gemm_bound(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Elementwise bound on |fl32(A^T B) - A^T B| for any summation order:
    gamma_K |A|^T |B| with gamma_K = K u / (1 - K u), u = 2^-24, plus the
    final rounding of the result to binary32."""
    K = A.shape[0]
    g = K * U32 / (1.0 - K * U32)
    absprod = np.abs(A).T @ np.abs(B)
    return g * absprod + U32 * absprod


def _round_columns(X: np.ndarray) -> np.ndarray:
    out = np.empty_like(X)
    for j in range(X.shape[1]):
        out[:, j] = bf16_round(X[:, j] * pow2_scale(X[:, j]))
    return out


def sketch_bf16(T22: np.ndarray, G: np.ndarray, q: int) -> np.ndarray:
    """The mixed sketch's steps (module docstring), products in FP64."""
    Tb = bf16_round(T22 * pow2_scale(T22))
    Gb = bf16_round(G)
    Y = Tb.T @ Gb
    for _ in range(q):
        Z = Tb @ _round_columns(Y)
        Y = Tb.T @ _round_columns(Z)
    return Y


def split_x3(x: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """(hi, lo) of the x3 split (module docstring), as binary64 arrays."""
    x32 = np.asarray(x, np.float64).astype(np.float32).astype(np.float64)
    hi = bf16_round(x32)
    lo = bf16_round(x32 - hi)
    return hi, lo


def gemm_x3(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """A B (A: M x K, B: K x N) by the three-pass split product, in FP64."""
    Ah, Al = split_x3(A)
    Bh, Bl = split_x3(B)
    return Ah @ Bh + Ah @ Bl + Al @ Bh


def fp32_x3_bound(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Elementwise bound on |GPU - gemm_x3(A, B)|: the 3K exact terms summed
    in binary32 in any order (gamma_{3K}) plus the final binary32 rounding."""
    Ah, Al = split_x3(A)
    Bh, Bl = split_x3(B)
    K3 = 3 * A.shape[1]
    g = K3 * U32 / (1.0 - K3 * U32)
    absprod = np.abs(Ah) @ np.abs(Bh) + np.abs(Ah) @ np.abs(Bl) + np.abs(Al) @ np.abs(Bh)
    return (g + U32) * absprod


def split_x6(x: np.ndarray) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(hi, mid, lo) of the x6 split (module docstring), as binary64 arrays."""
    x32 = np.asarray(x, np.float64).astype(np.float32).astype(np.float64)
    hi = bf16_round(x32)
    mid = bf16_round(x32 - hi)
    lo = bf16_round(x32 - hi - mid)
    return hi, mid, lo


def _x6_terms(A: np.ndarray, B: np.ndarray):
    Ah, Am, Al = split_x6(A)
    Bh, Bm, Bl = split_x6(B)
    return [(Ah, Bh), (Ah, Bm), (Am, Bh), (Ah, Bl), (Al, Bh), (Am, Bm)]


def gemm_x6(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """A B (A: M x K, B: K x N) by the six-term split product, in FP64."""
    return sum(a @ b for a, b in _x6_terms(A, B))


def fp32_x6_bound(A: np.ndarray, B: np.ndarray, slice_k: int = 32) -> np.ndarray:
    """Elementwise bound on |GPU - gemm_x6(A, B)|: per K slice of slice_k,
    its 6 slice_k exact terms summed in binary32 in any order
    (gamma_{6 slice_k}) and rounded to binary32, the slice sums added in
    binary64 (gamma of the slice count at u = 2^-53)."""
    K = A.shape[1]
    n6 = 6 * slice_k
    g32 = n6 * U32 / (1.0 - n6 * U32) + U32
    nslices = max(1, -(-K // slice_k))
    g64 = nslices * 2.0 ** -53 / (1.0 - nslices * 2.0 ** -53)
    absprod = sum(np.abs(a) @ np.abs(b) for a, b in _x6_terms(A, B))
    return (g32 + g64) * absprod
