"""Oracle side of the sketch generator: Philox4x64-10 followed by Box-Muller.

TEST INFRASTRUCTURE. Nothing under ``oracle/`` is part of the product path;
only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it.

The paper draws its sketch matrices with ``randn`` (Sec. 2.4 step 1, Alg. 1
first step, Alg. 3 inside the loop) and does not say how. This project fixes
one counter-based definition so that the CPU oracle and the GPU library, which
share no code, draw the *same* Gaussian matrix from ``(seed, stream)``:

* generator: Philox4x64 with 10 rounds (Salmon, Moraes, Dror, Shaw, "Parallel
  random numbers: as easy as 1, 2, 3", SC'11), key ``(seed, stream)``,
  counter ``(r // 4, c, 0, 0)`` for entry ``(r, c)`` of the matrix;
* the four 64-bit output words ``w0..w3`` become two pairs of uniforms
  ``u = ((w >> 11) + 1) * 2**-53`` in (0, 1] (from w0, w2) and
  ``v = (w >> 11) * 2**-53`` in [0, 1) (from w1, w3);
* Box-Muller: ``rho = sqrt(-2 ln u)``, ``theta = 2*pi*v``; rows ``4k+0,1``
  take ``rho_a*cos(theta_a), rho_a*sin(theta_a)`` and rows ``4k+2,3`` take
  ``rho_b*cos(theta_b), rho_b*sin(theta_b)``.

Entry (r, c) depends only on (seed, stream, r, c), so a smaller matrix drawn
from the same stream is the top-left block of a larger one.

This file implements the generator from its published definition with
vectorised numpy uint64 arithmetic; the test-suite pins it against numpy's own
``numpy.random.Philox`` bit generator, which is the same algorithm.
"""
from __future__ import annotations

import numpy as np

# Philox4x64 round multipliers and Weyl key increments (SC'11, Sec. 5).
PHILOX_M0 = np.uint64(0xD2E7470EE14C6C93)
PHILOX_M1 = np.uint64(0xCA5A826395121157)
PHILOX_W0 = np.uint64(0x9E3779B97F4A7C15)
PHILOX_W1 = np.uint64(0xBB67AE8584CAA73B)
ROUNDS = 10

TWO_PI = 6.283185307179586  # the double nearest 2*pi
_MASK32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a: np.ndarray, b: np.uint64) -> tuple[np.ndarray, np.ndarray]:
    """Full 64x64 -> 128-bit product of uint64 arrays, as (hi, lo)."""
    a = a.astype(np.uint64)
    b = np.uint64(b)
    a_lo, a_hi = a & _MASK32, a >> _S32
    b_lo, b_hi = b & _MASK32, b >> _S32
    with np.errstate(over="ignore"):
        ll = a_lo * b_lo
        lh = a_lo * b_hi
        hl = a_hi * b_lo
        hh = a_hi * b_hi
        mid = (ll >> _S32) + (lh & _MASK32) + (hl & _MASK32)
        lo = (ll & _MASK32) | ((mid & _MASK32) << _S32)
        hi = hh + (lh >> _S32) + (hl >> _S32) + (mid >> _S32)
    return hi, lo


def philox4x64_10(ctr, key):
    """Philox4x64-10 block function on arrays of counters.

    ``ctr`` is a sequence of four uint64 arrays (broadcastable), ``key`` a pair
    of uint64 scalars or arrays. Returns the four uint64 output words.
    """
    x0, x1, x2, x3 = (np.asarray(c, dtype=np.uint64) for c in ctr)
    k0 = np.asarray(key[0], dtype=np.uint64)
    k1 = np.asarray(key[1], dtype=np.uint64)
    with np.errstate(over="ignore"):
        for rnd in range(ROUNDS):
            if rnd:
                k0 = k0 + PHILOX_W0
                k1 = k1 + PHILOX_W1
            hi0, lo0 = _mulhilo(x0, PHILOX_M0)
            hi1, lo1 = _mulhilo(x2, PHILOX_M1)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return x0, x1, x2, x3


def uniforms_from_words(w: np.ndarray, open_at_zero: bool) -> np.ndarray:
    """53-bit uniform double from a 64-bit word; (0,1] if ``open_at_zero``."""
    top = (np.asarray(w, dtype=np.uint64) >> np.uint64(11)).astype(np.float64)
    if open_at_zero:
        top = top + 1.0
    return top * (2.0 ** -53)


def gaussian(seed: int, stream: int, rows: int, cols: int) -> np.ndarray:
    """The ``rows x cols`` standard Gaussian matrix of ``(seed, stream)``.

    Returned in column-major (Fortran) order, float64.
    """
    if rows <= 0 or cols <= 0:
        return np.zeros((max(rows, 0), max(cols, 0)), dtype=np.float64, order="F")
    groups = (rows + 3) // 4
    g = np.arange(groups, dtype=np.uint64)[:, None]
    c = np.arange(cols, dtype=np.uint64)[None, :]
    zero = np.zeros((1, 1), dtype=np.uint64)
    key = (np.uint64(seed & 0xFFFFFFFFFFFFFFFF), np.uint64(stream & 0xFFFFFFFFFFFFFFFF))
    w0, w1, w2, w3 = philox4x64_10((g, c, zero, zero), key)
    ua = uniforms_from_words(w0, True)
    va = uniforms_from_words(w1, False)
    ub = uniforms_from_words(w2, True)
    vb = uniforms_from_words(w3, False)
    rho_a = np.sqrt(-2.0 * np.log(ua))
    rho_b = np.sqrt(-2.0 * np.log(ub))
    th_a = TWO_PI * va
    th_b = TWO_PI * vb
    out = np.empty((groups * 4, cols), dtype=np.float64)
    out[0::4] = rho_a * np.cos(th_a)
    out[1::4] = rho_a * np.sin(th_a)
    out[2::4] = rho_b * np.cos(th_b)
    out[3::4] = rho_b * np.sin(th_b)
    return np.asfortranarray(out[:rows])
