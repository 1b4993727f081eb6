"""Pins of the mixed-sketch reference (oracle/bf16.py) against what fixes it
independently: torch's binary32 -> bfloat16 conversion (round to nearest
even) on values binary32 holds exactly, hand-worked rounding cases, BLAS
single-precision products, and exact arithmetic on representable inputs."""
import numpy as np
import pytest
import torch

from oracle.bf16 import (bf16_round, fp32_gemm_bound, fp32_x3_bound, fp32_x6_bound,
                         gemm_tn_reference, gemm_x3, gemm_x6, pow2_scale, sketch_bf16, split_x3,
                         split_x6)


def _torch_bf16(x32):
    return torch.from_numpy(np.asarray(x32, np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def test_bf16_round_matches_torch_on_binary32_values():
    rng = np.random.default_rng(0)
    x = np.concatenate([
        rng.standard_normal(20000),
        rng.standard_normal(20000) * 2.0 ** rng.integers(-140, 120, 20000),
        # exact ties between neighbouring bfloat16 values (odd and even)
        (np.arange(256, 512) + 0.5) * 2.0 ** -8,
        -(np.arange(256, 512) + 0.5) * 2.0 ** 20,
        # the subnormal range and its edge
        np.arange(1, 300) * 2.0 ** -136,
        np.array([2.0 ** -126, 2.0 ** -127, 2.0 ** -133, 1.5 * 2.0 ** -133, 2.5 * 2.0 ** -133]),
    ]).astype(np.float32).astype(np.float64)
    np.testing.assert_array_equal(bf16_round(x), _torch_bf16(x))


def test_bf16_round_hand_cases():
    # a tie rounds to the even neighbour: 1 + 2^-8 is halfway between 1 and 1 + 2^-7
    assert bf16_round(np.array([1.0 + 2.0 ** -8]))[0] == 1.0
    assert bf16_round(np.array([1.0 + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6
    # directly from binary64: just above the tie rounds up, although rounding
    # to binary32 first would land on the tie and then go down to 1
    x = 1.0 + 2.0 ** -8 + 2.0 ** -30
    assert np.float32(x) == np.float32(1.0 + 2.0 ** -8)
    assert bf16_round(np.array([x]))[0] == 1.0 + 2.0 ** -7
    # gradual underflow: quantum 2^-133 below 2^-126
    assert bf16_round(np.array([3 * 2.0 ** -134]))[0] == 2.0 ** -132  # 1.5 quanta -> 2
    assert bf16_round(np.array([2.0 ** -135]))[0] == 0.0              # a quarter quantum
    # overflow
    big = (2.0 - 2.0 ** -8) * 2.0 ** 127                              # tie with 2^128
    assert np.isinf(bf16_round(np.array([big]))[0])
    assert bf16_round(np.array([(2.0 - 2.0 ** -7) * 2.0 ** 127]))[0] == (2.0 - 2.0 ** -7) * 2.0 ** 127
    # specials pass through, the sign of zero is kept
    r = bf16_round(np.array([0.0, -0.0, np.inf, -np.inf, np.nan]))
    assert r[0] == 0.0 and np.signbit(r[1]) and np.isinf(r[2]) and r[3] < 0 and np.isnan(r[4])


def test_bf16_round_is_idempotent_and_monotone():
    rng = np.random.default_rng(1)
    x = np.sort(rng.standard_normal(100000) * 10.0)
    r = bf16_round(x)
    np.testing.assert_array_equal(bf16_round(r), r)
    assert np.all(np.diff(r) >= 0)
    # relative error at most half a unit in the 8th bit
    nz = x != 0
    assert np.max(np.abs(r[nz] - x[nz]) / np.abs(x[nz])) <= 2.0 ** -8


def test_pow2_scale():
    rng = np.random.default_rng(2)
    for s in (1e-300, 1e-20, 0.3, 1.0, 7.0, 1e30):
        x = rng.standard_normal((40, 7)) * s
        f = pow2_scale(x)
        assert np.frexp(f)[0] == 0.5                    # a power of two
        assert 0.5 <= np.max(np.abs(x)) * f < 1.0
    assert pow2_scale(np.zeros(5)) == 1.0
    assert pow2_scale(np.array([1.0])) == 0.5


def test_fp32_gemm_bound_covers_blas_single():
    rng = np.random.default_rng(3)
    for K in (16, 1000, 20000):
        A = bf16_round(rng.standard_normal((K, 24)))
        B = bf16_round(rng.standard_normal((K, 9)))
        exact = gemm_tn_reference(A, B)
        single = (A.astype(np.float32).T @ B.astype(np.float32)).astype(np.float64)
        assert np.all(np.abs(single - exact) <= fp32_gemm_bound(A, B))
        # the bound is not vacuous: well below the products' own size
        assert np.max(fp32_gemm_bound(A, B) / (np.abs(A).T @ np.abs(B))) < 2e-3


def test_sketch_bf16_exact_on_representable_inputs():
    # small integers and powers of two are bfloat16-exact and their products
    # and sums are exact in binary64, so q = 0 is exactly the scaled T^T G
    rng = np.random.default_rng(4)
    T = rng.integers(-8, 9, (50, 30)).astype(np.float64)
    G = rng.integers(-4, 5, (50, 6)).astype(np.float64)
    np.testing.assert_array_equal(sketch_bf16(T, G, 0), (T * pow2_scale(T)).T @ G)


def test_sketch_bf16_captures_the_dominant_subspace():
    # spectrum with a gap after 8 values: the mixed sketch spans the same
    # dominant right singular subspace as the exact one, to bfloat16 accuracy
    rng = np.random.default_rng(5)
    m, n, k = 400, 300, 8
    Q1, _ = np.linalg.qr(rng.standard_normal((m, n)))
    Q2, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = np.r_[np.linspace(10, 5, k), np.linspace(1e-2, 1e-4, n - k)]
    T = (Q1 * s) @ Q2.T
    G = rng.standard_normal((m, k))
    for q in (0, 1, 2):
        Y = sketch_bf16(T, G, q)
        Ye = T.T @ G
        for _ in range(q):
            Ye = T.T @ (T @ Ye)
        sin_mixed = np.linalg.norm(Q2[:, k:].T @ np.linalg.qr(Y)[0], 2)
        sin_exact = np.linalg.norm(Q2[:, k:].T @ np.linalg.qr(Ye)[0], 2)
        # as good as the exact sketch, down to the bfloat16 floor (~2^-8
        # relative, damped by the gap)
        assert sin_mixed <= max(1.2 * sin_exact, 2e-3), (q, sin_mixed, sin_exact)


def test_sketch_bf16_power_of_two_invariance():
    # scaling T or a column of G by a power of two changes no rounding:
    # T is renormalised, and for q >= 1 every column is renormalised before
    # each product, so the sketch is unchanged (q = 0 carries G's factor)
    rng = np.random.default_rng(6)
    T = rng.standard_normal((60, 40))
    G = rng.standard_normal((60, 5))
    D = 2.0 ** np.array([-60, -3, 0, 7, 90])
    for q in (1, 2):
        base = sketch_bf16(T, G, q)
        np.testing.assert_array_equal(sketch_bf16(T * 2.0 ** -100, G, q), base)
        np.testing.assert_array_equal(sketch_bf16(T, G * D, q), base)
    np.testing.assert_array_equal(sketch_bf16(T, G * D, 0), sketch_bf16(T, G, 0) * D)
    # far below the binary32 range: (1e-30)^5 would underflow without the
    # renormalisation, the sketch stays finite and non-zero
    Y = sketch_bf16(T * 1e-30, G, 2)
    assert np.all(np.isfinite(Y)) and np.all(np.linalg.norm(Y, axis=0) > 0.1)


# --------------------------------------------------------- x3 split product
def test_split_x3_matches_torch_roundings():
    # hi is torch's bfloat16 of the binary32 value, lo torch's bfloat16 of the
    # (exact) binary32 remainder
    rng = np.random.default_rng(10)
    x = np.concatenate([rng.standard_normal(20000),
                        rng.standard_normal(5000) * 2.0 ** rng.integers(-100, 100, 5000)])
    hi, lo = split_x3(x)
    x32 = torch.from_numpy(x).to(torch.float32)
    hi_t = x32.to(torch.bfloat16).to(torch.float32)
    lo_t = (x32 - hi_t).to(torch.bfloat16).to(torch.float64)
    np.testing.assert_array_equal(hi, hi_t.to(torch.float64).numpy())
    np.testing.assert_array_equal(lo, lo_t.numpy())


def test_split_x3_hand_cases():
    # x32 keeps 2^-20 and drops 2^-30; hi rounds the 2^-10 tail away (below
    # half an ulp of 1, 2^-8); lo rounds 2^-10 + 2^-20 to 2^-10 (2^-20 is
    # below half an ulp of 2^-10, 2^-18)
    hi, lo = split_x3(np.array([1.0 + 2.0 ** -10 + 2.0 ** -20 + 2.0 ** -30]))
    assert hi[0] == 1.0 and lo[0] == 2.0 ** -10
    # a binary32 tie of hi goes to the even neighbour, lo takes the rest
    hi, lo = split_x3(np.array([1.0 + 2.0 ** -8]))
    assert hi[0] == 1.0 and lo[0] == 2.0 ** -8
    hi, lo = split_x3(np.array([1.0 + 3 * 2.0 ** -8]))
    assert hi[0] == 1.0 + 2.0 ** -6 and lo[0] == -(2.0 ** -8)


def test_split_x3_error_bound_is_sharp():
    # x in [2^e, 2^(e+1)): |x32 - hi| < 2^(e-8) (half an ulp of hi), so the
    # remainder's leading exponent is at most e - 9 and lo is within half its
    # ulp, 2^(e-9-8): |x - hi - lo| <= (2^-24 + 2^-17) |x|, reached to within
    # a factor of 2 (the split keeps about 17 bits, not 24)
    rng = np.random.default_rng(11)
    x = rng.standard_normal(200000) * 2.0 ** rng.integers(-30, 30, 200000)
    hi, lo = split_x3(x)
    rel = np.abs(x - hi - lo) / np.abs(x)
    assert rel.max() <= 2.0 ** -24 + 2.0 ** -17
    assert rel.max() >= 2.0 ** -18


def test_gemm_x3_drops_exactly_the_lo_lo_term():
    # a = b = 1 + 2^-10 split exactly as hi = 1, lo = 2^-10: the exact
    # product is 1 + 2^-9 + 2^-20, the three-pass sum misses lo lo = 2^-20
    a = np.array([[1.0 + 2.0 ** -10]])
    assert gemm_x3(a, a)[0, 0] == 1.0 + 2.0 ** -9
    assert (a @ a)[0, 0] == 1.0 + 2.0 ** -9 + 2.0 ** -20
    # inner dimension: sums of such terms, with signs
    A = np.array([[1.0 + 2.0 ** -10, -(1.0 + 2.0 ** -10), 2.0]])
    B = np.array([[1.0 + 2.0 ** -10], [1.0 - 2.0 ** -10], [3.0]])
    # (1 + e)^2 - lo lo, -(1 + e)(1 - e) - (lo (-lo)), 6 with e = 2^-10
    assert gemm_x3(A, B)[0, 0] == (1 + 2.0 ** -9) - (1 - 2.0 ** -20) - 2.0 ** -20 + 6.0


def test_gemm_x3_error_bound():
    # per term, with r = x - hi - lo (<= 2^-17 (1 + 2^-7) |x|) and
    # |lo| <= 2^-8 (1 + 2^-8) |x|: ab - x3(a, b) = a r_b + r_a b - r_a r_b
    # + lo_a lo_b, at most 2^-15 (1 + 2^-6) |a| |b|
    rng = np.random.default_rng(12)
    A = rng.standard_normal((40, 300)) * 2.0 ** rng.integers(-8, 8, (40, 300))
    B = rng.standard_normal((300, 30))
    err = np.abs(gemm_x3(A, B) - A @ B)
    scale = np.abs(A) @ np.abs(B)
    bound = (2.0 ** -15 * (1 + 2.0 ** -6) + 1e-15) * scale
    assert np.all(err <= bound)
    # far from binary64 exactness, and far better than one bfloat16 pass
    assert np.max(err / scale) > 2.0 ** -26
    one_pass = np.abs(split_x3(A)[0] @ split_x3(B)[0] - A @ B)
    assert np.max(one_pass / scale) > 2.0 ** 6 * np.max(err / scale)


def test_fp32_x3_bound_covers_binary32_sums():
    # the 3K exact terms summed in binary32 in a random order
    rng = np.random.default_rng(13)
    for K in (8, 500, 4000):
        A = rng.standard_normal((5, K))
        B = rng.standard_normal((K, 4))
        Ah, Al = split_x3(A)
        Bh, Bl = split_x3(B)
        ref = gemm_x3(A, B)
        bound = fp32_x3_bound(A, B)
        for i in range(5):
            for j in range(4):
                terms = np.concatenate([Ah[i] * Bh[:, j], Ah[i] * Bl[:, j], Al[i] * Bh[:, j]])
                s = np.float32(0.0)
                for t in rng.permutation(terms).astype(np.float32):
                    s = np.float32(s + t)
                assert abs(float(s) - ref[i, j]) <= bound[i, j]
        assert np.max(bound / (np.abs(A) @ np.abs(B))) < 1e-3


# --------------------------------------------------------- x6 split product
def test_split_x6_matches_torch_roundings():
    # hi, mid and lo are torch's bfloat16 roundings of the binary32 value and
    # of the successive (exact) binary32 remainders
    rng = np.random.default_rng(20)
    x = np.concatenate([rng.standard_normal(20000),
                        rng.standard_normal(5000) * 2.0 ** rng.integers(-100, 100, 5000)])
    hi, mid, lo = split_x6(x)
    x32 = torch.from_numpy(x).to(torch.float32)
    hi_t = x32.to(torch.bfloat16).to(torch.float32)
    mid_t = (x32 - hi_t).to(torch.bfloat16).to(torch.float32)
    lo_t = (x32 - hi_t - mid_t).to(torch.bfloat16).to(torch.float32)
    np.testing.assert_array_equal(hi, hi_t.to(torch.float64).numpy())
    np.testing.assert_array_equal(mid, mid_t.to(torch.float64).numpy())
    np.testing.assert_array_equal(lo, lo_t.to(torch.float64).numpy())


def test_split_x6_is_exact_on_binary32():
    # three 8-bit parts hold the 24 bits of x32 (normal range): the split of
    # the binary32 value loses nothing, only the rounding to binary32 does
    rng = np.random.default_rng(21)
    x = rng.standard_normal(200000) * 2.0 ** rng.integers(-60, 60, 200000)
    hi, mid, lo = split_x6(x)
    x32 = x.astype(np.float32).astype(np.float64)
    np.testing.assert_array_equal(hi + mid + lo, x32)
    rel = np.abs(x - hi - mid - lo) / np.abs(x)
    assert rel.max() <= 2.0 ** -24 and rel.max() >= 2.0 ** -25
    # mid within half an ulp of hi, lo within half an ulp of mid
    assert np.all(np.abs(mid) <= 2.0 ** -8 * np.abs(hi))
    assert np.all(np.abs(lo) <= 2.0 ** -8 * np.abs(mid) + 1e-300)


def test_split_x6_hand_case_and_dropped_terms():
    # a = 1 + 2^-9 + 2^-18 splits as hi = 1, mid = 2^-9, lo = 2^-18; a a keeps
    # hh + hm + mh + hl + lh + mm = 1 + 2^-8 + 2^-17 + 2^-18 and drops
    # ml + lm + ll = 2^-26 + 2^-36
    a = np.array([[1.0 + 2.0 ** -9 + 2.0 ** -18]])
    hi, mid, lo = split_x6(a)
    assert hi[0, 0] == 1.0 and mid[0, 0] == 2.0 ** -9 and lo[0, 0] == 2.0 ** -18
    assert gemm_x6(a, a)[0, 0] == 1.0 + 2.0 ** -8 + 2.0 ** -17 + 2.0 ** -18
    assert (a @ a)[0, 0] - gemm_x6(a, a)[0, 0] == 2.0 ** -26 + 2.0 ** -36


def test_gemm_x6_error_bound():
    # per term ab - x6(a, b) = a r_b + r_a b - r_a r_b + (ml + lm + ll) with
    # r = x - x32 (<= 2^-24 |x|) and |mid| <= 2^-8 |x|, |lo| <= 2^-16 |x|:
    # at most about 2^-22 |a| |b|; far below the x3 product's 2^-15
    rng = np.random.default_rng(22)
    A = rng.standard_normal((40, 300)) * 2.0 ** rng.integers(-8, 8, (40, 300))
    B = rng.standard_normal((300, 30))
    err = np.abs(gemm_x6(A, B) - A @ B)
    scale = np.abs(A) @ np.abs(B)
    assert np.all(err <= 2.0 ** -22 * scale)
    err3 = np.abs(gemm_x3(A, B) - A @ B)
    assert np.max(err3 / scale) > 2.0 ** 6 * np.max(err / scale)


def test_fp32_x6_bound_covers_sliced_binary32_sums():
    # per K slice of 32 the 192 exact terms summed in binary32 in a random
    # order, the slice sums added in binary64
    rng = np.random.default_rng(23)
    for K in (8, 100, 3000):
        A = rng.standard_normal((4, K))
        B = rng.standard_normal((K, 3))
        Ah, Am, Al = split_x6(A)
        Bh, Bm, Bl = split_x6(B)
        ref = gemm_x6(A, B)
        bound = fp32_x6_bound(A, B)
        for i in range(4):
            for j in range(3):
                total = 0.0
                for k0 in range(0, K, 32):
                    sl = slice(k0, min(k0 + 32, K))
                    terms = np.concatenate([Ah[i, sl] * Bh[sl, j], Ah[i, sl] * Bm[sl, j],
                                            Am[i, sl] * Bh[sl, j], Ah[i, sl] * Bl[sl, j],
                                            Al[i, sl] * Bh[sl, j], Am[i, sl] * Bm[sl, j]])
                    s = np.float32(0.0)
                    for t in rng.permutation(terms).astype(np.float32):
                        s = np.float32(s + t)
                    total += float(s)
                assert abs(total - ref[i, j]) <= bound[i, j]
        # the slice bound does not grow with K
        assert np.max(bound / (np.abs(A) @ np.abs(B))) < 2e-5
