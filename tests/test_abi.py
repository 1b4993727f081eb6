"""C-ABI checks that need no GPU: the library loads, exports every symbol
include/rrf.h declares, and rejects invalid arguments (LAPACK-style -k)
before touching the device."""
import ctypes as C
import os
import re

import pytest

from paper_2106_13402_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def _declared():
    text = open(os.path.join(ROOT, "include", "rrf.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rrf_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("rrf_randutv", "rrf_powerurv", "rrf_randutv_ex", "rrf_powerurv_ex",
                 "rrf_workspace_size", "rrf_status_string", "rrf_last_error"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert missing == []
    # and the binding's prototype table covers them all
    assert sorted(_lib.PROTOTYPES) == _declared()


NULL = None
DUMMY = C.c_void_p(0x1000)  # never dereferenced: validation fails first


@pytest.mark.parametrize("args,code", [
    ((0, 1, DUMMY, 1, 1, 0), -1),        # m < 1
    ((4, 0, DUMMY, 4, 1, 0), -2),        # n < 1
    ((4, 4, NULL, 4, 1, 0), -3),         # A NULL
    ((4, 4, DUMMY, 3, 1, 0), -4),        # lda < m
    ((4, 4, DUMMY, 4, 0, 0), -5),        # b < 1
    ((4, 4, DUMMY, 4, 2, -1), -6),       # q < 0
])
@pytest.mark.parametrize("fn", ["rrf_randutv", "rrf_powerurv"])
def test_argument_errors(lib, fn, args, code):
    m, n, A, lda, b, q = args
    st = getattr(lib, fn)(m, n, A, lda, b, q, 1, NULL, DUMMY, NULL)
    assert st == code
    assert lib.rrf_last_error()


@pytest.mark.parametrize("fn", ["rrf_randutv", "rrf_powerurv"])
def test_null_T_and_wide_input(lib, fn):
    assert getattr(lib, fn)(4, 4, DUMMY, 4, 2, 0, 1, NULL, NULL, NULL) == -9
    # a wide A goes through its transpose; arguments are still checked
    assert getattr(lib, fn)(3, 5, DUMMY, 3, 2, 0, 1, NULL, NULL, NULL) == -9
    assert getattr(lib, fn)(3, 5, DUMMY, 2, 2, 0, 1, NULL, DUMMY, NULL) == -4
    assert getattr(lib, fn)(3, 5, DUMMY, 3, 2, -1, 1, NULL, DUMMY, NULL) == -6


def test_alias_requires_tight_lda(lib):
    assert lib.rrf_randutv(4, 4, DUMMY, 6, 2, 0, 1, NULL, DUMMY, NULL) == -4


def test_workspace_size(lib):
    f = lib.rrf_workspace_size
    assert f(_lib.RRF_ALG_RANDUTV, 512, 512, 32, 1, 0) > 0
    assert f(_lib.RRF_ALG_POWERURV, 512, 512, 32, 1, 0) > 0
    # powerURV's mixed mode adds bfloat16 copies of A (both layouts), V and
    # V_hat and the bfloat16 GEMM's partial sums; q = 0 has no power products
    pw = f(_lib.RRF_ALG_POWERURV, 512, 512, 32, 1, 0)
    pm = f(_lib.RRF_ALG_POWERURV, 512, 512, 32, 1, 1)
    assert pw + 4 * 2 * 512 * 512 <= pm <= pw + 4 * 2 * 512 * 512 + 16 * 4 * 512 * 512 + 2 ** 20
    assert f(_lib.RRF_ALG_POWERURV, 512, 512, 32, 0, 1) == f(_lib.RRF_ALG_POWERURV, 512, 512, 32, 0, 0)
    assert f(_lib.RRF_ALG_POWERURV, 512, 512, 32, 1, 2) == 0
    # m < n: the factorization of the transpose plus A^T and T^T
    assert f(_lib.RRF_ALG_RANDUTV, 512, 600, 32, 1, 0) == (
        f(_lib.RRF_ALG_RANDUTV, 600, 512, 32, 1, 0) + 2 * 512 * 600 * 8)
    for prec in (0, 1):
        wide, tall = (f(_lib.RRF_ALG_POWERURV, 512, 600, 32, 1, prec),
                      f(_lib.RRF_ALG_POWERURV, 600, 512, 32, 1, prec))
        assert tall + 2 * 512 * 600 * 8 <= wide < tall + 2 * 512 * 600 * 8 + 256
    assert f(_lib.RRF_ALG_POWERURV, 512, 600, 32, 1, _lib.RRF_PREC_BF16_X3) == 0
    assert f(_lib.RRF_ALG_RANDUTV, 512, 512, 300, 1, 0) == 0    # b > 256
    assert f(7, 512, 512, 32, 1, 0) == 0
    # the reflectors of every step are kept (m x n for U, n x n for V) so that
    # U and V can be formed backward after the loop; the rest is O(max(m,n) b)
    n = 16384
    big = f(_lib.RRF_ALG_RANDUTV, n, n, 128, 2, 0)
    assert 8 * 2 * n * n < big < 8 * 2 * n * n + 2 ** 31
    mixed = f(_lib.RRF_ALG_RANDUTV, n, n, 128, 2, 1)
    assert big < mixed < big + 2 * 2 * n * n + 2 ** 30  # + two bfloat16 copies of T22
    # the x3 updates need no buffers beyond the bfloat16 sketch's
    assert f(_lib.RRF_ALG_RANDUTV, n, n, 128, 2, _lib.RRF_PREC_BF16_X3) == mixed
    # powerURV has no x3 mode
    assert f(_lib.RRF_ALG_POWERURV, n, n, 128, 2, _lib.RRF_PREC_BF16_X3) == 0


def test_panel_workspace_size(lib):
    """rrf_panel_workspace_size(M, k) covers every panel height up to M, so it
    never shrinks as M grows (also across the 1024 rows from which panels of
    16 to 128 columns take CholeskyQR2); from there on it holds the CholeskyQR
    buffers: the status and flag words, the M x k orthonormal factor and six
    k x k matrices. Unsupported shapes give 0."""
    f = lib.rrf_panel_workspace_size
    for k in (1, 16, 33, 64, 100, 128, 200, 256):
        prev = 0
        for M in (k, 300, 1000, 1023, 1024, 1025, 2048, 4096, 16384, 32768, 40000):
            if M < k:
                continue
            w = f(M, k)
            assert w > 0, (M, k)
            assert w >= prev, (M, k, w, prev)
            prev = w
            if 16 <= k <= 128 and M >= 1024:
                assert w >= 256 + 256 + 8 * M * k + 6 * 8 * k * k, (M, k, w)
    assert f(100, 101) == 0       # M < k
    assert f(4096, 257) == 0      # k > 256
    assert f(4096, 0) == 0


def test_component_argument_errors(lib):
    assert lib.rrf_dgemm(2, 0, 1, 1, 1, 1.0, DUMMY, 1, DUMMY, 1, 0.0, DUMMY, 1, NULL, 0, NULL) == -1
    assert lib.rrf_dgemm(0, 0, 4, 4, 4, 1.0, DUMMY, 3, DUMMY, 4, 0.0, DUMMY, 4, NULL, 0, NULL) == -8
    assert lib.rrf_gemm_x3(0, 3, 1, 1, 1, 1.0, DUMMY, 1, DUMMY, 1, 0.0, DUMMY, 1, NULL, 0, NULL) == -2
    assert lib.rrf_gemm_x3(0, 1, 4, 4, 4, 1.0, DUMMY, 4, DUMMY, 3, 0.0, DUMMY, 4, NULL, 0, NULL) == -10
    assert lib.rrf_gemm_x3(0, 0, 4, 4, 4, 1.0, DUMMY, 4, DUMMY, 4, 0.0, DUMMY, 3, NULL, 0, NULL) == -13
    assert lib.rrf_householder_panel(3, 4, DUMMY, 3, DUMMY, 3, NULL, 4, DUMMY, 4, DUMMY, NULL, 0,
                                     NULL) == -1
    assert lib.rrf_block_svd(0, DUMMY, 1, DUMMY, DUMMY, DUMMY, NULL, 0, NULL) == -1
    assert lib.rrf_gaussian(1, 1, -1, 2, DUMMY, 1, NULL) == -3
    assert lib.rrf_panel_workspace_size(16384, 128) > 0
    assert lib.rrf_panel_workspace_size(10, 20) == 0


def test_status_strings(lib):
    for code in range(0, 6):
        assert lib.rrf_status_string(code)
    assert b"invalid" in lib.rrf_status_string(-3)


def test_opts_init(lib):
    o = _lib.rrf_opts()
    o.precision = 9
    o.async_ = 1
    lib.rrf_opts_init(C.byref(o))
    assert o.precision == 0 and o.async_ == 0 and o.workspace is None


def test_x3_mode_is_randutv_only(lib):
    # rejected before any device work: powerURV and the batched call have no
    # x3 updates
    o = _lib.rrf_opts()
    lib.rrf_opts_init(C.byref(o))
    o.precision = _lib.RRF_PREC_BF16_X3
    assert lib.rrf_powerurv_ex(8, 8, DUMMY, 8, 4, 1, 1, NULL, DUMMY, NULL,
                               C.byref(o)) == _lib.RRF_E_NOTSUP
    m = (C.c_int64 * 1)(8)
    A = (C.c_void_p * 1)(0x1000)
    T = (C.c_void_p * 1)(0x3000)
    assert lib.rrf_randutv_batched(1, m, m, A, m, 4, 1, 1, NULL, T, NULL,
                                   C.byref(o)) == _lib.RRF_E_NOTSUP
    assert lib.rrf_randutv_batched_workspace_size(1, m, m, 4, _lib.RRF_PREC_BF16_X3) == 0


def test_boosted_argument_errors(lib):
    f = lib.rrf_randutv_boosted
    assert f(8, 8, DUMMY, 8, 4, 1, -1, 1, NULL, DUMMY, NULL) == -7
    assert f(8, 8, DUMMY, 8, 4, -1, 2, 1, NULL, DUMMY, NULL) == -6
    assert f(8, 8, DUMMY, 8, 4, 1, 2, 1, NULL, NULL, NULL) == -10
    # m < n goes through the transpose: arguments checked, b + p against m
    assert f(8, 9, DUMMY, 7, 4, 1, 2, 1, NULL, DUMMY, NULL) == -4
    assert f(8, 9, DUMMY, 8, 4, 1, 2, 1, NULL, NULL, NULL) == -10
    assert f(300, 400, DUMMY, 300, 200, 1, 100, 1, NULL, DUMMY, NULL) == _lib.RRF_E_NOTSUP
    assert f(400, 300, DUMMY, 400, 200, 1, 100, 1, NULL, DUMMY, NULL) == _lib.RRF_E_NOTSUP
    o = _lib.rrf_opts()
    lib.rrf_opts_init(C.byref(o))
    o.precision = _lib.RRF_PREC_BF16_SKETCH
    assert lib.rrf_randutv_boosted_ex(8, 8, DUMMY, 8, 4, 1, 2, 1, NULL, DUMMY, NULL,
                                      C.byref(o)) == _lib.RRF_E_NOTSUP
    ws = lib.rrf_randutv_boosted_workspace_size
    assert ws(16384, 16384, 128, 2, 128) > lib.rrf_workspace_size(0, 16384, 16384, 128, 2, 0)
    assert ws(100, 50, 16, 1, 300) > 0  # p is clipped to n - b
    assert ws(1000, 500, 200, 1, 100) == 0 and ws(500, 1000, 200, 1, 100) == 0
    assert ws(10, 8, 4, 1, -1) == 0
    assert ws(10, 20, 4, 1, 2) >= ws(20, 10, 4, 1, 2) + 2 * 10 * 20 * 8  # + A^T and T^T


def test_partial_argument_errors(lib):
    f = lib.rrf_randutv_partial
    k = C.c_int64(7)
    assert f(8, 8, DUMMY, 8, 4, 1, 1, -1.0, 8, NULL, DUMMY, NULL, C.byref(k), NULL) == -8
    assert f(8, 8, DUMMY, 8, 4, 1, 1, float("nan"), 8, NULL, DUMMY, NULL, C.byref(k), NULL) == -8
    assert f(8, 8, DUMMY, 8, 4, 1, 1, 1e-3, -1, NULL, DUMMY, NULL, C.byref(k), NULL) == -9
    assert f(8, 8, DUMMY, 8, 4, 1, 1, 1e-3, 8, NULL, DUMMY, NULL, None, NULL) == -13
    assert f(8, 8, DUMMY, 8, 4, 1, 1, 1e-3, 8, NULL, NULL, NULL, C.byref(k), NULL) == -11
    assert f(8, 8, DUMMY, 7, 4, 1, 1, 1e-3, 8, NULL, DUMMY, NULL, C.byref(k), NULL) == -4
    # m < n goes through the transpose; its arguments are checked the same way
    assert f(6, 9, DUMMY, 5, 4, 1, 1, 1e-3, 8, NULL, DUMMY, NULL, C.byref(k), NULL) == -4
    assert f(6, 9, DUMMY, 6, 4, 1, 1, 1e-3, 8, NULL, NULL, NULL, C.byref(k), NULL) == -11


def test_rsvd_argument_errors(lib):
    f = lib.rrf_rsvd
    assert f(0, 8, DUMMY, 8, 4, 1, 1, NULL, DUMMY, NULL, NULL) == -1
    assert f(8, 8, DUMMY, 7, 4, 1, 1, NULL, DUMMY, NULL, NULL) == -4
    assert f(8, 6, DUMMY, 8, 7, 1, 1, NULL, DUMMY, NULL, NULL) == -5
    assert f(8, 6, DUMMY, 8, 0, 1, 1, NULL, DUMMY, NULL, NULL) == -5
    assert f(8, 6, DUMMY, 8, 4, -1, 1, NULL, DUMMY, NULL, NULL) == -6
    assert f(8, 6, DUMMY, 8, 4, 1, 1, NULL, NULL, NULL, NULL) == -9
    assert f(600, 600, DUMMY, 600, 300, 1, 1, NULL, DUMMY, NULL, NULL) == _lib.RRF_E_NOTSUP
    ws = lib.rrf_rsvd_workspace_size
    assert ws(1000, 500, 64, 1) > 0 and ws(500, 1000, 64, 1) > 0
    assert ws(100, 50, 60, 1) == 0 and ws(1000, 1000, 300, 1) == 0


def test_resume_argument_errors(lib):
    f = lib.rrf_randutv_resume
    k = C.c_int64(7)
    assert f(8, 8, 0, 1, 1, 1e-3, 8, 0, NULL, DUMMY, NULL, C.byref(k), NULL) == -3
    assert f(8, 8, 4, 1, 1, -1.0, 8, 0, NULL, DUMMY, NULL, C.byref(k), NULL) == -6
    assert f(8, 8, 4, 1, 1, 1e-3, 8, 3, NULL, DUMMY, NULL, C.byref(k), NULL) == -8
    assert f(8, 8, 4, 1, 1, 1e-3, 8, 12, NULL, DUMMY, NULL, C.byref(k), NULL) == -8
    assert f(8, 8, 4, 1, 1, 1e-3, 8, 4, NULL, NULL, NULL, C.byref(k), NULL) == -10
    assert f(8, 8, 4, 1, 1, 1e-3, 8, 4, NULL, DUMMY, NULL, None, NULL) == -12
    # everything already reduced: nothing to do, k unchanged
    assert f(8, 8, 4, 1, 1, 1e-3, 8, 8, NULL, DUMMY, NULL, C.byref(k), NULL) == 0 and k.value == 8
    # m < n: k_in counts the transpose's columns, at most min(m, n)
    assert f(6, 9, 4, 1, 1, 1e-3, 8, 8, NULL, DUMMY, NULL, C.byref(k), NULL) == -8
    assert f(6, 9, 4, 1, 1, 1e-3, 8, 6, NULL, DUMMY, NULL, C.byref(k), NULL) == 0 and k.value == 6


def _arr(t, vals):
    return (t * len(vals))(*vals)


def test_batched_argument_errors(lib):
    f = lib.rrf_randutv_batched
    m, n, lda = _arr(C.c_int64, [8, 6]), _arr(C.c_int64, [6, 6]), _arr(C.c_int64, [8, 6])
    A = _arr(C.c_void_p, [0x1000, 0x2000])
    T = _arr(C.c_void_p, [0x3000, 0x4000])
    assert f(-1, m, n, A, lda, 4, 1, 1, NULL, T, NULL, NULL) == -1
    assert f(0, NULL, NULL, NULL, NULL, 4, 1, 1, NULL, NULL, NULL, NULL) == 0  # nothing to do
    assert f(2, NULL, n, A, lda, 4, 1, 1, NULL, T, NULL, NULL) == -2
    assert f(2, m, n, A, lda, 65, 1, 1, NULL, T, NULL, NULL) == -6
    assert f(2, m, n, A, lda, -1, 1, 1, NULL, T, NULL, NULL) == -6
    assert f(2, m, n, A, lda, 4, -1, 1, NULL, T, NULL, NULL) == -7
    assert f(2, m, n, A, lda, 4, 1, 1, NULL, NULL, NULL, NULL) == -10
    bad_lda = _arr(C.c_int64, [8, 5])
    assert f(2, m, n, A, bad_lda, 4, 1, 1, NULL, T, NULL, NULL) == -5
    alias = _arr(C.c_void_p, [0x1000, 0x4000])
    assert f(2, m, n, A, _arr(C.c_int64, [9, 6]), 4, 1, 1, NULL, alias, NULL, NULL) == -5
    one_null = _arr(C.c_void_p, [0x5000, 0])
    assert f(2, m, n, A, lda, 4, 1, 1, one_null, T, NULL, NULL) == -9
    # a wide matrix goes through its transpose; its arguments are still checked
    wide = _arr(C.c_int64, [8, 7])
    assert f(2, m, wide, A, bad_lda, 4, 1, 1, NULL, T, NULL, NULL) == -5
    assert f(2, m, wide, A, lda, 4, 1, 1, one_null, T, NULL, NULL) == -9
    huge = _arr(C.c_int64, [8, 5000])
    assert f(2, huge, n, A, _arr(C.c_int64, [8, 5000]), 4, 1, 1, NULL, T, NULL,
             NULL) == _lib.RRF_E_NOTSUP


def test_batched_workspace_size(lib):
    f = lib.rrf_randutv_batched_workspace_size
    ms, ns = [100, 300, 512], [64, 200, 512]
    m, n = _arr(C.c_int64, ms), _arr(C.c_int64, ns)
    w16, w64, wauto = f(3, m, n, 16, 0), f(3, m, n, 64, 0), f(3, m, n, 0, 0)
    assert w16 > 0 and w64 > 0 and wauto > 0
    # at least the kept reflectors (m n + n^2 doubles per matrix), and the
    # automatic choice needs no more than the largest single group would
    refl = sum(8 * (a * c + c * c) for a, c in zip(ms, ns))
    assert refl < w16 and refl < w64
    assert wauto <= max(w16, w64)
    assert f(3, m, n, 65, 0) == 0
    # n > m: the transpose's arena plus the transposed copy (8 m n bytes, rounded)
    wn = f(3, m, _arr(C.c_int64, [64, 301, 512]), 16, 0)
    wt = f(3, _arr(C.c_int64, [100, 301, 512]), _arr(C.c_int64, [64, 300, 512]), 16, 0)
    assert wn >= 8 * 300 * 301 and wn > 0 and wt > 0
    assert f(1, _arr(C.c_int64, [4]), _arr(C.c_int64, [4097]), 16, 0) == 0
    assert f(1, _arr(C.c_int64, [4097]), _arr(C.c_int64, [4]), 16, 0) == 0
    assert f(2, m, n, 16, 0) < w16
    # the mixed sketch adds bfloat16 copies of T22 (both layouts), G, Y, Z and FP32 products
    wm = f(3, m, n, 16, 1)
    assert w16 + sum(4 * a * c for a, c in zip(ms, ns)) <= wm
    assert f(3, m, n, 16, 7) == 0


def test_batched_block_rule(lib):
    f = lib.rrf_randutv_batched_block
    assert f(100, 64) == 16 and f(512, 256) == 16 and f(300, 257) == 32 and f(1024, 512) == 32
    assert f(10, 11) == f(11, 10) == 16 and f(300, 600) == 32  # m < n: the transpose's rule
    assert f(5, 0) == 0 and f(0, 5) == 0


def test_trace_class_filter_arguments(lib):
    assert lib.rrf_trace_enable_class(None) == -1
    assert lib.rrf_trace_enable_class(b"no_such_kernel") == -1
    assert lib.rrf_trace_enable_class(b"dgemm_mfma_128x128_TN") == 0
    assert lib.rrf_trace_enable_class(b"dgemm_mfma_128x128_NN:UV") == 0
    assert lib.rrf_trace_enable(0) == 0


def test_noalloc_host_side_rejections(lib):
    """rrf_randutv_noalloc checks its arguments, a caller workspace and the
    static scratch limit before any device call."""
    f = lib.rrf_randutv_noalloc
    assert f(0, 4, DUMMY, 4, 2, 0, 1, NULL, DUMMY, NULL, None) == -1
    assert f(4, 4, DUMMY, 4, 2, -1, 1, NULL, DUMMY, NULL, None) == -6
    assert f(4, 4, DUMMY, 4, 2, 0, 1, NULL, NULL, NULL, None) == -9
    opts = _lib.rrf_opts()
    lib.rrf_opts_init(C.byref(opts))
    opts.workspace = 0x2000
    opts.workspace_bytes = 1 << 20
    assert f(64, 64, DUMMY, 64, 16, 1, 1, NULL, DUMMY, NULL, C.byref(opts)) == -11
    assert b"no workspace" in lib.rrf_last_error()
    # beyond the 64 MiB scratch: RRF_E_NOMEM with the sizes in the message
    limit = 64 << 20
    assert lib.rrf_workspace_size(_lib.RRF_ALG_RANDUTV, 4096, 4096, 128, 1, 0) > limit
    assert f(4096, 4096, DUMMY, 4096, 128, 1, 1, NULL, DUMMY, NULL, None) == _lib.RRF_E_NOMEM
    msg = lib.rrf_last_error()
    assert b"rrf_randutv_ex" in msg and str(limit).encode() in msg
    # the wide path is sized the same way (A^T's factorization plus A^T, T^T)
    assert f(1024, 4096, DUMMY, 1024, 128, 1, 1, NULL, DUMMY, NULL, None) == _lib.RRF_E_NOMEM
