"""ctypes loader for librrf.so and the C prototypes of include/rrf.h.

The library is built in-tree by ``paper_2106_13402_amd.build``; importing
this module never builds or falls back to anything: a missing library is an
ImportError.
"""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "librrf.so")

RRF_OK = 0
RRF_E_HIP = 1
RRF_E_NOMEM = 2
RRF_E_NOTSUP = 3
RRF_E_NUMERIC = 4
RRF_E_INTERNAL = 5
RRF_PREC_FP64 = 0
RRF_PREC_BF16_SKETCH = 1
RRF_PREC_BF16_X3 = 2
RRF_PREC_BF16_X6 = 3
RRF_ALG_RANDUTV = 0
RRF_ALG_POWERURV = 1


class rrf_opts(C.Structure):
    _fields_ = [
        ("precision", C.c_int),
        ("stream", C.c_void_p),
        ("workspace", C.c_void_p),
        ("workspace_bytes", C.c_size_t),
        ("async_", C.c_int),
        ("check_finite", C.c_int),
        ("thin_u", C.c_int),
        ("no_replay", C.c_int),
    ]


class rrf_batched_cfg(C.Structure):
    _fields_ = [
        ("b", C.c_int64),
        ("tile_mask", C.c_int),
        ("leaf", C.c_int),
        ("tuned", C.c_int),
    ]


class rrf_trace_entry(C.Structure):
    _fields_ = [
        ("name", C.c_char * 48),
        ("launches", C.c_int64),
        ("ms", C.c_double),
        ("flops", C.c_double),
        ("bytes", C.c_double),
    ]


_i64, _i32, _u64, _dp, _vp, _sz, _d = (C.c_int64, C.c_int32, C.c_uint64, C.c_void_p,
                                       C.c_void_p, C.c_size_t, C.c_double)

# name -> (restype, argtypes); every symbol declared in include/rrf.h
PROTOTYPES = {
    "rrf_opts_init": (None, [C.POINTER(rrf_opts)]),
    "rrf_randutv": (C.c_int, [_i64, _i64, _dp, _i64, _i64, _i32, _u64, _dp, _dp, _dp]),
    "rrf_randutv_ex": (C.c_int, [_i64, _i64, _dp, _i64, _i64, _i32, _u64, _dp, _dp, _dp,
                                 C.POINTER(rrf_opts)]),
    "rrf_randutv_noalloc": (C.c_int, [_i64, _i64, _dp, _i64, _i64, _i32, _u64, _dp, _dp, _dp,
                                      C.POINTER(rrf_opts)]),
    "rrf_powerurv": (C.c_int, [_i64, _i64, _dp, _i64, _i64, _i32, _u64, _dp, _dp, _dp]),
    "rrf_powerurv_ex": (C.c_int, [_i64, _i64, _dp, _i64, _i64, _i32, _u64, _dp, _dp, _dp,
                                  C.POINTER(rrf_opts)]),
    "rrf_workspace_size": (_sz, [C.c_int, _i64, _i64, _i64, _i32, C.c_int]),
    "rrf_randutv_batched": (C.c_int, [_i64, _vp, _vp, _vp, _vp, _i64, _i32, _u64, _vp, _vp, _vp,
                                      C.POINTER(rrf_opts)]),
    "rrf_randutv_batched_workspace_size": (_sz, [_i64, _vp, _vp, _i64, C.c_int]),
    "rrf_randutv_batched_block": (_i64, [_i64, _i64]),
    "rrf_batched_autotune": (C.c_int, [C.c_int, _i32, _i64, _vp, _vp, _i64, _u64, C.c_char_p,
                                       C.POINTER(rrf_opts)]),
    "rrf_batched_tune_load": (C.c_int, [C.c_char_p]),
    "rrf_batched_config": (C.c_int, [_i64, _i64, C.c_int, C.POINTER(rrf_batched_cfg)]),
    "rrf_randutv_resume": (C.c_int, [_i64, _i64, _i64, _i32, _u64, _d, _i64, _i64, _dp, _dp, _dp,
                                     C.POINTER(C.c_int64), C.POINTER(rrf_opts)]),
    "rrf_rsvd": (C.c_int, [_i64, _i64, _dp, _i64, _i64, _i32, _u64, _dp, _dp, _dp,
                           C.POINTER(rrf_opts)]),
    "rrf_rsvd_workspace_size": (_sz, [_i64, _i64, _i64, _i32]),
    "rrf_randutv_partial": (C.c_int, [_i64, _i64, _dp, _i64, _i64, _i32, _u64, _d, _i64, _dp, _dp,
                                      _dp, C.POINTER(C.c_int64), C.POINTER(rrf_opts)]),
    "rrf_randutv_boosted_ex": (C.c_int, [_i64, _i64, _dp, _i64, _i64, _i32, _i64, _u64, _dp, _dp,
                                         _dp, C.POINTER(rrf_opts)]),
    "rrf_randutv_boosted": (C.c_int, [_i64, _i64, _dp, _i64, _i64, _i32, _i64, _u64, _dp, _dp,
                                      _dp]),
    "rrf_randutv_boosted_workspace_size": (_sz, [_i64, _i64, _i64, _i32, _i64]),
    "rrf_release_workspace": (C.c_int, []),
    "rrf_gaussian": (C.c_int, [_u64, _u64, _i64, _i64, _dp, _i64, _vp]),
    "rrf_sketch_uniforms": (C.c_int, [_u64, _u64, _i64, _i64, _dp, _i64, _vp]),
    "rrf_dgemm": (C.c_int, [C.c_int, C.c_int, _i64, _i64, _i64, _d, _dp, _i64, _dp, _i64, _d,
                            _dp, _i64, _vp, _sz, _vp]),
    "rrf_gemm_x3": (C.c_int, [C.c_int, C.c_int, _i64, _i64, _i64, _d, _dp, _i64, _dp, _i64, _d,
                              _dp, _i64, _vp, _sz, _vp]),
    "rrf_gemm_x6": (C.c_int, [C.c_int, C.c_int, _i64, _i64, _i64, _d, _dp, _i64, _dp, _i64, _d,
                              _dp, _i64, _vp, _sz, _vp]),
    "rrf_panel_workspace_size": (_sz, [_i64, _i64]),
    "rrf_householder_panel": (C.c_int, [_i64, _i64, _dp, _i64, _dp, _i64, _dp, _i64, _dp, _i64,
                                        _dp, _vp, _sz, _vp]),
    "rrf_block_svd_workspace_size": (_sz, [_i64]),
    "rrf_block_svd": (C.c_int, [_i64, _dp, _i64, _dp, _dp, _dp, _vp, _sz, _vp]),
    "rrf_to_bf16": (C.c_int, [_i64, _i64, _dp, _i64, C.c_int, _vp, _i64, _vp, _i64, _vp, _sz,
                              _vp]),
    "rrf_gemm_bf16_workspace_size": (_sz, [_i64, _i64]),
    "rrf_gemm_bf16_tn": (C.c_int, [_i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _dp, _i64,
                                   _vp, _sz, _vp]),
    "rrf_trace_enable": (C.c_int, [C.c_int]),
    "rrf_trace_enable_class": (C.c_int, [C.c_char_p]),
    "rrf_trace_read": (C.c_int, [C.POINTER(rrf_trace_entry), C.c_int]),
    "rrf_status_string": (C.c_char_p, [C.c_int]),
    "rrf_last_error": (C.c_char_p, []),
}


def load(path: str = LIB_PATH) -> C.CDLL:
    # torch wheels bundle their own HIP runtime under the same SONAME
    # (libamdhip64.so.7) but a different file name. Loading torch first makes
    # librrf bind to that same runtime instead of mapping a second one from
    # /opt/rocm, which would leave two HIP runtimes in one process.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it with `python paper_2106_13402_amd/build.py` "
            "(hipcc, gfx950). There is no fallback implementation.")
    lib = C.CDLL(path)
    for name, (res, args) in PROTOTYPES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


class RRFError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status} ({detail})")
        self.status = status
