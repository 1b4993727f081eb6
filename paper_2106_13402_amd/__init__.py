"""Randomized rank-revealing UTV factorizations on AMD MI355X (gfx950).

Python binding of librrf (include/rrf.h): argument marshalling only. Torch
supplies device memory and the current HIP stream; every step of the
factorizations runs in the library's HIP kernels. There is no CPU fallback:
without the built library the import fails.

Matrices are column-major float64 device tensors (``x.stride(0) == 1``);
``colmajor(x)`` makes such a copy of any 2-D tensor.
"""
from __future__ import annotations

import ctypes as C

from . import _lib
from ._lib import RRFError

__all__ = [
    "RRFError", "randutv", "randutv_noalloc", "randutv_boosted", "randutv_partial", "randutv_resume", "rsvd", "powerurv", "gaussian", "sketch_uniforms", "dgemm", "gemm_x3", "gemm_x6", "householder_panel",
    "block_svd", "workspace_size", "colmajor", "empty_colmajor", "lib", "trace_enable", "trace_enable_class",
    "trace_read", "to_bf16", "gemm_bf16_tn", "PRECISIONS", "randutv_batched",
    "batched_workspace_size", "batched_block", "batched_config", "batched_autotune",
    "batched_tune_load", "default_tune_path",
]

# precision names of rrf_opts.precision
PRECISIONS = {"fp64": _lib.RRF_PREC_FP64, "bf16_sketch": _lib.RRF_PREC_BF16_SKETCH,
              "bf16_x3": _lib.RRF_PREC_BF16_X3, "bf16_x6": _lib.RRF_PREC_BF16_X6}

lib = _lib.load()


def _check(status: int, where: str) -> None:
    if status != 0:
        detail = lib.rrf_last_error().decode(errors="replace")
        raise RRFError(status, where, detail)


def _torch():
    import torch
    return torch


def _stream_ptr(device) -> int:
    torch = _torch()
    return torch.cuda.current_stream(device).cuda_stream


def _require(x, name: str, rows: int | None = None):
    torch = _torch()
    if not isinstance(x, torch.Tensor) or x.dim() != 2:
        raise TypeError(f"{name}: expected a 2-D torch tensor")
    if x.dtype != torch.float64:
        raise TypeError(f"{name}: expected float64, got {x.dtype}")
    if not x.is_cuda:
        raise TypeError(f"{name}: expected a device (HIP) tensor")
    if x.shape[0] > 1 and x.stride(0) != 1:
        raise ValueError(f"{name}: expected column-major storage (stride(0) == 1); use colmajor()")
    if rows is not None and x.shape[0] != rows:
        raise ValueError(f"{name}: expected {rows} rows, got {x.shape[0]}")


def _ld(x) -> int:
    return max(int(x.stride(1)), int(x.shape[0]), 1) if x.shape[1] > 1 else max(int(x.shape[0]), 1)


def empty_colmajor(rows: int, cols: int, device, dtype=None):
    torch = _torch()
    return torch.empty((cols, rows), dtype=dtype or torch.float64, device=device).t()


def colmajor(x):
    """A column-major copy (or ``x`` itself if it already is one)."""
    if x.dim() == 2 and (x.shape[0] <= 1 or x.stride(0) == 1):
        return x
    return x.t().contiguous().t()


_WS = {}


def _workspace(device, nbytes: int):
    torch = _torch()
    key = (str(device),)
    buf = _WS.get(key)
    if buf is None or buf.numel() < nbytes:
        buf = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)
        _WS[key] = buf
    return buf


def workspace_size(alg: str, m: int, n: int, b: int, q: int, precision: str = "fp64") -> int:
    code = _lib.RRF_ALG_RANDUTV if alg == "randutv" else _lib.RRF_ALG_POWERURV
    return int(lib.rrf_workspace_size(code, m, n, b, q, PRECISIONS[precision]))


def _factor(fname: str, alg: str, A, b: int, q: int, seed: int, want_u: bool, want_v: bool,
            check_finite: bool, inplace: bool, precision: str = "fp64", p=None,
            thin_u: bool = False):
    _require(A, "A")
    m, n = int(A.shape[0]), int(A.shape[1])
    dev = A.device
    U = empty_colmajor(m, n if thin_u and m >= n else m, dev) if want_u else None
    V = empty_colmajor(n, n, dev) if want_v else None
    if inplace:
        if _ld(A) != m:
            raise ValueError("in-place factorization needs a tight A (lda == m)")
        T = A
    else:
        T = empty_colmajor(m, n, dev)
    if p is None:
        nbytes = workspace_size(alg, m, n, b, q, precision)
    else:
        nbytes = int(lib.rrf_randutv_boosted_workspace_size(m, n, b, q, p))
    if nbytes == 0:
        raise RRFError(_lib.RRF_E_NOTSUP, fname, "no workspace size for these arguments")
    ws = _workspace(dev, nbytes)
    opts = _lib.rrf_opts()
    lib.rrf_opts_init(C.byref(opts))
    opts.precision = PRECISIONS[precision]
    opts.stream = _stream_ptr(dev)
    opts.workspace = ws.data_ptr()
    opts.workspace_bytes = ws.numel()
    opts.async_ = 0
    opts.check_finite = 1 if check_finite else 0
    opts.thin_u = 1 if thin_u else 0
    fn = getattr(lib, fname)
    extra = () if p is None else (p,)
    st = fn(m, n, A.data_ptr(), _ld(A), b, q, *extra, seed,
            U.data_ptr() if U is not None else None, T.data_ptr(),
            V.data_ptr() if V is not None else None, C.byref(opts))
    _check(st, fname)
    return U, T, V


def randutv(A, b: int, q: int, seed: int, *, want_u: bool = True, want_v: bool = True,
            check_finite: bool = False, inplace: bool = False, precision: str = "fp64",
            thin_u: bool = False):
    """randUTV (Alg. 3): returns (U, T, V) with A = U T V^T (U/V None if not wanted).

    precision "bf16_sketch" forms each step's sketch from bfloat16 copies with
    FP32 accumulation (RRF_PREC_BF16_SKETCH); everything else stays FP64.
    "bf16_x3" adds the split-bfloat16 three-pass product to every update of
    T, U and V (RRF_PREC_BF16_X3; results accurate to about 1e-5).
    thin_u forms only U(:, :n) (m x n), all that A = U T V^T needs."""
    return _factor("rrf_randutv_ex", "randutv", A, b, q, seed, want_u, want_v, check_finite,
                   inplace, precision, thin_u=thin_u)


def randutv_noalloc(A, b: int, q: int, seed: int, *, want_u: bool = True, want_v: bool = True,
                    precision: str = "fp64", out=None):
    """randUTV through rrf_randutv_noalloc: the library works in its static
    device scratch and allocates nothing during the call. ``out`` = (U, T, V)
    preallocated column-major outputs (U/V may be None); allocated here when
    omitted. Returns (U, T, V)."""
    _require(A, "A")
    m, n = int(A.shape[0]), int(A.shape[1])
    dev = A.device
    if out is None:
        U = empty_colmajor(m, m, dev) if want_u else None
        T = empty_colmajor(m, n, dev)
        V = empty_colmajor(n, n, dev) if want_v else None
    else:
        U, T, V = out
    opts = _lib.rrf_opts()
    lib.rrf_opts_init(C.byref(opts))
    opts.precision = PRECISIONS[precision]
    opts.stream = _stream_ptr(dev)
    st = lib.rrf_randutv_noalloc(m, n, A.data_ptr(), _ld(A), b, q, seed,
                                 U.data_ptr() if U is not None else None, T.data_ptr(),
                                 V.data_ptr() if V is not None else None, C.byref(opts))
    _check(st, "rrf_randutv_noalloc")
    return U, T, V


def rsvd(A, l: int, q: int, seed: int, *, want_u: bool = True, want_v: bool = True,
         check_finite: bool = False):
    """Randomized SVD (Sec. 3.3): returns (U, S, V), U m x l, S (l,), V n x l
    (U/V None if not wanted), A ~ U diag(S) V^T."""
    torch = _torch()
    _require(A, "A")
    m, n = int(A.shape[0]), int(A.shape[1])
    dev = A.device
    U = empty_colmajor(m, l, dev) if want_u else None
    V = empty_colmajor(n, l, dev) if want_v else None
    S = torch.empty(l, dtype=torch.float64, device=dev)
    nbytes = int(lib.rrf_rsvd_workspace_size(m, n, l, q))
    if nbytes == 0:
        raise RRFError(_lib.RRF_E_NOTSUP, "rrf_rsvd", "no workspace size for these arguments")
    ws = _workspace(dev, nbytes)
    opts = _lib.rrf_opts()
    lib.rrf_opts_init(C.byref(opts))
    opts.stream = _stream_ptr(dev)
    opts.workspace = ws.data_ptr()
    opts.workspace_bytes = ws.numel()
    opts.check_finite = 1 if check_finite else 0
    _check(lib.rrf_rsvd(m, n, A.data_ptr(), _ld(A), l, q, seed,
                        U.data_ptr() if U is not None else None, S.data_ptr(),
                        V.data_ptr() if V is not None else None, C.byref(opts)), "rrf_rsvd")
    return U, S, V


def randutv_partial(A, b: int, q: int, seed: int, tol: float, kmax: int | None = None, *,
                    want_u: bool = True, want_v: bool = True, precision: str = "fp64"):
    """randUTV halted once ||T22||_F <= tol ||A||_F or kmax columns are
    reduced (Sec. 4.1); returns (U, T, V, k) with T(k:, k:) unreduced."""
    _require(A, "A")
    m, n = int(A.shape[0]), int(A.shape[1])
    dev = A.device
    U = empty_colmajor(m, m, dev) if want_u else None
    V = empty_colmajor(n, n, dev) if want_v else None
    T = empty_colmajor(m, n, dev)
    nbytes = workspace_size("randutv", m, n, b, q, precision)
    if nbytes == 0:
        raise RRFError(_lib.RRF_E_NOTSUP, "rrf_randutv_partial", "no workspace size")
    ws = _workspace(dev, nbytes)
    opts = _lib.rrf_opts()
    lib.rrf_opts_init(C.byref(opts))
    opts.precision = PRECISIONS[precision]
    opts.stream = _stream_ptr(dev)
    opts.workspace = ws.data_ptr()
    opts.workspace_bytes = ws.numel()
    k = C.c_int64(0)
    st = lib.rrf_randutv_partial(m, n, A.data_ptr(), _ld(A), b, q, seed, float(tol),
                                 n if kmax is None else int(kmax),
                                 U.data_ptr() if U is not None else None, T.data_ptr(),
                                 V.data_ptr() if V is not None else None, C.byref(k),
                                 C.byref(opts))
    _check(st, "rrf_randutv_partial")
    return U, T, V, int(k.value)


def randutv_resume(U, T, V, k: int, b: int, q: int, seed: int, tol: float,
                   kmax: int | None = None, precision: str = "fp64"):
    """Continue a randutv_partial result (U, T, V, k) in place with new
    stopping criteria; returns the new k."""
    _require(T, "T")
    m, n = int(T.shape[0]), int(T.shape[1])
    dev = T.device
    nbytes = workspace_size("randutv", m, n, b, q, precision)
    if nbytes == 0:
        raise RRFError(_lib.RRF_E_NOTSUP, "rrf_randutv_resume", "no workspace size")
    ws = _workspace(dev, nbytes)
    opts = _lib.rrf_opts()
    lib.rrf_opts_init(C.byref(opts))
    opts.precision = PRECISIONS[precision]
    opts.stream = _stream_ptr(dev)
    opts.workspace = ws.data_ptr()
    opts.workspace_bytes = ws.numel()
    kout = C.c_int64(0)
    _check(lib.rrf_randutv_resume(m, n, b, q, seed, float(tol), n if kmax is None else int(kmax),
                                  int(k), U.data_ptr() if U is not None else None, T.data_ptr(),
                                  V.data_ptr() if V is not None else None, C.byref(kout),
                                  C.byref(opts)), "rrf_randutv_resume")
    return int(kout.value)


def randutv_boosted(A, b: int, q: int, p: int, seed: int, *, want_u: bool = True,
                    want_v: bool = True, check_finite: bool = False, inplace: bool = False):
    """randUTV_boosted (Alg. 2): randUTV with b + p samples per step and the
    extra samples recycled into the next step; returns (U, T, V). FP64."""
    return _factor("rrf_randutv_boosted_ex", "randutv", A, b, q, seed, want_u, want_v,
                   check_finite, inplace, "fp64", p=int(p))


def _i64_array(vals):
    return (C.c_int64 * max(len(vals), 1))(*vals)


def _ptr_array(vals):
    return (C.c_void_p * max(len(vals), 1))(*vals)


def batched_block(m: int, n: int, precision: str = "fp64") -> int:
    """Block size the batched call uses for an m x n matrix when b = 0."""
    return batched_config(m, n, precision)["b"]


def batched_config(m: int, n: int, precision: str = "fp64") -> dict:
    """The configuration (b, tile_mask, leaf, tuned) the batched call uses for
    an m x n matrix when b = 0 (rrf_batched_config)."""
    cfg = _lib.rrf_batched_cfg()
    _check(lib.rrf_batched_config(m, n, PRECISIONS[precision], C.byref(cfg)), "rrf_batched_config")
    return {"b": int(cfg.b), "tile_mask": int(cfg.tile_mask), "leaf": int(cfg.leaf),
            "tuned": bool(cfg.tuned)}


def batched_autotune(precision: str = "fp64", q: int = 1, count: int = 256, nmax: int = 512,
                     seed: int = 0, path: str | None = None, shapes=None) -> None:
    """Run the batched call's autotuner on the current device
    (rrf_batched_autotune): on ``shapes`` (a list of (m, n)) when given, else
    on ``count`` synthetic matrices per size bucket. The table is loaded and,
    with ``path``, written."""
    torch = _torch()
    opts = _lib.rrf_opts()
    lib.rrf_opts_init(C.byref(opts))
    opts.stream = torch.cuda.current_stream().cuda_stream
    if shapes is not None:
        count = len(shapes)
        ms, ns = _i64_array([m for m, n in shapes]), _i64_array([n for m, n in shapes])
    else:
        ms = ns = None
    _check(lib.rrf_batched_autotune(PRECISIONS[precision], q, count, ms, ns, nmax, seed,
                                    path.encode() if path else None, C.byref(opts)),
           "rrf_batched_autotune")


def batched_tune_load(path: str | None) -> None:
    """Replace the loaded tuning tables by the cache file ``path`` (None:
    unload them; b = 0 then follows the built-in rule)."""
    _check(lib.rrf_batched_tune_load(path.encode() if path else None), "rrf_batched_tune_load")


def default_tune_path() -> str:
    """The cache the library loads by default (tuning/batched.json beside it)."""
    import os
    return os.path.join(os.path.dirname(_lib.LIB_PATH), "tuning", "batched.json")


def batched_workspace_size(ms, ns, b: int, precision: str = "fp64") -> int:
    """Bytes of workspace rrf_randutv_batched needs for these sizes (0: invalid)."""
    return int(lib.rrf_randutv_batched_workspace_size(len(ms), _i64_array(ms), _i64_array(ns), b,
                                                      PRECISIONS[precision]))


def randutv_batched(As, b: int, q: int, seed: int, *, want_u: bool = True, want_v: bool = True,
                    check_finite: bool = False, out=None, precision: str = "fp64",
                    replay: bool = True):
    """Batched randUTV (Alg. 3) of the matrices in the list ``As``; matrix j is
    keyed by ``seed + j``; ``b = 0`` picks the block size per matrix;
    precision "bf16_sketch" forms every step's sketch from bfloat16 copies.
    ``replay`` (default) records the call as HIP graphs on first use and
    replays them for later calls with the same shapes; False issues the
    lockstep rounds directly (rrf_opts.no_replay).

    Returns three lists (Us, Ts, Vs) (Us / Vs None when not wanted). ``out``
    may pass such lists (tight column-major tensors of the right shapes) to be
    written instead of new ones."""
    count = len(As)
    for j, A in enumerate(As):
        _require(A, f"As[{j}]")
    ms = [int(A.shape[0]) for A in As]
    ns = [int(A.shape[1]) for A in As]
    if count == 0:
        return ([] if want_u else None), [], ([] if want_v else None)
    dev = As[0].device
    if out is not None:
        Us, Ts, Vs = out
        for j in range(count):
            _require(Ts[j], f"Ts[{j}]", ms[j])
            if _ld(Ts[j]) != ms[j]:
                raise ValueError("outputs must be tight column-major tensors")
    else:
        Us = [empty_colmajor(m, m, dev) for m in ms] if want_u else None
        Ts = [empty_colmajor(m, n, dev) for m, n in zip(ms, ns)]
        Vs = [empty_colmajor(n, n, dev) for n in ns] if want_v else None
    nbytes = batched_workspace_size(ms, ns, b, precision)
    if nbytes == 0:
        raise RRFError(_lib.RRF_E_NOTSUP, "rrf_randutv_batched", "no workspace size for these sizes")
    ws = _workspace(dev, nbytes)
    opts = _lib.rrf_opts()
    lib.rrf_opts_init(C.byref(opts))
    opts.precision = PRECISIONS[precision]
    opts.stream = _stream_ptr(dev)
    opts.workspace = ws.data_ptr()
    opts.workspace_bytes = ws.numel()
    opts.check_finite = 1 if check_finite else 0
    opts.no_replay = 0 if replay else 1
    st = lib.rrf_randutv_batched(
        count, _i64_array(ms), _i64_array(ns), _ptr_array([A.data_ptr() for A in As]),
        _i64_array([_ld(A) for A in As]), b, q, seed,
        _ptr_array([U.data_ptr() for U in Us]) if Us is not None else None,
        _ptr_array([T.data_ptr() for T in Ts]),
        _ptr_array([V.data_ptr() for V in Vs]) if Vs is not None else None, C.byref(opts))
    _check(st, "rrf_randutv_batched")
    return Us, Ts, Vs


def powerurv(A, q: int, seed: int, *, b: int = 128, want_u: bool = True, want_v: bool = True,
             check_finite: bool = False, inplace: bool = False, precision: str = "fp64"):
    """powerURV (Alg. 1): returns (U, T, V); b is the QR panel width.

    precision "bf16_sketch" forms the 2q power products from bfloat16 values
    with FP32 accumulation (RRF_PREC_BF16_SKETCH); everything else stays FP64."""
    k = min(int(A.shape[0]), int(A.shape[1]))
    return _factor("rrf_powerurv_ex", "powerurv", A, min(b, max(k, 1)), q, seed, want_u, want_v,
                   check_finite, inplace, precision)


def gaussian(seed: int, stream_id: int, rows: int, cols: int, device="cuda"):
    """The rows x cols sketch Gaussian of (seed, stream) (column-major)."""
    out = empty_colmajor(rows, cols, device)
    _check(lib.rrf_gaussian(seed, stream_id, rows, cols, out.data_ptr() if out.numel() else None,
                            max(rows, 1), _stream_ptr(out.device)), "rrf_gaussian")
    return out


def sketch_uniforms(seed: int, stream_id: int, rows: int, cols: int, device="cuda"):
    """The uniforms behind gaussian(): row 4g + i holds uniform i
    (u_a, v_a, u_b, v_b) of counter (g, column)."""
    out = empty_colmajor(rows, cols, device)
    _check(lib.rrf_sketch_uniforms(seed, stream_id, rows, cols,
                                   out.data_ptr() if out.numel() else None, max(rows, 1),
                                   _stream_ptr(out.device)), "rrf_sketch_uniforms")
    return out


def dgemm(A, B, *, transa: bool = False, transb: bool = False, alpha: float = 1.0,
          beta: float = 0.0, C_out=None, split_work: bool = True):
    """C = alpha op(A) op(B) + beta C on the FP64 MFMA kernel."""
    return _gemm("rrf_dgemm", A, B, transa, transb, alpha, beta, C_out, split_work)


def gemm_x3(A, B, *, transa: bool = False, transb: bool = False, alpha: float = 1.0,
            beta: float = 0.0, C_out=None, split_work: bool = True):
    """C = alpha op(A) op(B) + beta C by the split-bfloat16 three-pass product."""
    return _gemm("rrf_gemm_x3", A, B, transa, transb, alpha, beta, C_out, split_work)


def gemm_x6(A, B, *, transa: bool = False, transb: bool = False, alpha: float = 1.0,
            beta: float = 0.0, C_out=None, split_work: bool = True):
    """C = alpha op(A) op(B) + beta C by the split-bfloat16 six-term product."""
    return _gemm("rrf_gemm_x6", A, B, transa, transb, alpha, beta, C_out, split_work)


def _gemm(name, A, B, transa, transb, alpha, beta, C_out, split_work):
    torch = _torch()
    _require(A, "A")
    _require(B, "B")
    M = int(A.shape[1] if transa else A.shape[0])
    K = int(A.shape[0] if transa else A.shape[1])
    Kb = int(B.shape[1] if transb else B.shape[0])
    N = int(B.shape[0] if transb else B.shape[1])
    if K != Kb:
        raise ValueError("inner dimensions differ")
    if C_out is None:
        C_out = empty_colmajor(M, N, A.device)
        if beta != 0.0:
            raise ValueError("beta != 0 needs C_out")
    _require(C_out, "C", rows=M)
    work = torch.empty(8 * M * N * 8 if split_work else 0, dtype=torch.uint8, device=A.device)
    _check(getattr(lib, name)(int(transa), int(transb), M, N, K, alpha, A.data_ptr(), _ld(A),
                              B.data_ptr(), _ld(B), beta, C_out.data_ptr(), _ld(C_out),
                              work.data_ptr() if work.numel() else None, work.numel(),
                              _stream_ptr(A.device)), name)
    return C_out


def householder_panel(P, *, inplace: bool = False):
    """Householder QR of a tall panel: returns (W, R, Tf, tau), Q = I - W Tf W^T."""
    torch = _torch()
    _require(P, "P")
    M, k = int(P.shape[0]), int(P.shape[1])
    W = P if inplace else empty_colmajor(M, k, P.device)
    R = empty_colmajor(k, k, P.device)
    Tf = empty_colmajor(k, k, P.device)
    tau = torch.empty(k, dtype=torch.float64, device=P.device)
    nbytes = int(lib.rrf_panel_workspace_size(M, k))
    if nbytes == 0:
        raise RRFError(_lib.RRF_E_NOTSUP, "householder_panel", "shape not supported")
    work = torch.empty(nbytes, dtype=torch.uint8, device=P.device)
    _check(lib.rrf_householder_panel(M, k, P.data_ptr(), _ld(P), W.data_ptr(), _ld(W),
                                     R.data_ptr(), k, Tf.data_ptr(), k, tau.data_ptr(),
                                     work.data_ptr(), nbytes, _stream_ptr(P.device)),
           "rrf_householder_panel")
    return W, R, Tf, tau


def trace_enable(on: bool = True) -> None:
    """Switch the library's per-kernel event timing on/off (clears totals)."""
    _check(lib.rrf_trace_enable(1 if on else 0), "rrf_trace_enable")


def trace_enable_class(name: str) -> None:
    """Time only the launches of one kernel class (clears totals)."""
    _check(lib.rrf_trace_enable_class(name.encode()), "rrf_trace_enable_class")


def trace_read() -> list[dict]:
    """Per-kernel-class totals recorded since trace_enable()."""
    buf = (_lib.rrf_trace_entry * 64)()
    n = lib.rrf_trace_read(buf, 64)
    return [dict(name=e.name.decode(), launches=int(e.launches), ms=float(e.ms),
                 flops=float(e.flops), bytes=float(e.bytes)) for e in buf[:n]]


def block_svd(B):
    """SVD of a small k x k block: returns (Us, d, Vs) with B = Us diag(d) Vs^T."""
    torch = _torch()
    _require(B, "B")
    k = int(B.shape[0])
    if int(B.shape[1]) != k:
        raise ValueError("block_svd needs a square block")
    Us = empty_colmajor(k, k, B.device)
    Vs = empty_colmajor(k, k, B.device)
    d = torch.empty(k, dtype=torch.float64, device=B.device)
    nbytes = int(lib.rrf_block_svd_workspace_size(k))
    work = torch.empty(nbytes, dtype=torch.uint8, device=B.device)
    _check(lib.rrf_block_svd(k, B.data_ptr(), _ld(B), Us.data_ptr(), d.data_ptr(), Vs.data_ptr(),
                             work.data_ptr(), nbytes, _stream_ptr(B.device)), "rrf_block_svd")
    return Us, d, Vs


def _ld8(rows: int) -> int:
    return (max(rows, 1) + 7) // 8 * 8


def to_bf16(X, *, scaled: bool = False, transpose: bool = False):
    """bfloat16 bit patterns (torch.int16, column-major, ld a multiple of 8)
    of X, or of X times the power of two putting max|X| in [0.5, 1) when
    `scaled`; with `transpose` also of X^T. Returns (out, outT or None), each
    a (ld x cols) tensor whose first rows hold the values."""
    torch = _torch()
    _require(X, "X")
    rows, cols = int(X.shape[0]), int(X.shape[1])
    out = empty_colmajor(_ld8(rows), cols, X.device, torch.int16)
    outT = empty_colmajor(_ld8(cols), rows, X.device, torch.int16) if transpose else None
    work = torch.empty(256, dtype=torch.uint8, device=X.device)
    _check(lib.rrf_to_bf16(rows, cols, X.data_ptr() if X.numel() else None, _ld(X),
                           1 if scaled else 0, out.data_ptr(), _ld8(rows),
                           outT.data_ptr() if outT is not None else None,
                           _ld8(cols) if outT is not None else 0, work.data_ptr(), 256,
                           _stream_ptr(X.device)), "rrf_to_bf16")
    return out, outT


def gemm_bf16_tn(A16, K: int, B16, *, out: str = "f64"):
    """A^T B of bfloat16 matrices given as int16 bit patterns (K valid rows,
    leading dimension = the tensors' first dimension, a multiple of 8, rows
    past K zero). out "f64" widens the FP32 result; "bf16" returns it column-
    rescaled by powers of two and rounded (as int16 bit patterns)."""
    torch = _torch()
    M, N = int(A16.shape[1]), int(B16.shape[1])
    work_bytes = int(lib.rrf_gemm_bf16_workspace_size(M, N))
    work = torch.empty(work_bytes, dtype=torch.uint8, device=A16.device)
    if out == "f64":
        C64 = empty_colmajor(M, N, A16.device)
        o16, ld16, o64, ld64 = None, 0, C64.data_ptr(), M
    else:
        C16 = empty_colmajor(_ld8(M), N, A16.device, torch.int16)
        o16, ld16, o64, ld64 = C16.data_ptr(), _ld8(M), None, 0
    _check(lib.rrf_gemm_bf16_tn(M, N, K, A16.data_ptr(), int(A16.shape[0]), B16.data_ptr(),
                                int(B16.shape[0]), o16, ld16, o64, ld64, work.data_ptr(),
                                work_bytes, _stream_ptr(A16.device)), "rrf_gemm_bf16_tn")
    return C64 if out == "f64" else C16
