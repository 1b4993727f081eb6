#!/usr/bin/env python3
"""Time-to-factor of randUTV (Alg. 3) on one MI355X: FP64, and the mixed sketch.

Workload (default): A = Q1 diag(s) Q2^T, n = 16384, s_j = exp(-j/800), Q1/Q2
Haar (synthetic, seeded, generated on the GPU), b = 128, q = 2, sketch seed 1,
U and V accumulated. One "step" is one complete factorization A = U T V^T with
A, U, T, V and the workspace resident in HBM before the timed region starts.

Printed on stdout: ONE short JSON line (the last line) with the time per FP64
factorization (`value`, seconds, lower is better), the roofline entry of the
dominant kernel measured live with HIP events on the library's stream, the
FP64 CPU oracle timed on a bounded sample of the same workload
(`cpu_baseline`), the accuracy of the result against the known spectrum, and
one scalar summary per further leg: the same factorization with the bfloat16
sketch (RRF_PREC_BF16_SKETCH) held to e_k <= max(1.5 sigma_{k+1}, 1.1
e_k(FP64)) on the k-grid ("mixed"), with the split-bfloat16 updates
(RRF_PREC_BF16_X3, "mixed_x3") and with the six-term updates (RRF_PREC_BF16_X6,
"mixed_x6"; "mixed_best" names the fastest mode meeting recon <= 1e-6 and the
e_k gate), powerURV, Alg. 2 with p = b, the early-stopped
randUTV, the RSVD, the 32768 x 8192 sharp-gap workload in the four precision
modes ("gap") and the batched call on 4096 small matrices (n ~ U{64..512},
m ~ U{n..2n}, graded spectrum, q = 1, automatic b) in matrices per second.
The full object (kernel tables, e_k arrays, per-mode details) is written to
the file `--full-json` names (none by default).

    python bench.py [--steps K] [--warmup W] [--n N] [--b B] [--q Q]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "time-to-factor & %MFMA peak, n=16384 randUTV FP64 vs mixed at equal e_k"
PEAK_FP64_TFLOPS = 78.6     # MI355X dense FP64 matrix peak
PEAK_HBM_GBS = 8000.0       # MI355X HBM3E

# HBM bytes per launch of each FP64 GEMM class on the default workload, from
# rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs scaled by the counters' reading
# for a 1 GiB device copy (profiles/randutv_n16384_b128_q2_fp64_hbm_traffic.md).
# They describe the GEMM sources whose concatenation has this SHA-256 prefix.
TRAFFIC_SOURCES = ("paper_2106_13402_amd/csrc/gemm_f64.hip",
                   "paper_2106_13402_amd/csrc/gemm_tile.hpp")
TRAFFIC_SHA256_16 = "ecd0d9b2ecc041be"
TRAFFIC_BYTES_PER_LAUNCH = {
    "dgemm_mfma_128x128_NN": 608569199,
    "dgemm_mfma_128x128_TN": 595920261,
    "dgemm_mfma_128x128_NT": 759931359,
    "dgemm_mfma_128x128_NN:UV": 426668034,
    "dgemm_mfma_128x128_TN:UV": 857692318,
}

# Matrix-core counters of the same classes on the same sources
# (profiles/randutv_n16384_b128_q2_fp64_mfma_counters.md): FP64 MFMA flops
# from SQ_INSTS_VALU_MFMA_MOPS_F64 over the dispatch time, as a fraction of
# peak, and SQ_VALU_MFMA_BUSY_CYCLES over the active cycles of all SIMDs.
MFMA_COUNTERS = {
    "dgemm_mfma_128x128_TN": (0.572, 0.627),
    "dgemm_mfma_128x128_NN": (0.635, 0.693),
    "dgemm_mfma_128x128_NT": (0.566, 0.625),
    "dgemm_mfma_128x128_NN:UV": (0.558, 0.581),
    "dgemm_mfma_128x128_TN:UV": (0.553, 0.591),
}


def _sources_match() -> bool:
    import hashlib
    h = hashlib.sha256()
    for src in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16] == TRAFFIC_SHA256_16


def measured_mfma(kernel: str, n: int, b: int, q: int):
    """(counter flop fraction, MFMA busy fraction) of a GEMM class, or None
    when the workload or the GEMM sources differ from the profiled ones."""
    if (n, b, q) != (16384, 128, 2) or not _sources_match():
        return None
    return MFMA_COUNTERS.get(kernel)


def measured_traffic(kernel: str, n: int, b: int, q: int):
    """Counter-measured HBM bytes per launch, or None when the workload or
    the GEMM source differ from those the counters were taken on."""
    if (n, b, q) != (16384, 128, 2) or not _sources_match():
        return None
    return TRAFFIC_BYTES_PER_LAUNCH.get(kernel)


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ---------------------------------------------------------- algorithmic work
def step_flops(m: int, n: int, b: int, q: int, i: int) -> float:
    """Flops of loop iteration i (1-based) of Alg. 3 with U and V accumulated.

    Sketch (2 + 4q) M N b; the two compact-WY applications of V_i (to T: m
    rows, to V: n rows) and of U_i (to T(I2uI3, J3) and to U: m rows), each
    4 rows x cols x b; the two panel QRs 2 (M + N) b^2; the small b x b block
    updates. The O(b^3) Jacobi SVD is not counted.
    """
    c0 = b * (i - 1)
    M, N = m - c0, n - c0
    if c0 + b >= n:
        nb = N
        f = 2.0 * c0 * nb * nb + 2.0 * (m + n) * nb * nb
        if M > nb:
            f += 2.0 * M * nb * nb + 4.0 * m * M * nb
        return f
    f = (2.0 + 4.0 * q) * M * N * b
    f += 4.0 * m * N * b + 4.0 * M * (N - b) * b
    f += 4.0 * n * N * b + 4.0 * m * M * b
    f += 2.0 * (M + N) * b * b
    f += 2.0 * b * b * (N - b) + 2.0 * c0 * b * b + 2.0 * (m + n) * b * b
    return f


def total_flops(m: int, n: int, b: int, q: int) -> float:
    return sum(step_flops(m, n, b, q, i) for i in range(1, math.ceil(n / b) + 1))


# ----------------------------------------------------------- error estimates
def _power_norm(apply, apply_t, n, device, iters=40, seed=0):
    """||M||_2 by power iteration on M^T M (matvecs only)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    x = torch.randn(n, 1, dtype=torch.float64, device=device, generator=g)
    x /= torch.linalg.vector_norm(x)
    est = 0.0
    for _ in range(iters):
        y = apply_t(apply(x))
        nrm = float(torch.linalg.vector_norm(y))
        if nrm == 0.0:
            return 0.0
        est = math.sqrt(nrm)
        x = y / nrm
    return est


def accuracy(A, U, T, V, s, kgrid):
    import torch
    dev = A.device
    n = A.shape[1]
    nA = float(s[0])

    def orth(Q):
        return _power_norm(lambda x: Q.t() @ (Q @ x) - x, lambda x: Q.t() @ (Q @ x) - x,
                           Q.shape[1], dev, iters=30)

    rec = _power_norm(lambda x: A @ x - U @ (T @ (V.t() @ x)),
                      lambda y: A.t() @ y - V @ (T.t() @ (U.t() @ y)), n, dev) / nA
    ratios, eks = [], []
    for k in kgrid:
        Tk = T[k:, k:]
        ek = _power_norm(lambda x: Tk @ x, lambda y: Tk.t() @ y, n - k, dev, iters=30)
        eks.append(ek)
        ratios.append(ek / float(s[k]))
    worst = max(range(len(kgrid)), key=lambda i: ratios[i])
    return {
        "orth_U": orth(U), "orth_V": orth(V), "recon": rec,
        "ek_over_sigma_max": ratios[worst], "ek_over_sigma_argmax_k": int(kgrid[worst]),
        "ek_over_sigma_min": min(ratios), "k_grid": [int(k) for k in kgrid], "e_k": eks,
        "norm_estimator": "power iteration (30-40 steps)",
    }


# -------------------------------------------------------------- CPU baseline
def cpu_baseline(A_host, b, q, seed, budget_s):
    """Time the oracle on its first steps of the same factorization and scale
    by the algorithmic flop model to a whole factorization."""
    import numpy as np
    import oracle

    m, n = A_host.shape
    marks = [time.perf_counter()]

    class Enough(Exception):
        pass

    def on_step(i, T):
        marks.append(time.perf_counter())
        if marks[-1] - marks[0] >= budget_s:
            raise Enough()

    try:
        oracle.randutv(np.asfortranarray(A_host), b, q, seed, on_step=on_step)
    except Enough:
        pass
    steps = len(marks) - 1
    elapsed = marks[-1] - marks[0]
    done = sum(step_flops(m, n, b, q, i) for i in range(1, steps + 1))
    rate = done / elapsed
    total = total_flops(m, n, b, q)
    cores = len(os.sched_getaffinity(0))
    try:
        from threadpoolctl import threadpool_info
        cores = max(int(p.get("num_threads", 0)) for p in threadpool_info()) or cores
    except Exception:
        pass
    return {
        "value": total / rate, "unit": "s", "cores": cores, "kind": "oracle",
        "sample": (f"first {steps} of {math.ceil(n / b)} steps of the same randUTV "
                   f"(n={n}, b={b}, q={q}, U and V accumulated) in {elapsed:.1f} s; "
                   f"time per factorization extrapolated by the algorithmic flop model "
                   f"({rate / 1e9:.1f} GFLOP/s over the sample)"),
    }


# ------------------------------------------------------------ powerURV leg
def powerurv_flops(m: int, n: int, q: int) -> float:
    """Algorithmic flops of Alg. 1 with explicit Q factors (U formed), with
    LAPACK's counts: QR of m x n 2 m n^2 - 2/3 n^3, its thin Q the same, a
    full m x m Q 4 m^2 n - 4 m n^2 + 4/3 n^3. Per power round A V and
    A^T V_hat (2 m n^2 each), QR + thin Q of the m x n product, QR + Q of the
    n x n one (8/3 n^3); then A V, its QR and the m x m U. For m = n this is
    (28 q / 3 + 14 / 3) n^3 (q = 0: the RURV start QR adds 8/3 n^3)."""
    per_round = 4 * m * n * n + (4 * m * n * n - 4 / 3 * n ** 3) + 8 / 3 * n ** 3
    tail = 2 * m * n * n + (2 * m * n * n - 2 / 3 * n ** 3) + (4 * m * m * n - 4 * m * n * n
                                                               + 4 / 3 * n ** 3)
    start = 8 / 3 * n ** 3 if q == 0 else 0.0
    return q * per_round + tail + start


def powerurv_leg(A, U, T, V, s, kgrid, b, q, args, dev, fp64_acc):
    """powerURV (Alg. 1) on the same matrix, FP64 and with the bfloat16 power
    products, timed like the randUTV legs (U and V formed)."""
    import ctypes as C
    import torch
    import paper_2106_13402_amd as rrf
    from paper_2106_13402_amd import _lib
    n = A.shape[1]

    def factor(precision):
        nbytes = rrf.workspace_size("powerurv", n, n, b, q, precision)
        ws = rrf._workspace(dev, nbytes)
        opts = _lib.rrf_opts()
        rrf.lib.rrf_opts_init(C.byref(opts))
        opts.precision = rrf.PRECISIONS[precision]
        opts.stream = torch.cuda.current_stream(dev).cuda_stream
        opts.workspace = ws.data_ptr()
        opts.workspace_bytes = ws.numel()
        st = rrf.lib.rrf_powerurv_ex(n, n, A.data_ptr(), n, b, q, args.seed, U.data_ptr(),
                                     T.data_ptr(), V.data_ptr(), C.byref(opts))
        if st != 0:
            raise RuntimeError(f"rrf_powerurv_ex failed: {st} {rrf.lib.rrf_last_error().decode()}")

    leg = {"workload": f"powerURV n={n} b={b} q={q}, same matrix, U and V formed",
           "model_flops": powerurv_flops(n, n, q)}
    ref = None
    for precision in ("fp64", "bf16_sketch"):
        for _ in range(args.warmup):
            factor(precision)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            factor(precision)
        torch.cuda.synchronize()
        per = (time.perf_counter() - t0) / args.steps
        log(f"powerURV {precision}: {per:.3f} s per factorization")
        r = {"value": per, "unit": "s", "model_tflops": leg["model_flops"] / per / 1e12}
        if fp64_acc is not None:
            acc = accuracy(A, U, T, V, s, kgrid)
            r["accuracy"] = acc
            if ref is None:
                ref = acc["e_k"]
            else:
                # the bfloat16 power products act on the whole of A, so they
                # resolve directions down to about 1e-3 sigma_1 only
                ks = [i for i, k in enumerate(kgrid) if s[k] >= 1e-3 * s[0]]
                r["ek_over_fp64_max"] = max(acc["e_k"][i] / ref[i] for i in ks)
                r["ek_gate"] = ("e_k <= max(1.5 sigma_{k+1}, 1.1 e_k(FP64)) on the k-grid where "
                                "sigma_{k+1} >= 1e-3 sigma_1")
                r["ek_gate_pass"] = all(acc["e_k"][i] <= max(1.5 * s[kgrid[i]], 1.1 * ref[i])
                                        for i in ks)
                r["ek_over_fp64_max_all_k"] = max(a / f for a, f in zip(acc["e_k"], ref))
        leg[precision] = r
    leg["speedup_mixed"] = leg["fp64"]["value"] / leg["bf16_sketch"]["value"]
    return leg


# ------------------------------------------------------------- batched leg
def gap_leg(args, dev):
    """The rectangular sharp-gap workload: m = 32768, n = 8192,
    A = Q1 diag(s) Q2^T + 1e-12 N(0,1) with s_j = 1 for j <= 1000 and 1e-10
    after, b = 256, q = 2, U and V formed, in FP64, with the bfloat16 sketch
    and with the x3 updates. e_k on k = 900, 904, ..., 1100. Below the gap
    sigma_{k+1} = 1 to within ||E||_2; above it Weyl's bound only brackets it,
    sigma_{k+1} <= 1e-10 + ||E||_2, so e_k / (s_{k+1} + ||E||_2) is reported
    (a lower bound of e_k / sigma_{k+1}) with the FP64 run's e_k beside it."""
    import numpy as np
    import torch

    import paper_2106_13402_amd as rrf
    from synthetic import gaussian_matrix, spectral_matrix

    m, n, b, q = 32768, 8192, 256, 2
    j = np.arange(1, n + 1)
    s = np.where(j <= 1000, 1.0, 1e-10)
    log(f"gap: generating A, {m} x {n}")
    E = gaussian_matrix(m, n, 0, 3, dev)
    e_norm = 1e-12 * _power_norm(lambda x: E @ x, lambda y: E.t() @ y, n, dev, iters=40)
    del E
    A = spectral_matrix(m, n, s, seed=0, noise=1e-12, device=dev)
    U = rrf.empty_colmajor(m, m, dev)
    T = rrf.empty_colmajor(m, n, dev)
    V = rrf.empty_colmajor(n, n, dev)
    kgrid = list(range(900, 1101, 4))

    def factor(precision, thin_u=False):
        import ctypes as C
        from paper_2106_13402_amd import _lib
        ws = rrf._workspace(dev, rrf.workspace_size("randutv", m, n, b, q, precision))
        opts = _lib.rrf_opts()
        rrf.lib.rrf_opts_init(C.byref(opts))
        opts.precision = rrf.PRECISIONS[precision]
        opts.thin_u = 1 if thin_u else 0
        opts.stream = torch.cuda.current_stream(dev).cuda_stream
        opts.workspace = ws.data_ptr()
        opts.workspace_bytes = ws.numel()
        st = rrf.lib.rrf_randutv_ex(m, n, A.data_ptr(), m, b, q, args.seed, U.data_ptr(),
                                    T.data_ptr(), V.data_ptr(), C.byref(opts))
        if st != 0:
            raise RuntimeError(f"rrf_randutv_ex failed: {st} {rrf.lib.rrf_last_error().decode()}")

    leg = {"workload": f"randUTV m={m} n={n} b={b} q={q}, A=Q1 diag(s) Q2^T + 1e-12 N(0,1), "
                       "s_j = 1 (j <= 1000), 1e-10 after; U and V accumulated",
           "noise_norm": e_norm, "k_grid": kgrid, "modes": {}}
    ek64 = None
    for precision in ("fp64", "bf16_sketch", "bf16_x3", "bf16_x6"):
        factor(precision)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        factor(precision)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        acc = accuracy(A, U, T, V, s, [0])
        eks = []
        for k in kgrid:
            Tk = T[k:, k:]
            eks.append(_power_norm(lambda x: Tk @ x, lambda y: Tk.t() @ y, n - k, dev, iters=60))
        if ek64 is None:
            ek64 = eks
        lo = [e / (float(s[k]) + e_norm) for e, k in zip(eks, kgrid)]
        below = [i for i, k in enumerate(kgrid) if k < 1000]
        above = [i for i, k in enumerate(kgrid) if k >= 1000]
        leg["modes"][precision] = {
            "value": sec, "unit": "s", "speedup_vs_fp64": None,
            "recon": acc["recon"], "orth_U": acc["orth_U"], "orth_V": acc["orth_V"],
            "e_k": eks, "ek_over_fp64": [e / r for e, r in zip(eks, ek64)],
            "ek_over_sigma_below_gap_max": max(lo[i] for i in below),
            "ek_over_sigma_bound_above_gap_max": max(lo[i] for i in above),
            "e_1000": eks[kgrid.index(1000)], "e_1024": eks[kgrid.index(1024)],
        }
        log(f"gap {precision}: {sec:.3f} s, recon {acc['recon']:.2e}, "
            f"e_1000 {eks[kgrid.index(1000)]:.3e} (FP64 {ek64[kgrid.index(1000)]:.3e})")
    t64 = leg["modes"]["fp64"]["value"]
    for v in leg["modes"].values():
        v["speedup_vs_fp64"] = t64 / v["value"]
    # the same FP64 factorization forming only U(:, 1:n) (rrf_opts.thin_u):
    # U's accumulation is most of this workload's flops
    factor("fp64", thin_u=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    factor("fp64", thin_u=True)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    Ut = U[:, :n]
    rec = _power_norm(lambda x: A @ x - Ut @ (T[:n] @ (V.t() @ x)),
                      lambda y: A.t() @ y - V @ (T[:n].t() @ (Ut.t() @ y)), n, dev) / float(s[0])
    leg["fp64_thin_u"] = {"value": sec, "unit": "s", "speedup_vs_full_u": t64 / sec,
                          "recon": rec}
    log(f"gap fp64 thin U: {sec:.3f} s, recon {rec:.2e}")
    del A, U, T, V
    torch.cuda.empty_cache()
    return leg


def extra_legs(A, s, kgrid, b, q, args, dev, ek_basic):
    """The rows built beyond the headline path, on the headline matrix:
    randUTV_boosted (Alg. 2, p = b), randUTV halted at ||T22||_F <= 1e-2
    ||A||_F (Sec. 4.1) and the RSVD at l = b (Sec. 3.3). One warm call and
    one timed call each (the boosted run takes seconds)."""
    import numpy as np
    import torch

    import paper_2106_13402_amd as rrf

    n = A.shape[1]
    out = {}

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, r

    sec, (U, T, V) = timed(lambda: rrf.randutv_boosted(A, b, q, b, args.seed))
    acc = accuracy(A, U, T, V, s, kgrid) if not args.no_accuracy else None
    leg = {"workload": f"randUTV_boosted n={n} b={b} p={b} q={q}", "value": sec, "unit": "s"}
    if acc:
        leg["accuracy"] = acc
        if ek_basic:
            leg["ek_over_basic"] = [e / r for e, r in zip(acc["e_k"], ek_basic)]
    out["boosted"] = leg
    log(f"boosted: {sec:.3f} s")
    del U, T, V
    torch.cuda.empty_cache()

    tol = 1e-2
    sec, (U, T, V, k) = timed(lambda: rrf.randutv_partial(A, b, q, args.seed, tol))
    e = float(torch.linalg.matrix_norm(T[k:, k:])) / float(torch.linalg.matrix_norm(A))
    out["partial"] = {"workload": f"randUTV n={n} b={b} q={q} halted at ||T22||_F <= {tol} ||A||_F",
                      "value": sec, "unit": "s", "k": k, "rel_frobenius_remainder": e,
                      "expected_k": int(np.ceil(400 * np.log(1 / tol ** 2) / b) * b)}
    log(f"partial: {sec:.3f} s, k = {k}, ||T22||_F / ||A||_F = {e:.2e}")
    del U, T, V
    torch.cuda.empty_cache()

    l = b
    sec, (U, S, V) = timed(lambda: rrf.rsvd(A, l, q, args.seed))
    err = _power_norm(lambda x: A @ x - U @ (S[:, None] * (V.t() @ x)),
                      lambda y: A.t() @ y - V @ (S[:, None] * (U.t() @ y)), n, dev)
    sv = np.asarray(s[:l])
    out["rsvd"] = {"workload": f"RSVD n={n} l={l} q={q}", "value": sec, "unit": "s",
                   "err_over_sigma_l1": err / float(s[l]),
                   "sigma_rel_err_max": float(np.max(np.abs(S.cpu().numpy() - sv) / sv))}
    log(f"rsvd: {sec * 1e3:.1f} ms, ||A - U S V^T|| / sigma_(l+1) = {err / float(s[l]):.3f}")
    return out


def auto_block(n: int, m: int = 0) -> int:
    """Block size the batched call picks for b = 0."""
    import paper_2106_13402_amd as rrf
    return rrf.batched_block(max(m, n), n)


def batched_leg(count: int, q: int, steps: int, warmup: int, seed: int, cpu_seconds: float,
                cpu: bool) -> dict:
    """rrf_randutv_batched on `count` matrices, n ~ U{64..512}, m ~ U{n..2n},
    A_j = Q1 diag(10^(-8 (i-1)/(n-1))) Q2^T, automatic b, U and V accumulated;
    matrices per second over `steps` timed calls, the relative residual of
    every matrix, and the oracle timed on a bounded sample."""
    import numpy as np
    import torch

    import paper_2106_13402_amd as rrf
    from synthetic import batch_shapes, batch_spectral

    dev = torch.device("cuda:0")
    shapes = batch_shapes(count, seed=0)
    t0 = time.perf_counter()
    As = batch_spectral(shapes, seed=0, decades=8.0, device=dev)
    torch.cuda.synchronize()
    log(f"batched: {count} matrices generated in {time.perf_counter() - t0:.1f} s")
    out = ([rrf.empty_colmajor(m, m, dev) for m, n in shapes],
           [rrf.empty_colmajor(m, n, dev) for m, n in shapes],
           [rrf.empty_colmajor(n, n, dev) for m, n in shapes])
    for _ in range(max(warmup, 1)):
        rrf.randutv_batched(As, 0, q, seed, out=out)  # checks the arguments once
    # the timed calls go straight to the C-ABI with the arrays built once
    import ctypes as C
    from paper_2106_13402_amd import _lib
    count = len(shapes)
    i64 = lambda v: (C.c_int64 * count)(*v)
    ptrs = lambda ts: (C.c_void_p * count)(*[t.data_ptr() for t in ts])
    ms, ns = i64([m for m, n in shapes]), i64([n for m, n in shapes])
    pa, pu, pt, pv = ptrs(As), ptrs(out[0]), ptrs(out[1]), ptrs(out[2])
    ldas = i64([int(A.stride(1)) for A in As])
    nbytes = rrf.batched_workspace_size([m for m, n in shapes], [n for m, n in shapes], 0, "fp64")
    ws = rrf._workspace(dev, nbytes)
    opts = _lib.rrf_opts()
    rrf.lib.rrf_opts_init(C.byref(opts))
    opts.stream = torch.cuda.current_stream(dev).cuda_stream
    opts.workspace = ws.data_ptr()
    opts.workspace_bytes = ws.numel()

    def call():
        st = rrf.lib.rrf_randutv_batched(count, ms, ns, pa, ldas, 0, q, seed, pu, pt, pv,
                                         C.byref(opts))
        if st != 0:
            raise RuntimeError(f"rrf_randutv_batched failed: {st} "
                               f"{rrf.lib.rrf_last_error().decode()}")

    call()
    # one more untimed call with every launch timed by HIP events (the
    # per-class breakdown); the timed calls instrument no launch
    rrf.trace_enable(True)
    call()
    torch.cuda.synchronize()
    kern = rrf.trace_read()
    rrf.trace_enable(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        call()
    torch.cuda.synchronize()
    per = (time.perf_counter() - t0) / steps
    log(f"batched: {per * 1e3:.1f} ms per call, {count / per:.0f} matrices/s")
    flops = sum(total_flops(m, n, auto_block(n, m), q) for m, n in shapes)
    Us, Ts, Vs = out
    res = torch.empty(count, dtype=torch.float64, device=dev)
    orth = torch.empty(count, dtype=torch.float64, device=dev)
    for j, (m, n) in enumerate(shapes):
        A = As[j]
        res[j] = torch.linalg.norm(A - Us[j] @ Ts[j] @ Vs[j].t()) / torch.linalg.norm(A)
        eu = torch.linalg.norm(Us[j].t() @ Us[j] - torch.eye(m, dtype=A.dtype, device=dev))
        ev = torch.linalg.norm(Vs[j].t() @ Vs[j] - torch.eye(n, dtype=A.dtype, device=dev))
        orth[j] = torch.maximum(eu, ev)
    res, orth = res.cpu().numpy(), orth.cpu().numpy()
    kernels = {e["name"]: {"launches": e["launches"], "ms_per_call": e["ms"],
                           "tflops": (e["flops"] / (e["ms"] * 1e-3) / 1e12) if e["flops"] else None}
               for e in kern}
    leg = {
        "workload": (f"randUTV of {count} matrices, n ~ U{{64..512}}, m ~ U{{n..2n}}, "
                     f"A = Q1 diag(10^(-8(i-1)/(n-1))) Q2^T, q={q}, b per size bucket from "
                     f"the loaded tuning table, U and V accumulated, FP64"),
        "value": count / per, "unit": "matrices/s", "ms_per_call": per * 1e3,
        "model_flops": flops, "model_tflops": flops / per / 1e12,
        # the whole call against FP64 matrix-core peak: the flop model of
        # Alg. 3 summed over the batch, as if every flop ran at 78.6 TFLOP/s
        "roofline": {"bound": "mfma", "ideal_ms": flops / (PEAK_FP64_TFLOPS * 1e12) * 1e3,
                     "frac": flops / per / 1e12 / PEAK_FP64_TFLOPS, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s"},
        "roofline_frac": flops / per / 1e12 / PEAK_FP64_TFLOPS,
        "blocks": {str(b): sum(1 for m, n in shapes if auto_block(n, m) == b)
                   for b in sorted({auto_block(n, m) for m, n in shapes})},
        "residual_fro_rel": {"max": float(res.max()), "median": float(np.median(res)),
                             "p99": float(np.quantile(res, 0.99))},
        "orth_fro_max": float(orth.max()),
        "kernels": kernels,
    }
    if cpu:
        import oracle
        done, fl, t0 = 0, 0.0, time.perf_counter()
        for j, (m, n) in enumerate(shapes):
            oracle.randutv(As[j].cpu().numpy().copy(order="F"), auto_block(n, m), q, seed + j)
            done += 1
            fl += total_flops(m, n, auto_block(n, m), q)
            if time.perf_counter() - t0 >= cpu_seconds:
                break
        el = time.perf_counter() - t0
        rate = fl / el
        cores = len(os.sched_getaffinity(0))
        try:
            from threadpoolctl import threadpool_info
            cores = max(int(p.get("num_threads", 0)) for p in threadpool_info()) or cores
        except Exception:
            pass
        leg["cpu_baseline"] = {
            "value": count / (flops / rate), "unit": "matrices/s", "cores": cores,
            "kind": "oracle",
            "sample": (f"the first {done} matrices of the batch, one after another, in "
                       f"{el:.1f} s ({rate / 1e9:.1f} GFLOP/s); matrices/s for the whole batch "
                       f"by the algorithmic flop model"),
        }
    return leg


# ------------------------------------------------------------ headline line
def _r(x, digits=4):
    """Round a float to `digits` significant digits (None passes through)."""
    if x is None or isinstance(x, bool) or not isinstance(x, float):
        return x
    if x == 0.0 or not math.isfinite(x):
        return x
    return float(f"{x:.{digits}g}")


def _acc_summary(acc):
    if not acc:
        return None
    return {"recon": _r(acc["recon"], 3), "orth_U": _r(acc["orth_U"], 3),
            "orth_V": _r(acc["orth_V"], 3), "ek_over_sigma_max": _r(acc["ek_over_sigma_max"], 4),
            "ek_over_sigma_argmax_k": acc["ek_over_sigma_argmax_k"]}


def headline(out: dict) -> dict:
    """The one-line result: the contract's keys, the roofline and CPU baseline
    of the headline workload, and one scalar summary per extra leg. Arrays and
    kernel tables stay in the full object (written to a file)."""
    keys = ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
            "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config")
    h = {k: _r(out[k]) if isinstance(out[k], float) else out[k] for k in keys}
    h["roofline"] = {k: _r(v) for k, v in out["roofline"].items()}
    if "cpu_baseline" in out:
        h["cpu_baseline"] = {k: _r(v) for k, v in out["cpu_baseline"].items()}
    h["model_tflops"] = _r(out["model_tflops"])
    h["gemm_all_frac"] = _r(out["gemm_all"]["frac"])
    if "accuracy" in out:
        h["accuracy"] = _acc_summary(out["accuracy"])
    legs = {}
    for name in ("mixed", "mixed_x3", "mixed_x6"):
        if name in out:
            leg = out[name]
            legs[name] = {"precision": leg["precision"], "value": _r(leg["value"]),
                          "speedup_vs_fp64": _r(leg["speedup_vs_fp64"]),
                          "recon": _r(leg["accuracy"]["recon"], 3) if "accuracy" in leg else None,
                          "ek_over_fp64_max": _r(leg.get("ek_over_fp64_max")),
                          "ek_gate_pass": leg.get("ek_gate_pass"),
                          "recon_le_1e-6": leg.get("recon_le_1e-6")}
    # the fastest mixed mode that meets both accuracy targets
    ok = [v for v in legs.values() if v.get("ek_gate_pass") and v.get("recon_le_1e-6")]
    if ok:
        best = max(ok, key=lambda v: v["speedup_vs_fp64"])
        h["mixed_best"] = {"precision": best["precision"], "value": best["value"],
                           "speedup_vs_fp64": best["speedup_vs_fp64"], "recon": best["recon"]}
    if "powerurv" in out:
        p = out["powerurv"]
        legs["powerurv"] = {"fp64_s": _r(p["fp64"]["value"]),
                            "fp64_model_tflops": _r(p["fp64"]["model_tflops"]),
                            "bf16_s": _r(p["bf16_sketch"]["value"]),
                            "speedup_mixed": _r(p["speedup_mixed"]),
                            "bf16_ek_gate_pass": p["bf16_sketch"].get("ek_gate_pass"),
                            "fp64_recon": _r(p["fp64"]["accuracy"]["recon"], 3)
                            if "accuracy" in p["fp64"] else None}
    if "gap" in out:
        g = out["gap"]["modes"]
        legs["gap"] = {mode: {"value": _r(v["value"]), "speedup_vs_fp64": _r(v["speedup_vs_fp64"]),
                              "recon": _r(v["recon"], 3), "e_1000": _r(v["e_1000"], 4)}
                       for mode, v in g.items()}
        if "fp64_thin_u" in out["gap"]:
            legs["gap"]["fp64_thin_u_s"] = _r(out["gap"]["fp64_thin_u"]["value"])
    if "boosted" in out:
        legs["boosted_s"] = _r(out["boosted"]["value"])
    if "partial" in out:
        legs["partial"] = {"value": _r(out["partial"]["value"]), "k": out["partial"]["k"]}
    if "rsvd" in out:
        legs["rsvd"] = {"value": _r(out["rsvd"]["value"]),
                        "err_over_sigma_l1": _r(out["rsvd"]["err_over_sigma_l1"])}
    if "batched" in out:
        bt = out["batched"]
        legs["batched"] = {k: _r(bt[k]) for k in ("value", "unit", "ms_per_call", "model_tflops")
                           if k in bt}
        for k in ("roofline_frac", "mode"):
            if k in bt:
                legs["batched"][k] = _r(bt[k])
        legs["batched"]["residual_max"] = _r(bt["residual_fro_rel"]["max"], 3)
        if "cpu_baseline" in bt:
            legs["batched"]["cpu_matrices_per_s"] = _r(bt["cpu_baseline"]["value"])
    h["legs"] = legs
    h["full_results"] = out.get("full_results")
    return h


# ---------------------------------------------------------------------- main
def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--b", type=int, default=128)
    ap.add_argument("--q", type=int, default=2)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-powerurv", action="store_true")
    ap.add_argument("--no-gap", action="store_true", help="skip the 32768 x 8192 gap workload")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the boosted, early-stop and RSVD legs")
    ap.add_argument("--batch", type=int, default=4096, help="matrices in the batched leg")
    ap.add_argument("--full-json", default="",
                    help="file for the full results (kernel tables, e_k arrays); "
                         "none when empty")
    ap.add_argument("--batch-q", type=int, default=1)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2106_13402_amd as rrf
    from synthetic import spectral_matrix, spectrum

    dev = torch.device("cuda:0")
    n, b, q = args.n, args.b, args.q
    s = spectrum("exp", n, scale=800.0)
    log(f"generating A = Q1 diag(exp(-j/800)) Q2^T, n={n}")
    A = spectral_matrix(n, n, s, seed=0, device=dev)
    U = rrf.empty_colmajor(n, n, dev)
    T = rrf.empty_colmajor(n, n, dev)
    V = rrf.empty_colmajor(n, n, dev)
    torch.cuda.synchronize()

    def factor(precision="fp64"):
        # same entry point as rrf.randutv, with preallocated outputs
        import ctypes as C
        from paper_2106_13402_amd import _lib
        nbytes = rrf.workspace_size("randutv", n, n, b, q, precision)
        ws = rrf._workspace(dev, nbytes)
        opts = _lib.rrf_opts()
        rrf.lib.rrf_opts_init(C.byref(opts))
        opts.precision = rrf.PRECISIONS[precision]
        opts.stream = torch.cuda.current_stream(dev).cuda_stream
        opts.workspace = ws.data_ptr()
        opts.workspace_bytes = ws.numel()
        st = rrf.lib.rrf_randutv_ex(n, n, A.data_ptr(), n, b, q, args.seed, U.data_ptr(),
                                    T.data_ptr(), V.data_ptr(), C.byref(opts))
        if st != 0:
            raise RuntimeError(f"rrf_randutv_ex failed: {st} "
                               f"{rrf.lib.rrf_last_error().decode()}")

    # The last warmup step (or, without warmup, one extra untimed step) runs
    # with every launch timed by HIP events: the per-class breakdown, and the
    # choice of the roofline kernel, the GEMM class with the most time on the
    # caller's stream (":UV" classes run concurrently after the loop, their
    # event intervals overlap). The timed steps then record events around
    # that class's launches only, so the other launches run uninstrumented.
    for w in range(max(args.warmup, 1)):
        traced = w == max(args.warmup, 1) - 1
        if traced:
            rrf.trace_enable(True)
        t0 = time.perf_counter()
        factor()
        if traced:
            torch.cuda.synchronize()
            kern = rrf.trace_read()
            rrf.trace_enable(False)
        log(f"{'warmup' if args.warmup else 'traced untimed step'} {w + 1}: "
            f"{time.perf_counter() - t0:.3f} s")
    gemms = [e for e in kern if e["name"].startswith("dgemm")]
    dom_name = max((e for e in gemms if not e["name"].endswith(":UV")), key=lambda e: e["ms"])["name"]
    gemm_ms = sum(e["ms"] for e in gemms)
    gemm_flops = sum(e["flops"] for e in gemms)
    rrf.trace_enable_class(dom_name)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        factor()
        log(f"step {k + 1}/{args.steps} done at {time.perf_counter() - t0:.3f} s")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    dom = [e for e in rrf.trace_read() if e["name"] == dom_name][0]
    rrf.trace_enable(False)
    per = elapsed / args.steps
    achieved = dom["flops"] / (dom["ms"] * 1e-3) / 1e12
    breakdown = {e["name"]: {"launches": e["launches"],
                             "ms_per_step": e["ms"],
                             "tflops": (e["flops"] / (e["ms"] * 1e-3) / 1e12) if e["flops"] else None,
                             "gbs": (e["bytes"] / (e["ms"] * 1e-3) / 1e9) if e["bytes"] else None}
                 for e in kern}
    model_flops = total_flops(n, n, b, q)

    out = {
        "metric": METRIC,
        "value": per,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": per * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"randUTV n={n} b={b} q={q}, A=Q1 diag(exp(-j/800)) Q2^T, "
                               f"U and V accumulated, FP64", "n": n, "b": b, "q": q,
                   "precision": "fp64", "sketch_seed": args.seed},
        "roofline": {
            "bound": "mfma", "kernel": dom["name"], "achieved": achieved,
            "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
            "traffic": measured_traffic(dom["name"], n, b, q),
            "traffic_unit": "bytes per launch (HBM read + write, counter-measured)",
            "algorithmic_bytes_per_launch": dom["bytes"] / dom["launches"],
            "flops_per_launch": dom["flops"] / dom["launches"],
            "avg_launch_ms": dom["ms"] / dom["launches"],
            "counter_frac": (measured_mfma(dom["name"], n, b, q) or (None, None))[0],
            "mfma_busy": (measured_mfma(dom["name"], n, b, q) or (None, None))[1],
        },
        "gemm_all": {"tflops": gemm_flops / (gemm_ms * 1e-3) / 1e12,
                     "frac": gemm_flops / (gemm_ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
                     "ms_per_step": gemm_ms},
        "model_tflops": model_flops / per / 1e12,
        "kernels": breakdown,
        "kernels_from": "the last warmup step, every launch timed by HIP events",
    }
    kgrid = [k for k in (0, 64, 127, 128, 129, 256, 1000, 2000, 4000, 8000, 12000) if k < n]
    if not args.no_accuracy:
        out["accuracy"] = accuracy(A, U, T, V, s, kgrid)
        log(f"accuracy: {out['accuracy']}")
    def mixed_leg(precision):
        # the same factorization in a mixed mode, timed the same way as the
        # FP64 run, with the kernel breakdown of a fully traced warmup step
        # (the timed steps here instrument no launch)
        for w in range(max(args.warmup, 1)):
            traced = w == max(args.warmup, 1) - 1
            if traced:
                rrf.trace_enable(True)
            factor(precision)
            if traced:
                torch.cuda.synchronize()
                kern_m = rrf.trace_read()
                rrf.trace_enable(False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            factor(precision)
        torch.cuda.synchronize()
        per_m = (time.perf_counter() - t0) / args.steps
        log(f"{precision}: {per_m:.3f} s per factorization")
        leg = {"precision": precision, "value": per_m, "unit": "s",
               "ms_per_step": per_m * 1e3, "speedup_vs_fp64": per / per_m,
               "model_tflops": model_flops / per_m / 1e12,
               "kernels_from": "the last warmup step, every launch timed by HIP events",
               "kernels": {e["name"]: {
                   "launches": e["launches"], "ms_per_step": e["ms"],
                   "tflops": (e["flops"] / (e["ms"] * 1e-3) / 1e12) if e["flops"] else None,
                   "gbs": (e["bytes"] / (e["ms"] * 1e-3) / 1e9) if e["bytes"] else None}
                   for e in kern_m}}
        if not args.no_accuracy:
            acc = accuracy(A, U, T, V, s, kgrid)
            ref = out["accuracy"]["e_k"]
            # gate on the k with sigma_{k+1} well above the reconstruction error
            ks = [i for i, k in enumerate(kgrid) if s[k] >= 100 * acc["recon"] * s[0]]
            ratio = [acc["e_k"][i] / ref[i] for i in ks]
            leg["accuracy"] = acc
            leg["ek_over_fp64_max"] = max(ratio)
            leg["ek_gate"] = "e_k <= max(1.5 sigma_{k+1}, 1.1 e_k(FP64)) on the k-grid"
            leg["ek_gate_k"] = [kgrid[i] for i in ks]
            leg["ek_gate_pass"] = all(acc["e_k"][i] <= max(1.5 * s[kgrid[i]], 1.1 * ref[i])
                                      for i in ks)
            leg["recon_le_1e-6"] = acc["recon"] <= 1e-6
            log(f"{precision} accuracy: {acc}")
        return leg

    if not args.no_mixed:
        out["mixed"] = mixed_leg("bf16_sketch")
        out["mixed_x3"] = mixed_leg("bf16_x3")
        out["mixed_x6"] = mixed_leg("bf16_x6")
    if not args.no_extra:
        out.update(extra_legs(A, s, kgrid, b, q, args, dev,
                              None if args.no_accuracy else out["accuracy"]["e_k"]))
    if not args.no_powerurv:
        out["powerurv"] = powerurv_leg(A, U, T, V, s, kgrid, b, q, args, dev,
                                       None if args.no_accuracy else out["accuracy"])
    if not args.no_gap:
        del U, T, V
        torch.cuda.empty_cache()
        out["gap"] = gap_leg(args, dev)
        U = T = V = None
    if not args.no_cpu_baseline:
        log(f"timing the CPU oracle for ~{args.cpu_seconds:.0f} s")
        A_host = A.cpu().numpy()
        del U, T, V
        out["cpu_baseline"] = cpu_baseline(A_host, b, q, args.seed, args.cpu_seconds)
    if not args.no_batched:
        out["batched"] = batched_leg(args.batch, args.batch_q, args.steps, args.warmup, args.seed,
                                     args.cpu_seconds / 2, not args.no_cpu_baseline)
    full_path = args.full_json
    out["full_results"] = full_path or None
    if full_path:
        os.makedirs(os.path.dirname(os.path.abspath(full_path)), exist_ok=True)
        with open(full_path, "w") as f:
            json.dump(out, f, indent=1)
        log(f"full results written to {full_path}")
    line = json.dumps(headline(out), separators=(",", ":"))
    print(line, flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
