// Stand-alone C-ABI client: factor a Gaussian n x n matrix with librrf and
// print one line of timings. Used to profile the library without any Python
// or torch runtime in the process (rocprofv3 --kernel-trace / --pmc).
//
//   rrf_bench [--alg randutv|powerurv] [--m M] [--n N] [--b B] [--q Q] [--reps R] [--trace]
//             [--copy-bytes BYTES] [--precision 0|1] [--no-uv]
//   rrf_bench --alg batched [--count C] [--b B] [--q Q] [--reps R] [--trace] [--precision 0|1]
//
// The batched form factors C Gaussian matrices (default 4096) with n drawn
// uniformly from [64, 512] and m from [n, 2n] by a fixed xorshift sequence
// (the distribution of the benchmark's batch, not its exact sizes); b = 0
// (default) picks the block size per matrix.
//
// --copy-bytes first runs one device-to-device copy of BYTES bytes: a plain
// copy kernel of known traffic, against which the HBM byte counters of a
// --pmc run are calibrated.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "rrf.h"

static int fail(const char* what, int st) {
  fprintf(stderr, "rrf_bench: %s failed: %d (%s)\n", what, st, rrf_last_error());
  return 1;
}

static void print_trace() {
  rrf_trace_entry e[64];
  int k = rrf_trace_read(e, 64);
  for (int i = 0; i < k; ++i)
    printf("  %-24s launches %8lld  %10.3f ms  %8.2f TF/s  %8.1f GB/s\n", e[i].name,
           (long long)e[i].launches, e[i].ms, e[i].flops / (e[i].ms * 1e-3) / 1e12,
           e[i].bytes / (e[i].ms * 1e-3) / 1e9);
}

static int run_batched(long count, long b, long q, long reps, bool trace, long precision) {
  std::vector<int64_t> m(count), n(count), ld(count);
  uint64_t x = 0x9E3779B97F4A7C15ull;
  auto next = [&]() {
    x ^= x << 13;
    x ^= x >> 7;
    x ^= x << 17;
    return x;
  };
  size_t a_el = 0, u_el = 0, v_el = 0;
  for (long j = 0; j < count; ++j) {
    n[j] = 64 + (int64_t)(next() % 449);
    m[j] = n[j] + (int64_t)(next() % (n[j] + 1));
    ld[j] = m[j];
    a_el += m[j] * n[j];
    u_el += m[j] * m[j];
    v_el += n[j] * n[j];
  }
  double *A = nullptr, *T = nullptr, *U = nullptr, *V = nullptr;
  void* ws = nullptr;
  const size_t wsb =
      rrf_randutv_batched_workspace_size(count, m.data(), n.data(), b, (int)precision);
  if (wsb == 0) return fail("rrf_randutv_batched_workspace_size", -1);
  if (hipMalloc(&A, a_el * 8) != hipSuccess || hipMalloc(&T, a_el * 8) != hipSuccess ||
      hipMalloc(&U, u_el * 8) != hipSuccess || hipMalloc(&V, v_el * 8) != hipSuccess ||
      hipMalloc(&ws, wsb) != hipSuccess) {
    fprintf(stderr, "rrf_bench: device allocation failed\n");
    return 1;
  }
  std::vector<const double*> pa(count);
  std::vector<double*> pt(count), pu(count), pv(count);
  size_t oa = 0, ou = 0, ov = 0;
  for (long j = 0; j < count; ++j) {
    pa[j] = A + oa;
    pt[j] = T + oa;
    pu[j] = U + ou;
    pv[j] = V + ov;
    const int st = rrf_gaussian(j, 1ull << 40, m[j], n[j], A + oa, m[j], nullptr);
    if (st) return fail("rrf_gaussian", st);
    oa += m[j] * n[j];
    ou += m[j] * m[j];
    ov += n[j] * n[j];
  }
  rrf_opts o;
  rrf_opts_init(&o);
  o.workspace = ws;
  o.workspace_bytes = wsb;
  o.precision = (int)precision;
  if (trace) rrf_trace_enable(1);
  double best = 1e30, total = 0.0;
  for (long r = 0; r < reps; ++r) {
    auto t0 = std::chrono::steady_clock::now();
    const int st = rrf_randutv_batched(count, m.data(), n.data(), pa.data(), ld.data(), b, (int)q,
                                       1000, pu.data(), pt.data(), pv.data(), &o);
    if (st) return fail("rrf_randutv_batched", st);
    const double s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    best = s < best ? s : best;
    total += s;
    printf("rrf_bench: batched count=%ld b=%ld q=%ld rep %ld: %.4f s (%.0f matrices/s)\n", count,
           b, q, r, s, count / s);
    fflush(stdout);
  }
  if (trace) print_trace();
  printf("rrf_bench: best %.4f s, mean %.4f s\n", best, total / reps);
  hipFree(A); hipFree(T); hipFree(U); hipFree(V); hipFree(ws);
  return 0;
}

int main(int argc, char** argv) {
  std::string alg = "randutv";
  long m = 0, n = 16384, b = 128, q = 2, reps = 1, copy_bytes = 0, precision = RRF_PREC_FP64;
  long count = 4096;
  bool b_given = false, q_given = false;
  bool trace = false, no_uv = false;
  for (int i = 1; i < argc; ++i) {
    std::string a = argv[i];
    auto next = [&](long& v) { if (i + 1 < argc) v = atol(argv[++i]); };
    if (a == "--alg" && i + 1 < argc) alg = argv[++i];
    else if (a == "--m") next(m);
    else if (a == "--n") next(n);
    else if (a == "--b") { next(b); b_given = true; }
    else if (a == "--q") { next(q); q_given = true; }
    else if (a == "--count") next(count);
    else if (a == "--reps") next(reps);
    else if (a == "--trace") trace = true;
    else if (a == "--no-uv") no_uv = true;
    else if (a == "--copy-bytes") next(copy_bytes);
    else if (a == "--precision") next(precision);
    else { fprintf(stderr, "unknown argument %s\n", a.c_str()); return 2; }
  }
  if (alg == "batched")
    return run_batched(count, b_given ? b : 0, q_given ? q : 1, reps, trace, precision);
  if (m < n) m = n;
  const size_t bytes = (size_t)m * n * sizeof(double);
  double *A = nullptr, *U = nullptr, *T = nullptr, *V = nullptr;
  void* ws = nullptr;
  const int code = alg == "powerurv" ? RRF_ALG_POWERURV : RRF_ALG_RANDUTV;
  const size_t wsb = rrf_workspace_size(code, m, n, b, (int)q, (int)precision);
  if (wsb == 0) return fail("rrf_workspace_size", -1);
  if (hipMalloc(&A, bytes) != hipSuccess || hipMalloc(&U, (size_t)m * m * 8) != hipSuccess ||
      hipMalloc(&T, bytes) != hipSuccess || hipMalloc(&V, (size_t)n * n * 8) != hipSuccess ||
      hipMalloc(&ws, wsb) != hipSuccess) {
    fprintf(stderr, "rrf_bench: device allocation failed\n");
    return 1;
  }
  int st = rrf_gaussian(0, 1ull << 40, m, n, A, m, nullptr);
  if (st) return fail("rrf_gaussian", st);
  if (copy_bytes > 0) {
    if ((size_t)copy_bytes > bytes) copy_bytes = (long)bytes;
    if (hipMemcpyAsync(T, A, (size_t)copy_bytes, hipMemcpyDeviceToDevice, nullptr) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
      fprintf(stderr, "rrf_bench: calibration copy failed\n");
      return 1;
    }
    printf("rrf_bench: calibration copy of %ld bytes\n", copy_bytes);
  }
  rrf_opts o;
  rrf_opts_init(&o);
  o.workspace = ws;
  o.workspace_bytes = wsb;
  o.precision = (int)precision;
  if (trace) rrf_trace_enable(1);
  double best = 1e30, total = 0.0;
  for (long r = 0; r < reps; ++r) {
    auto t0 = std::chrono::steady_clock::now();
    double* Uo = no_uv ? nullptr : U;
    double* Vo = no_uv ? nullptr : V;
    st = code == RRF_ALG_RANDUTV ? rrf_randutv_ex(m, n, A, m, b, (int)q, 1, Uo, T, Vo, &o)
                                 : rrf_powerurv_ex(m, n, A, m, b, (int)q, 1, Uo, T, Vo, &o);
    if (st) return fail(alg.c_str(), st);
    double s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    best = s < best ? s : best;
    total += s;
    printf("rrf_bench: %s m=%ld n=%ld b=%ld q=%ld precision=%ld rep %ld: %.4f s\n", alg.c_str(), m,
           n, b, q, precision, r, s);
    fflush(stdout);
  }
  if (trace) print_trace();
  printf("rrf_bench: best %.4f s, mean %.4f s\n", best, total / reps);
  hipFree(A); hipFree(U); hipFree(T); hipFree(V); hipFree(ws);
  return 0;
}
