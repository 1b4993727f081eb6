// The C-ABI of librrf: argument checks (before any HIP call), workspace
// management, status read-back, and the exported building blocks.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "common.hpp"
#include "context.hpp"
#include "driver.hpp"
#include "kernels.hpp"

namespace rrf {

namespace {
thread_local std::string g_last_error;
constexpr int64_t kBatchedMaxB = 64;      // one-workgroup panel width
constexpr int64_t kBatchedMaxDim = 4096;  // panel rows reachable by column splits

struct DeviceCache {
  void* ptr = nullptr;
  size_t bytes = 0;
};
std::mutex g_cache_mu;
std::unordered_map<int, DeviceCache> g_cache;
}  // namespace

int set_hip_error(hipError_t e, const char* what, const char* file, int line) {
  char buf[512];
  snprintf(buf, sizeof buf, "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
  g_last_error = buf;
  return RRF_E_HIP;
}

int set_error(int status, const char* msg) {
  g_last_error = msg;
  return status;
}

namespace {

// Fault injection for tests of the error paths, read at every call:
// RRF_TEST_FAIL=hip fails the device check, RRF_TEST_FAIL=alloc the device
// allocation of the library-managed workspace; each then takes the path a
// real failure takes.
bool fail_injected(const char* what) {
  const char* v = getenv("RRF_TEST_FAIL");
  return v != nullptr && strcmp(v, what) == 0;
}

int device_ready(int* dev) {
  int count = 0;
  hipError_t e = fail_injected("hip") ? hipErrorNoDevice : hipGetDeviceCount(&count);
  if (e != hipSuccess || count < 1) return set_error(RRF_E_HIP, "no HIP device available");
  RRF_CHECK_HIP(hipGetDevice(dev));
  return RRF_OK;
}

// -k if `p` (argument k) is not device memory of a HIP device.
int check_device_ptr(const void* p, int argpos) {
  if (p == nullptr) return RRF_OK;
  hipPointerAttribute_t attr;
  hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    set_error(-argpos, "argument is not a HIP device pointer");
    return -argpos;
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged) {
    set_error(-argpos, "argument is not device memory");
    return -argpos;
  }
  return RRF_OK;
}

// Library-managed workspace of the current device (grown, never shrunk).
int cached_workspace(int dev, size_t bytes, void** out) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  DeviceCache& c = g_cache[dev];
  if (c.bytes < bytes) {
    if (c.ptr) {
      RRF_CHECK_HIP(hipDeviceSynchronize());
      RRF_CHECK_HIP(hipFree(c.ptr));
      c.ptr = nullptr;
      c.bytes = 0;
    }
    hipError_t e = fail_injected("alloc") ? hipErrorOutOfMemory : hipMalloc(&c.ptr, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      c.ptr = nullptr;
      return set_error(RRF_E_NOMEM, "device allocation of the workspace failed");
    }
    c.bytes = bytes;
  }
  *out = c.ptr;
  return RRF_OK;
}

// Read the status words written by the kernels (stream-ordered, synchronous).
int finish(hipStream_t st, const int* status_dev) {
  int h[2] = {0, 0};
  RRF_CHECK_HIP(hipMemcpyAsync(h, status_dev, sizeof h, hipMemcpyDeviceToHost, st));
  RRF_CHECK_HIP(hipStreamSynchronize(st));
  if (h[1] & 1) return set_error(RRF_E_NUMERIC, "input holds NaN or infinity");
  if (h[0] & 4) return set_error(RRF_E_INTERNAL, "panel kernel: grid barrier did not complete");
  if (h[0] & 2) return set_error(RRF_E_INTERNAL, "block SVD: Jacobi sweeps did not converge");
  if (h[0]) return set_error(RRF_E_INTERNAL, "device-side failure");
  return RRF_OK;
}

// Shared argument checks of rrf_randutv / rrf_powerurv (LAPACK numbering).
int check_args(int64_t m, int64_t n, const double* A, int64_t lda, int64_t b, int32_t q,
               const double* T, int shift = 0, bool allow_wide = false) {
  if (m < 1) return set_error(-1, "m must be >= 1"), -1;
  if (n < 1) return set_error(-2, "n must be >= 1"), -2;
  if (A == nullptr) return set_error(-3, "A is NULL"), -3;
  if (lda < m) return set_error(-4, "lda must be >= m"), -4;
  if (b < 1) return set_error(-5, "b must be >= 1"), -5;
  if (q < 0) return set_error(-6, "q must be >= 0"), -6;
  if (T == nullptr) return set_error(-9 - shift, "T is NULL"), -9 - shift;
  if (T == A && lda != m) return set_error(-4, "T may alias A only when lda == m"), -4;
  if (m < n && !allow_wide)
    return set_error(RRF_E_NOTSUP, "m < n is not supported here (factor A^T instead)");
  return RRF_OK;
}

// Bytes of the arena that factors the n x m transpose of a wide A (alg and
// boost_p as in run_alg), rounded; 0 outside the kernel limits.
size_t wide_arena(int alg, int64_t m, int64_t n, int64_t b, int32_t q, int precision,
                  int64_t boost_p = -1) {
  size_t w = 0;
  if (alg == RRF_ALG_RANDUTV)
    w = randutv_supported(n, m, b) ? randutv_workspace(n, m, b, precision, boost_p) : 0;
  else if (alg == RRF_ALG_POWERURV)
    w = powerurv_supported(n, m, b) ? powerurv_workspace(n, m, b, q, precision) : 0;
  return w == 0 ? 0 : (size_t)round_up((int64_t)w, 256);
}

// The wide path's whole workspace: the arena, then A^T and T^T (n x m each).
size_t wide_workspace(int alg, int64_t m, int64_t n, int64_t b, int32_t q, int precision,
                      int64_t boost_p = -1) {
  const size_t w = wide_arena(alg, m, n, b, q, precision, boost_p);
  return w == 0 ? 0 : w + (size_t)2 * round_up((int64_t)m * n * 8, 256);
}

// b + p <= 256 for Alg. 2 on an n-column input (p is clipped to n - b).
bool boosted_fits(int64_t n, int64_t b, int64_t p) {
  return std::min(b, n) + std::min(p, std::max<int64_t>(n - b, 0)) <= 256;
}

// Precision modes each algorithm implements (boost_p >= 0: Alg. 2, FP64 only).
bool precision_ok(int alg, int precision, int64_t boost_p = -1) {
  if (boost_p >= 0) return precision == RRF_PREC_FP64;
  if (precision == RRF_PREC_FP64 || precision == RRF_PREC_BF16_SKETCH) return true;
  return alg == RRF_ALG_RANDUTV &&
         (precision == RRF_PREC_BF16_X3 || precision == RRF_PREC_BF16_X6);
}

typedef bool (*SupportedFn)(int64_t, int64_t, int64_t);

// boost_p >= 0: randUTV_boosted with that oversampling (its argument list has
// p after q, so the pointer positions move by one).
template <typename Run>
int run_alg(int alg, int64_t m, int64_t n, const double* A, int64_t lda, int64_t b, int32_t q,
            double* U, double* T, double* V, const rrf_opts* opts, Run run,
            int64_t boost_p = -1, int ptr_shift = -1) {
  const int shift = ptr_shift >= 0 ? ptr_shift : (boost_p >= 0 ? 1 : 0);
  RRF_TRY(check_args(m, n, A, lda, b, q, T, shift));
  rrf_opts o;
  rrf_opts_init(&o);
  if (opts) o = *opts;
  if (boost_p >= 0) {
    if (o.precision != RRF_PREC_FP64)
      return set_error(RRF_E_NOTSUP, "randutv_boosted: only RRF_PREC_FP64");
    if (!boosted_fits(n, b, boost_p))
      return set_error(RRF_E_NOTSUP, "randutv_boosted: needs b + p <= 256");
  } else if (!precision_ok(alg, o.precision)) {
    return set_error(RRF_E_NOTSUP, "precision mode not implemented for this algorithm");
  }
  const bool ok = alg == RRF_ALG_RANDUTV ? randutv_supported(m, n, b) : powerurv_supported(m, n, b);
  if (!ok) return set_error(RRF_E_NOTSUP, "block size or shape outside the panel kernel limits");
  int dev = 0;
  RRF_TRY(device_ready(&dev));
  RRF_TRY(check_device_ptr(A, 3));
  RRF_TRY(check_device_ptr(U, 8 + shift));
  RRF_TRY(check_device_ptr(T, 9 + shift));
  RRF_TRY(check_device_ptr(V, 10 + shift));
  const size_t need = boost_p >= 0 ? randutv_workspace(m, n, b, RRF_PREC_FP64, boost_p)
                                   : rrf_workspace_size(alg, m, n, b, q, o.precision);
  if (need == 0) return set_error(RRF_E_NOTSUP, "shape outside the kernel limits");
  void* ws = o.workspace;
  size_t ws_bytes = o.workspace_bytes;
  if (ws == nullptr) {
    RRF_TRY(cached_workspace(dev, need, &ws));
    ws_bytes = need;
  } else if (ws_bytes < need) {
    return set_error(RRF_E_NOMEM, "workspace smaller than rrf_workspace_size()");
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(o.stream);
  if (o.check_finite) {
    // Reject non-finite input before any factorization work is enqueued
    // (this check synchronizes the stream, also in async mode).
    int* flag = reinterpret_cast<int*>(ws) + 1;
    RRF_TRY(fill_u32(st, reinterpret_cast<unsigned*>(flag), 1, 0u));
    RRF_TRY(check_finite(st, m, n, A, lda, flag));
    int h = 0;
    RRF_CHECK_HIP(hipMemcpyAsync(&h, flag, sizeof h, hipMemcpyDeviceToHost, st));
    RRF_CHECK_HIP(hipStreamSynchronize(st));
    if (h) return set_error(RRF_E_NUMERIC, "input holds NaN or infinity");
  }
  RRF_TRY(run(st, ws, ws_bytes, false));
  if (o.async) return RRF_OK;
  return finish(st, reinterpret_cast<const int*>(ws));
}

}  // namespace
}  // namespace rrf

using namespace rrf;

extern "C" {

void rrf_opts_init(rrf_opts* opts) {
  if (!opts) return;
  memset(opts, 0, sizeof *opts);
  opts->precision = RRF_PREC_FP64;
}

size_t rrf_workspace_size(int alg, int64_t m, int64_t n, int64_t b, int32_t q, int precision) {
  if (m < 1 || n < 1 || b < 1 || q < 0) return 0;
  if (alg != RRF_ALG_RANDUTV && alg != RRF_ALG_POWERURV) return 0;
  if (!precision_ok(alg, precision)) return 0;
  if (m < n) return wide_workspace(alg, m, n, b, q, precision);  // A^T's factorization
  if (alg == RRF_ALG_RANDUTV)
    return randutv_supported(m, n, b) ? randutv_workspace(m, n, b, precision) : 0;
  return powerurv_supported(m, n, b) ? powerurv_workspace(m, n, b, q, precision) : 0;
}

// m < n (Sec. 3.2: the paper factors the transpose): A^T = U' T' V'^T, so
// A = V' T'^T U'^T; U' is written to V, V' to U, and T = T'^T is lower
// trapezoidal. alg, boost_p and ptr_shift as in run_alg; stop as for
// randutv_run (a resumed state is the transpose's: T is transposed in, the
// caller's V continues U' and U continues V'); a_arg numbers A's pointer in
// error codes. thin_u does not apply (U is m x m = m x min(m, n) already).
static int wide_run(int alg, int64_t m, int64_t n, const double* A, int64_t lda, int64_t b,
                    int32_t q, uint64_t seed, double* U, double* T, double* V,
                    const rrf_opts* opts, int64_t boost_p = -1, const EarlyStop* stop = nullptr,
                    int ptr_shift = -1, int a_arg = 3) {
  const int shift = ptr_shift >= 0 ? ptr_shift : (boost_p >= 0 ? 1 : 0);
  RRF_TRY(check_args(m, n, A, lda, b, q, T, shift, true));
  rrf_opts o;
  rrf_opts_init(&o);
  if (opts) o = *opts;
  if (boost_p >= 0) {
    if (o.precision != RRF_PREC_FP64)
      return set_error(RRF_E_NOTSUP, "randutv_boosted: only RRF_PREC_FP64");
    if (!boosted_fits(m, b, boost_p))
      return set_error(RRF_E_NOTSUP, "randutv_boosted: needs b + p <= 256");
  } else if (!precision_ok(alg, o.precision)) {
    return set_error(RRF_E_NOTSUP, "precision mode not implemented for this algorithm");
  }
  const size_t arena = wide_arena(alg, m, n, b, q, o.precision, boost_p);
  if (arena == 0)
    return set_error(RRF_E_NOTSUP, "block size or shape outside the panel kernel limits");
  int dev = 0;
  RRF_TRY(device_ready(&dev));
  RRF_TRY(check_device_ptr(A, a_arg));
  RRF_TRY(check_device_ptr(U, 8 + shift));
  RRF_TRY(check_device_ptr(T, 9 + shift));
  RRF_TRY(check_device_ptr(V, 10 + shift));
  const size_t need = wide_workspace(alg, m, n, b, q, o.precision, boost_p);
  void* ws = o.workspace;
  size_t ws_bytes = o.workspace_bytes;
  if (ws == nullptr) {
    RRF_TRY(cached_workspace(dev, need, &ws));
    ws_bytes = need;
  } else if (ws_bytes < need) {
    return set_error(RRF_E_NOMEM, "workspace smaller than rrf_workspace_size()");
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(o.stream);
  double* At = reinterpret_cast<double*>(reinterpret_cast<char*>(ws) + arena);
  double* Tt = At + round_up((int64_t)m * n * 8, 256) / 8;
  if (o.check_finite) {
    int* flag = reinterpret_cast<int*>(ws) + 1;
    RRF_TRY(fill_u32(st, reinterpret_cast<unsigned*>(flag), 1, 0u));
    RRF_TRY(check_finite(st, m, n, A, lda, flag));
    int h = 0;
    RRF_CHECK_HIP(hipMemcpyAsync(&h, flag, sizeof h, hipMemcpyDeviceToHost, st));
    RRF_CHECK_HIP(hipStreamSynchronize(st));
    if (h) return set_error(RRF_E_NUMERIC, "input holds NaN or infinity");
  }
  RRF_TRY(transpose_matrix(st, m, n, A, lda, At, n));
  if (alg == RRF_ALG_RANDUTV) {
    int dummy = 0;
    RRF_TRY(randutv_run(st, n, m, At, n, b, q, seed, V, Tt, U, ws, arena, false, o.precision,
                        &dummy, boost_p, stop));
  } else {
    RRF_TRY(powerurv_run(st, n, m, At, n, b, q, seed, V, Tt, U, ws, arena, false, o.precision));
  }
  RRF_TRY(transpose_matrix(st, n, m, Tt, n, T, m));
  if (o.async) return RRF_OK;
  return finish(st, reinterpret_cast<const int*>(ws));
}

int rrf_randutv_ex(int64_t m, int64_t n, const double* A, int64_t lda, int64_t b, int32_t q,
                   uint64_t seed, double* U, double* T, double* V, const rrf_opts* opts) {
  if (m >= 1 && n >= 1 && m < n)
    return wide_run(RRF_ALG_RANDUTV, m, n, A, lda, b, q, seed, U, T, V, opts);
  return run_alg(RRF_ALG_RANDUTV, m, n, A, lda, b, q, U, T, V, opts,
                 [&](hipStream_t st, void* ws, size_t bytes, bool chk) {
                   int dummy = 0;
                   return randutv_run(st, m, n, A, lda, b, q, seed, U, T, V, ws, bytes, chk,
                                      opts ? opts->precision : RRF_PREC_FP64, &dummy, -1,
                                      nullptr, opts && opts->thin_u);
                 });
}

size_t rrf_randutv_boosted_workspace_size(int64_t m, int64_t n, int64_t b, int32_t q,
                                          int64_t p) {
  (void)q;
  if (m < 1 || n < 1 || b < 1 || q < 0 || p < 0) return 0;
  if (!boosted_fits(std::min(m, n), b, p)) return 0;
  if (m < n) return wide_workspace(RRF_ALG_RANDUTV, m, n, b, q, RRF_PREC_FP64, p);
  return randutv_supported(m, n, b) ? randutv_workspace(m, n, b, RRF_PREC_FP64, p) : 0;
}

int rrf_randutv_boosted_ex(int64_t m, int64_t n, const double* A, int64_t lda, int64_t b,
                           int32_t q, int64_t p, uint64_t seed, double* U, double* T, double* V,
                           const rrf_opts* opts) {
  if (p < 0) return set_error(-7, "p must be >= 0"), -7;
  if (m >= 1 && n >= 1 && m < n)
    return wide_run(RRF_ALG_RANDUTV, m, n, A, lda, b, q, seed, U, T, V, opts, p);
  return run_alg(RRF_ALG_RANDUTV, m, n, A, lda, b, q, U, T, V, opts,
                 [&](hipStream_t st, void* ws, size_t bytes, bool chk) {
                   int dummy = 0;
                   return randutv_run(st, m, n, A, lda, b, q, seed, U, T, V, ws, bytes, chk,
                                      RRF_PREC_FP64, &dummy, p, nullptr, opts && opts->thin_u);
                 },
                 p);
}

int rrf_randutv_boosted(int64_t m, int64_t n, const double* A, int64_t lda, int64_t b, int32_t q,
                        int64_t p, uint64_t seed, double* U, double* T, double* V) {
  return rrf_randutv_boosted_ex(m, n, A, lda, b, q, p, seed, U, T, V, nullptr);
}

int rrf_randutv_partial(int64_t m, int64_t n, const double* A, int64_t lda, int64_t b,
                        int32_t q, uint64_t seed, double tol, int64_t kmax, double* U, double* T,
                        double* V, int64_t* k_out, const rrf_opts* opts) {
  if (!(tol >= 0.0)) return set_error(-8, "tol must be >= 0"), -8;
  if (kmax < 0) return set_error(-9, "kmax must be >= 0"), -9;
  if (k_out == nullptr) return set_error(-13, "k_out is NULL"), -13;
  *k_out = 0;
  EarlyStop stop{tol, kmax, k_out, 0};
  rrf_opts o;
  rrf_opts_init(&o);
  if (opts) o = *opts;
  o.async = 0;  // the stopping test reads each step's norm on the host
  if (m >= 1 && n >= 1 && m < n)
    return wide_run(RRF_ALG_RANDUTV, m, n, A, lda, b, q, seed, U, T, V, &o, -1, &stop, 2);
  return run_alg(RRF_ALG_RANDUTV, m, n, A, lda, b, q, U, T, V, &o,
                 [&](hipStream_t st, void* ws, size_t bytes, bool chk) {
                   int dummy = 0;
                   return randutv_run(st, m, n, A, lda, b, q, seed, U, T, V, ws, bytes, chk,
                                      o.precision, &dummy, -1, &stop, o.thin_u != 0);
                 },
                 -1, 2);
}

int rrf_randutv_resume(int64_t m, int64_t n, int64_t b, int32_t q, uint64_t seed, double tol,
                       int64_t kmax, int64_t k_in, double* U, double* T, double* V, int64_t* k_out,
                       const rrf_opts* opts) {
  if (m < 1) return set_error(-1, "m must be >= 1"), -1;
  if (n < 1) return set_error(-2, "n must be >= 1"), -2;
  if (b < 1) return set_error(-3, "b must be >= 1"), -3;
  if (q < 0) return set_error(-4, "q must be >= 0"), -4;
  if (!(tol >= 0.0)) return set_error(-6, "tol must be >= 0"), -6;
  if (kmax < 0) return set_error(-7, "kmax must be >= 0"), -7;
  const int64_t kdim = std::min(m, n);  // m < n: the transpose's column count
  if (k_in < 0 || k_in > kdim || (k_in % b != 0 && k_in != kdim))
    return set_error(-8, "k_in must be a multiple of b in [0, min(m, n)] (or min(m, n))"), -8;
  if (T == nullptr) return set_error(-10, "T is NULL"), -10;
  if (k_out == nullptr) return set_error(-12, "k_out is NULL"), -12;
  *k_out = k_in;
  rrf_opts o;
  rrf_opts_init(&o);
  if (opts) o = *opts;
  if (o.thin_u) return set_error(RRF_E_NOTSUP, "resume needs the full m x m U");
  o.async = 0;
  if (k_in >= kdim) return RRF_OK;  // nothing left to reduce
  EarlyStop stop{tol, kmax, k_out, k_in / b};
  if (m < n)  // the state is the transpose's, T = T'^T (factored from a copy)
    return wide_run(RRF_ALG_RANDUTV, m, n, T, m, b, q, seed, U, T, V, &o, -1, &stop, 1, 10);
  // T holds the state and is factored in place (A = T, lda = m)
  return run_alg(RRF_ALG_RANDUTV, m, n, T, m, b, q, U, T, V, &o,
                 [&](hipStream_t st, void* ws, size_t bytes, bool chk) {
                   int dummy = 0;
                   return randutv_run(st, m, n, T, m, b, q, seed, U, T, V, ws, bytes, chk,
                                      o.precision, &dummy, -1, &stop, false);
                 },
                 -1, 1);
}

size_t rrf_rsvd_workspace_size(int64_t m, int64_t n, int64_t l, int32_t q) {
  if (m < 1 || n < 1 || q < 0 || !rsvd_supported(m, n, l)) return 0;
  return rsvd_workspace(m, n, l);
}

int rrf_rsvd(int64_t m, int64_t n, const double* A, int64_t lda, int64_t l, int32_t q,
             uint64_t seed, double* U, double* S, double* V, const rrf_opts* opts) {
  if (m < 1) return set_error(-1, "m must be >= 1"), -1;
  if (n < 1) return set_error(-2, "n must be >= 1"), -2;
  if (A == nullptr) return set_error(-3, "A is NULL"), -3;
  if (lda < m) return set_error(-4, "lda must be >= m"), -4;
  if (l < 1 || l > std::min(m, n)) return set_error(-5, "l must be in [1, min(m, n)]"), -5;
  if (q < 0) return set_error(-6, "q must be >= 0"), -6;
  if (S == nullptr) return set_error(-9, "S is NULL"), -9;
  if (!rsvd_supported(m, n, l)) return set_error(RRF_E_NOTSUP, "rsvd: needs l <= 256");
  rrf_opts o;
  rrf_opts_init(&o);
  if (opts) o = *opts;
  if (o.precision != RRF_PREC_FP64) return set_error(RRF_E_NOTSUP, "rsvd: only RRF_PREC_FP64");
  int dev = 0;
  RRF_TRY(device_ready(&dev));
  RRF_TRY(check_device_ptr(A, 3));
  RRF_TRY(check_device_ptr(U, 8));
  RRF_TRY(check_device_ptr(S, 9));
  RRF_TRY(check_device_ptr(V, 10));
  const size_t need = rsvd_workspace(m, n, l);
  void* ws = o.workspace;
  size_t ws_bytes = o.workspace_bytes;
  if (ws == nullptr) {
    RRF_TRY(cached_workspace(dev, need, &ws));
    ws_bytes = need;
  } else if (ws_bytes < need) {
    return set_error(RRF_E_NOMEM, "workspace smaller than rrf_rsvd_workspace_size()");
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(o.stream);
  RRF_TRY(rsvd_run(st, m, n, A, lda, l, q, seed, U, m, S, V, n, ws, ws_bytes, o.check_finite != 0));
  if (o.async) return RRF_OK;
  return finish(st, reinterpret_cast<const int*>(ws));
}

int rrf_randutv(int64_t m, int64_t n, const double* A, int64_t lda, int64_t b, int32_t q,
                uint64_t seed, double* U, double* T, double* V) {
  return rrf_randutv_ex(m, n, A, lda, b, q, seed, U, T, V, nullptr);
}

int64_t rrf_randutv_batched_block(int64_t m, int64_t n) {
  if (m < 1 || n < 1) return 0;
  return randutv_batched_block(std::max(m, n), std::min(m, n));  // m < n: the transpose's
}

}  // extern "C"

namespace rrf {
namespace {

// The batched call runs its matrices in groups, one lockstep run each: per
// configuration (block size, tile shapes and panel leaf: b, or the tuned or
// built-in choice for b = 0) and per orientation. A wide matrix (m < n)
// enters its group as its transpose (Sec. 3.2, as for rrf_randutv): A^T is
// copied into a buffer of its own after the runs' arena, factored there in
// place with U and V exchanged, and T = T'^T is copied back.
struct BatchedGroup {
  std::vector<int64_t> m, n;  // the factored shape (m >= n)
  std::vector<int64_t> idx;   // caller's matrix index
};

bool cfg_less(const BatchedCfg& x, const BatchedCfg& y) {
  if (x.b != y.b) return x.b < y.b;
  if (x.tile_mask != y.tile_mask) return x.tile_mask < y.tile_mask;
  return x.leaf < y.leaf;
}

std::vector<std::pair<BatchedCfg, BatchedGroup>> batched_groups(int64_t count, const int64_t* m,
                                                                const int64_t* n, int64_t b,
                                                                int precision) {
  std::vector<BatchedCfg> cfg(count);
  std::vector<BatchedCfg> distinct;
  for (int64_t j = 0; j < count; ++j) {
    const int64_t M = std::max(m[j], n[j]), N = std::min(m[j], n[j]);
    cfg[j] = b > 0 ? BatchedCfg{b, kTileMaskAll, 0} : batched_config(M, N, precision);
    bool seen = false;
    for (const auto& d : distinct)
      seen = seen || (!cfg_less(d, cfg[j]) && !cfg_less(cfg[j], d));
    if (!seen) distinct.push_back(cfg[j]);
  }
  std::sort(distinct.begin(), distinct.end(), cfg_less);
  std::vector<std::pair<BatchedCfg, BatchedGroup>> out;
  for (const auto& c : distinct)
    for (int wide = 0; wide < 2; ++wide) {
      BatchedGroup g;
      for (int64_t j = 0; j < count; ++j) {
        if ((m[j] < n[j]) != (wide == 1)) continue;
        if (cfg_less(cfg[j], c) || cfg_less(c, cfg[j])) continue;
        g.m.push_back(std::max(m[j], n[j]));
        g.n.push_back(std::min(m[j], n[j]));
        g.idx.push_back(j);
      }
      if (!g.idx.empty()) out.emplace_back(c, std::move(g));
    }
  return out;
}

size_t wide_copy_bytes(int64_t m, int64_t n) {
  return m < n ? (size_t)round_up(m * n * 8, 256) : 0;
}

// Arena of the largest group (0 if a group is outside the kernel limits).
size_t batched_arena(int64_t count, const int64_t* m, const int64_t* n, int64_t b, int precision) {
  size_t arena = 0;
  for (const auto& [cg, g] : batched_groups(count, m, n, b, precision)) {
    const size_t w = randutv_batched_workspace((int64_t)g.idx.size(), g.m.data(), g.n.data(), cg.b,
                                               precision);
    if (w == 0) return 0;
    arena = std::max(arena, w);
  }
  return arena;
}

}  // namespace
}  // namespace rrf

extern "C" {

size_t rrf_randutv_batched_workspace_size(int64_t count, const int64_t* m, const int64_t* n,
                                          int64_t b, int precision) {
  if (count <= 0 || m == nullptr || n == nullptr || b < 0 || b > kBatchedMaxB) return 0;
  if (precision != RRF_PREC_FP64 && precision != RRF_PREC_BF16_SKETCH) return 0;
  size_t wide = 0;
  for (int64_t j = 0; j < count; ++j) {
    if (m[j] < 1 || n[j] < 1 || std::max(m[j], n[j]) > kBatchedMaxDim) return 0;
    wide += wide_copy_bytes(m[j], n[j]);
  }
  const size_t arena = batched_arena(count, m, n, b, precision);
  if (arena == 0) return 0;
  return wide == 0 ? arena : (size_t)round_up((int64_t)arena, 256) + wide;
}

int rrf_randutv_batched(int64_t count, const int64_t* m, const int64_t* n,
                        const double* const* A, const int64_t* lda, int64_t b, int32_t q,
                        uint64_t seed, double* const* U, double* const* T, double* const* V,
                        const rrf_opts* opts) {
  if (count < 0) return set_error(-1, "count must be >= 0"), -1;
  if (count == 0) return RRF_OK;
  if (m == nullptr) return set_error(-2, "m is NULL"), -2;
  if (n == nullptr) return set_error(-3, "n is NULL"), -3;
  if (A == nullptr) return set_error(-4, "A is NULL"), -4;
  if (lda == nullptr) return set_error(-5, "lda is NULL"), -5;
  if (b < 0 || b > kBatchedMaxB) return set_error(-6, "b must be 0 or in [1, 64]"), -6;
  if (q < 0) return set_error(-7, "q must be >= 0"), -7;
  if (T == nullptr) return set_error(-10, "T is NULL"), -10;
  size_t wide_bytes = 0;
  for (int64_t j = 0; j < count; ++j) {
    if (m[j] < 1) return set_error(-2, "m[j] must be >= 1"), -2;
    if (n[j] < 1) return set_error(-3, "n[j] must be >= 1"), -3;
    if (A[j] == nullptr) return set_error(-4, "A[j] is NULL"), -4;
    if (lda[j] < m[j]) return set_error(-5, "lda[j] must be >= m[j]"), -5;
    if (U && U[j] == nullptr) return set_error(-9, "U[j] is NULL"), -9;
    if (T[j] == nullptr) return set_error(-10, "T[j] is NULL"), -10;
    if (V && V[j] == nullptr) return set_error(-11, "V[j] is NULL"), -11;
    if (T[j] == A[j] && lda[j] != m[j])
      return set_error(-5, "T[j] may alias A[j] only when lda[j] == m[j]"), -5;
    if (std::max(m[j], n[j]) > kBatchedMaxDim)
      return set_error(RRF_E_NOTSUP, "batched randutv: m or n above 4096 (use rrf_randutv)");
    wide_bytes += wide_copy_bytes(m[j], n[j]);
  }
  rrf_opts o;
  rrf_opts_init(&o);
  if (opts) o = *opts;
  if (o.precision != RRF_PREC_FP64 && o.precision != RRF_PREC_BF16_SKETCH)
    return set_error(RRF_E_NOTSUP, "batched randutv: precision mode not implemented");
  int dev = 0;
  RRF_TRY(device_ready(&dev));
  for (int64_t j = 0; j < count; ++j) {
    RRF_TRY(check_device_ptr(A[j], 4));
    if (U) RRF_TRY(check_device_ptr(U[j], 9));
    RRF_TRY(check_device_ptr(T[j], 10));
    if (V) RRF_TRY(check_device_ptr(V[j], 11));
  }
  const size_t need = rrf_randutv_batched_workspace_size(count, m, n, b, o.precision);
  if (need == 0) return set_error(RRF_E_NOTSUP, "batched randutv: sizes outside the kernel limits");
  void* ws = o.workspace;
  size_t ws_bytes = o.workspace_bytes;
  if (ws == nullptr) {
    RRF_TRY(cached_workspace(dev, need, &ws));
    ws_bytes = need;
  } else if (ws_bytes < need) {
    return set_error(RRF_E_NOMEM, "workspace smaller than rrf_randutv_batched_workspace_size()");
  }
  // the runs' arena first, then the transposed copies of the wide matrices
  const size_t arena_bytes = need - wide_bytes;
  std::vector<double*> Wt(count, nullptr);
  {
    char* base = reinterpret_cast<char*>(ws) + arena_bytes;
    for (int64_t j = 0; j < count; ++j) {
      if (m[j] >= n[j]) continue;
      Wt[j] = reinterpret_cast<double*>(base);
      base += wide_copy_bytes(m[j], n[j]);
    }
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(o.stream);
  int* status = reinterpret_cast<int*>(ws);
  RRF_TRY(fill_u32(st, reinterpret_cast<unsigned*>(status), 2, 0u));
  if (o.check_finite) {
    for (int64_t j = 0; j < count; ++j) RRF_TRY(check_finite(st, m[j], n[j], A[j], lda[j], status + 1));
    int h = 0;
    RRF_CHECK_HIP(hipMemcpyAsync(&h, status + 1, sizeof h, hipMemcpyDeviceToHost, st));
    RRF_CHECK_HIP(hipStreamSynchronize(st));
    if (h) return set_error(RRF_E_NUMERIC, "input holds NaN or infinity");
  }
  for (int64_t j = 0; j < count; ++j)
    if (Wt[j]) RRF_TRY(transpose_matrix(st, m[j], n[j], A[j], lda[j], Wt[j], n[j]));
  for (const auto& [cg, g] : batched_groups(count, m, n, b, o.precision)) {
    const int64_t cnt = (int64_t)g.idx.size();
    const bool wide = m[g.idx[0]] < n[g.idx[0]];
    // the factored matrix's U is the caller's V for a wide matrix, and vice versa
    double* const* Uf = wide ? V : U;
    double* const* Vf = wide ? U : V;
    std::vector<int64_t> gl(cnt);
    std::vector<const double*> gA(cnt);
    std::vector<double*> gU, gT(cnt), gV;
    std::vector<uint64_t> gs(cnt);
    for (int64_t t = 0; t < cnt; ++t) {
      const int64_t j = g.idx[t];
      gl[t] = wide ? n[j] : lda[j];
      gA[t] = wide ? Wt[j] : A[j];
      gT[t] = wide ? Wt[j] : T[j];
      if (Uf) gU.push_back(Uf[j]);
      if (Vf) gV.push_back(Vf[j]);
      gs[t] = seed + (uint64_t)j;  // matrix j is keyed by seed + j
    }
    RRF_TRY(randutv_batched_run(st, cnt, g.m.data(), g.n.data(), gA.data(), gl.data(), cg, q,
                                gs.data(), Uf ? gU.data() : nullptr, gT.data(),
                                Vf ? gV.data() : nullptr, ws, arena_bytes, o.precision,
                                !o.no_replay));
  }
  for (int64_t j = 0; j < count; ++j)
    if (Wt[j]) RRF_TRY(transpose_matrix(st, n[j], m[j], Wt[j], n[j], T[j], m[j]));
  if (o.async) return RRF_OK;
  return finish(st, status);
}

int rrf_powerurv_ex(int64_t m, int64_t n, const double* A, int64_t lda, int64_t b, int32_t q,
                    uint64_t seed, double* U, double* T, double* V, const rrf_opts* opts) {
  if (m >= 1 && n >= 1 && m < n)
    return wide_run(RRF_ALG_POWERURV, m, n, A, lda, b, q, seed, U, T, V, opts);
  return run_alg(RRF_ALG_POWERURV, m, n, A, lda, b, q, U, T, V, opts,
                 [&](hipStream_t st, void* ws, size_t bytes, bool chk) {
                   return powerurv_run(st, m, n, A, lda, b, q, seed, U, T, V, ws, bytes, chk,
                                       opts ? opts->precision : RRF_PREC_FP64);
                 });
}

int rrf_powerurv(int64_t m, int64_t n, const double* A, int64_t lda, int64_t b, int32_t q,
                 uint64_t seed, double* U, double* T, double* V) {
  return rrf_powerurv_ex(m, n, A, lda, b, q, seed, U, T, V, nullptr);
}

}  // extern "C"

// ---- allocation-free randUTV ------------------------------------------------
// A file-scope device array stands in for the workspace of rrf_randutv_noalloc.
// Its name is a host-side handle: host code only ever passes the device
// address that hipGetSymbolAddress returns for the current device, looked up
// once per device and kept in g_scratch.
namespace rrf {
namespace {
constexpr size_t kScratchBytes = (size_t)RRF_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
std::unordered_map<int, void*> g_scratch;

// Device address of `scratch` on device `dev` (current); the first call on a
// device also creates the side streams and events the drivers use there.
int scratch_pointer(int dev, void** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch.find(dev);
  if (it != g_scratch.end()) {
    *out = it->second;
    return RRF_OK;
  }
  void* p = nullptr;
  RRF_CHECK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (p == nullptr) return set_error(RRF_E_HIP, "no device address for the static scratch");
  DeviceContext* ctx = nullptr;
  RRF_TRY(device_context(&ctx));
  g_scratch[dev] = p;
  *out = p;
  return RRF_OK;
}
}  // namespace
}  // namespace rrf

extern "C" {

int rrf_randutv_noalloc(int64_t m, int64_t n, const double* A, int64_t lda, int64_t b,
                        int32_t q, uint64_t seed, double* U, double* T, double* V,
                        const rrf_opts* opts) {
  rrf_opts o;
  rrf_opts_init(&o);
  if (opts) o = *opts;
  if (o.workspace != nullptr || o.workspace_bytes != 0)
    return set_error(-11, "rrf_randutv_noalloc takes no workspace (opts->workspace must be "
                          "NULL); use rrf_randutv_ex to pass one"), -11;
  RRF_TRY(check_args(m, n, A, lda, b, q, T, 0, true));
  const size_t need = rrf_workspace_size(RRF_ALG_RANDUTV, m, n, b, q, o.precision);
  if (need == 0)
    return set_error(RRF_E_NOTSUP, "block size, shape or precision outside the kernel limits");
  if (need > kScratchBytes) {
    char buf[256];
    snprintf(buf, sizeof buf,
             "rrf_randutv_noalloc: this factorization needs %zu bytes of scratch, more than "
             "the static %zu (use rrf_randutv_ex with a workspace)", need, kScratchBytes);
    return set_error(RRF_E_NOMEM, buf);
  }
  int dev = 0;
  RRF_TRY(device_ready(&dev));
  void* p = nullptr;
  RRF_TRY(scratch_pointer(dev, &p));
  o.workspace = p;
  o.workspace_bytes = kScratchBytes;
  return rrf_randutv_ex(m, n, A, lda, b, q, seed, U, T, V, &o);
}

int rrf_release_workspace(void) {
  int dev = 0;
  RRF_TRY(device_ready(&dev));
  RRF_TRY(randutv_batched_release());
  std::lock_guard<std::mutex> lk(g_cache_mu);
  auto it = g_cache.find(dev);
  if (it != g_cache.end() && it->second.ptr) {
    RRF_CHECK_HIP(hipDeviceSynchronize());
    RRF_CHECK_HIP(hipFree(it->second.ptr));
    g_cache.erase(it);
  }
  return RRF_OK;
}

int rrf_gaussian(uint64_t seed, uint64_t stream_id, int64_t rows, int64_t cols, double* out,
                 int64_t ld, void* stream) {
  if (rows < 0) return set_error(-3, "rows must be >= 0"), -3;
  if (cols < 0) return set_error(-4, "cols must be >= 0"), -4;
  if (out == nullptr && rows > 0 && cols > 0) return set_error(-5, "out is NULL"), -5;
  if (ld < (rows > 1 ? rows : 1)) return set_error(-6, "ld must be >= rows"), -6;
  int dev = 0;
  RRF_TRY(device_ready(&dev));
  return gaussian(reinterpret_cast<hipStream_t>(stream), seed, stream_id, rows, cols, out, ld);
}

int rrf_sketch_uniforms(uint64_t seed, uint64_t stream_id, int64_t rows, int64_t cols,
                        double* out, int64_t ld, void* stream) {
  if (rows < 0) return set_error(-3, "rows must be >= 0"), -3;
  if (cols < 0) return set_error(-4, "cols must be >= 0"), -4;
  if (out == nullptr && rows > 0 && cols > 0) return set_error(-5, "out is NULL"), -5;
  if (ld < (rows > 1 ? rows : 1)) return set_error(-6, "ld must be >= rows"), -6;
  int dev = 0;
  RRF_TRY(device_ready(&dev));
  return sketch_uniforms(reinterpret_cast<hipStream_t>(stream), seed, stream_id, rows, cols, out,
                         ld);
}

static int gemm_entry(GemmFn fn, int transa, int transb, int64_t M, int64_t N, int64_t K,
                      double alpha, const double* A, int64_t lda, const double* B, int64_t ldb,
                      double beta, double* C, int64_t ldc, void* work, size_t work_bytes,
                      void* stream) {
  if (transa != 0 && transa != 1) return set_error(-1, "transa must be 0 or 1"), -1;
  if (transb != 0 && transb != 1) return set_error(-2, "transb must be 0 or 1"), -2;
  if (M < 0) return set_error(-3, "M must be >= 0"), -3;
  if (N < 0) return set_error(-4, "N must be >= 0"), -4;
  if (K < 0) return set_error(-5, "K must be >= 0"), -5;
  const int64_t arows = transa ? K : M, brows = transb ? N : K;
  if (K > 0 && M > 0 && A == nullptr) return set_error(-7, "A is NULL"), -7;
  if (lda < (arows > 1 ? arows : 1)) return set_error(-8, "lda too small"), -8;
  if (K > 0 && N > 0 && B == nullptr) return set_error(-9, "B is NULL"), -9;
  if (ldb < (brows > 1 ? brows : 1)) return set_error(-10, "ldb too small"), -10;
  if (M > 0 && N > 0 && C == nullptr) return set_error(-12, "C is NULL"), -12;
  if (ldc < (M > 1 ? M : 1)) return set_error(-13, "ldc too small"), -13;
  int dev = 0;
  RRF_TRY(device_ready(&dev));
  return fn(reinterpret_cast<hipStream_t>(stream), transa != 0, transb != 0, M, N, K, alpha, A, lda,
            B, ldb, beta, C, ldc, reinterpret_cast<double*>(work), work_bytes / 8);
}

int rrf_dgemm(int transa, int transb, int64_t M, int64_t N, int64_t K, double alpha,
              const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
              int64_t ldc, void* work, size_t work_bytes, void* stream) {
  return gemm_entry(dgemm, transa, transb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, work,
                    work_bytes, stream);
}

int rrf_gemm_x3(int transa, int transb, int64_t M, int64_t N, int64_t K, double alpha,
                const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                double* C, int64_t ldc, void* work, size_t work_bytes, void* stream) {
  return gemm_entry(gemm_x3, transa, transb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, work,
                    work_bytes, stream);
}

int rrf_gemm_x6(int transa, int transb, int64_t M, int64_t N, int64_t K, double alpha,
                const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                double* C, int64_t ldc, void* work, size_t work_bytes, void* stream) {
  return gemm_entry(gemm_x6, transa, transb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, work,
                    work_bytes, stream);
}

size_t rrf_panel_workspace_size(int64_t M, int64_t k) {
  if (k < 1 || k > 256 || M < k) return 0;
  const size_t w = panel_work_bytes(M, (int)k);
  return w == 0 ? 0 : w + 256;
}

int rrf_householder_panel(int64_t M, int64_t k, double* P, int64_t ldp, double* W, int64_t ldw,
                          double* R, int64_t ldr, double* Tf, int64_t ldt, double* tau,
                          void* work, size_t work_bytes, void* stream) {
  if (k < 1 || k > 256) return set_error(-2, "k must be in [1, 256]"), -2;
  if (M < k) return set_error(-1, "M must be >= k"), -1;
  if (P == nullptr) return set_error(-3, "P is NULL"), -3;
  if (ldp < M) return set_error(-4, "ldp must be >= M"), -4;
  if (W == nullptr) return set_error(-5, "W is NULL"), -5;
  if (ldw < M) return set_error(-6, "ldw must be >= M"), -6;
  if (W == P && ldw != ldp) return set_error(-6, "W may alias P only with ldw == ldp"), -6;
  if (R != nullptr && ldr < k) return set_error(-8, "ldr must be >= k"), -8;
  if (Tf == nullptr) return set_error(-9, "Tf is NULL"), -9;
  if (ldt < k) return set_error(-10, "ldt must be >= k"), -10;
  if (tau == nullptr) return set_error(-11, "tau is NULL"), -11;
  const size_t need = rrf_panel_workspace_size(M, k);
  if (need == 0) return set_error(RRF_E_NOTSUP, "panel too large for one launch");
  if (work == nullptr || work_bytes < need)
    return set_error(RRF_E_NOMEM, "work smaller than rrf_panel_workspace_size()");
  int dev = 0;
  RRF_TRY(device_ready(&dev));
  // status word in the first 256 bytes of work; the panel scratch follows it
  int* status = reinterpret_cast<int*>(work);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  RRF_TRY(fill_u32(st, reinterpret_cast<unsigned*>(status), 1, 0u));
  return householder_panel(st, M, (int)k, P, ldp, W, ldw, R, ldr, Tf, ldt, tau, nullptr, 0,
                           reinterpret_cast<char*>(work) + 256, work_bytes - 256, status);
}

int rrf_to_bf16(int64_t rows, int64_t cols, const double* X, int64_t ldx, int scaled,
                uint16_t* out, int64_t ldo, uint16_t* outT, int64_t ldot, void* work,
                size_t work_bytes, void* stream) {
  if (rows < 0) return set_error(-1, "rows must be >= 0"), -1;
  if (cols < 0) return set_error(-2, "cols must be >= 0"), -2;
  if (rows > 0 && cols > 0 && X == nullptr) return set_error(-3, "X is NULL"), -3;
  if (ldx < (rows > 1 ? rows : 1)) return set_error(-4, "ldx too small"), -4;
  if (rows > 0 && cols > 0 && out == nullptr) return set_error(-6, "out is NULL"), -6;
  if (ldo < rows || (ldo & 7)) return set_error(-7, "ldo must be >= rows and a multiple of 8"), -7;
  if (outT && (ldot < cols || (ldot & 7)))
    return set_error(-9, "ldot must be >= cols and a multiple of 8"), -9;
  if (work == nullptr || work_bytes < 256) return set_error(-10, "work needs 256 bytes"), -10;
  int dev = 0;
  RRF_TRY(device_ready(&dev));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  unsigned long long* word = reinterpret_cast<unsigned long long*>(work);
  if (scaled) RRF_TRY(maxabs(st, rows, cols, X, ldx, word));
  return to_bf16(st, rows, cols, X, ldx, scaled ? word : nullptr, out, ldo, outT, ldot);
}

size_t rrf_gemm_bf16_workspace_size(int64_t M, int64_t N) {
  if (M < 1 || N < 1) return 0;
  return gemm_bf16_work_bytes(M, N);
}

int rrf_gemm_bf16_tn(int64_t M, int64_t N, int64_t K, const uint16_t* A, int64_t lda,
                     const uint16_t* B, int64_t ldb, uint16_t* out16, int64_t ld16,
                     double* out64, int64_t ld64, void* work, size_t work_bytes, void* stream) {
  if (M < 1) return set_error(-1, "M must be >= 1"), -1;
  if (N < 1) return set_error(-2, "N must be >= 1"), -2;
  if (K < 0) return set_error(-3, "K must be >= 0"), -3;
  if (K > 0 && A == nullptr) return set_error(-4, "A is NULL"), -4;
  if (lda < K || (lda & 7)) return set_error(-5, "lda must be >= K and a multiple of 8"), -5;
  if (K > 0 && B == nullptr) return set_error(-6, "B is NULL"), -6;
  if (ldb < K || (ldb & 7)) return set_error(-7, "ldb must be >= K and a multiple of 8"), -7;
  if (out16 == nullptr && out64 == nullptr) return set_error(-8, "no output"), -8;
  if (out16 && (ld16 < M || (ld16 & 7)))
    return set_error(-9, "ld16 must be >= M and a multiple of 8"), -9;
  if (!out16 && ld64 < M) return set_error(-11, "ld64 must be >= M"), -11;
  if (work == nullptr || work_bytes < gemm_bf16_work_bytes(M, N))
    return set_error(RRF_E_NOMEM, "work smaller than rrf_gemm_bf16_workspace_size()");
  if (K > 0 && ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B)) & 15))
    return set_error(RRF_E_NOTSUP, "A and B must be 16-byte aligned");
  int dev = 0;
  RRF_TRY(device_ready(&dev));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  return gemm_bf16_tn(st, M, N, K, A, lda, B, ldb, out16, ld16, out16 ? nullptr : out64, ld64,
                      work, work_bytes);
}

size_t rrf_block_svd_workspace_size(int64_t k) {
  if (k < 1 || k > 256) return 0;
  return block_svd_work_bytes((int)k) + 256;
}

int rrf_block_svd(int64_t k, const double* B, int64_t ldb, double* Us, double* d, double* Vs,
                  void* work, size_t work_bytes, void* stream) {
  if (k < 1 || k > 256) return set_error(-1, "k must be in [1, 256]"), -1;
  if (B == nullptr) return set_error(-2, "B is NULL"), -2;
  if (ldb < k) return set_error(-3, "ldb must be >= k"), -3;
  if (Us == nullptr) return set_error(-4, "Us is NULL"), -4;
  if (d == nullptr) return set_error(-5, "d is NULL"), -5;
  if (Vs == nullptr) return set_error(-6, "Vs is NULL"), -6;
  const size_t need = rrf_block_svd_workspace_size(k);
  if (work == nullptr || work_bytes < need)
    return set_error(RRF_E_NOMEM, "work smaller than rrf_block_svd_workspace_size()");
  int dev = 0;
  RRF_TRY(device_ready(&dev));
  int* status = reinterpret_cast<int*>(work);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  RRF_TRY(fill_u32(st, reinterpret_cast<unsigned*>(status), 1, 0u));
  return block_svd(st, (int)k, B, ldb, Us, d, Vs, reinterpret_cast<char*>(work) + 256,
                   work_bytes - 256, status);
}

const char* rrf_status_string(int status) {
  switch (status) {
    case RRF_OK: return "success";
    case RRF_E_HIP: return "HIP runtime or kernel failure";
    case RRF_E_NOMEM: return "workspace too small or device allocation failed";
    case RRF_E_NOTSUP: return "request outside what is implemented";
    case RRF_E_NUMERIC: return "non-finite input";
    case RRF_E_INTERNAL: return "device-side consistency check failed";
    default: return status < 0 ? "invalid argument" : "unknown status";
  }
}

const char* rrf_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
