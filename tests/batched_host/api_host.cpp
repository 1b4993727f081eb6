// Host harness of the library's own C ABI (api.hip: argument checks,
// workspace management, grouping by configuration and orientation) for the
// batched call and its autotuner (autotune.hip), built with the host compiler
// and linked with the batched driver and its test double (mock_kernels.cpp).
// HIP events report made-up but deterministic times, so the autotuner's
// search runs its whole course (install a candidate, record, replay, time,
// keep the fastest) with no device. Entry points the batched path never
// reaches are stubs that fail.
//
//   api_host <cache> workload <count> <nhi>   tune on `count` matrices with n
//                                             in [1, nhi] (m in [n/2, 2n])
//   api_host <cache> buckets <count> <nmax>   tune the synthetic buckets
//   api_host - batched <count> <nhi>          rrf_randutv_batched on such a
//                                             batch with the library-managed
//                                             workspace, under the caller's
//                                             environment, then again with
//                                             RRF_TEST_FAIL unset
//
// Output of the tuning modes: "autotune <rc> <mock errors>", then the
// configurations for n = 1..8 and 64 as tuned, after an unload (the built-in
// rule), and after loading the cache the search wrote. Of the batched mode:
// "batched <rc> <mock errors> <device property queries so far>" for each call.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "driver.hpp"
#include "kernels.hpp"
#include "rrf.h"

extern "C" long mock_errors();

static long g_prop_queries = 0;
hipError_t hipGetDeviceProperties(hipDeviceProp_t* prop, int) {
  ++g_prop_queries;
  memset(prop, 0, sizeof *prop);
  strcpy(prop->gcnArchName, "gfx950:sramecc+:xnack-");
  return hipSuccess;
}
hipError_t hipGetLastError() { return hipSuccess; }
hipError_t hipGetDeviceCount(int* c) {
  *c = 1;
  return hipSuccess;
}
hipError_t hipPointerGetAttributes(hipPointerAttribute_t* a, const void*) {
  memset(a, 0, sizeof *a);
  a->type = hipMemoryTypeDevice;
  return hipSuccess;
}
hipError_t hipGetSymbolAddress(void** p, const void* symbol) {
  *p = const_cast<void*>(symbol);
  return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t* e) {
  *e = (hipEvent_t)malloc(8);
  return hipSuccess;
}
static long g_timings = 0;
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  *ms = 1.0f + (float)((++g_timings * 7919) % 13) / 10.0f;
  return hipSuccess;
}

namespace rrf {
#define RRF_STUB return set_error(RRF_E_NOTSUP, "not part of the host harness")
int gaussian(hipStream_t, uint64_t key, uint64_t ctr, int64_t m, int64_t n, double* a,
             int64_t lda) {
  uint64_t x = key * 6364136223846793005ull + ctr;
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = 0; i < m; ++i) {
      x = x * 6364136223846793005ull + 1442695040888963407ull;
      a[i + j * lda] = (double)(x >> 11) / 9007199254740992.0 - 0.5;
    }
  return RRF_OK;
}
int check_finite(hipStream_t, int64_t, int64_t, const double*, int64_t, int*) { return RRF_OK; }
int transpose_matrix(hipStream_t, int64_t m, int64_t n, const double* A, int64_t lda, double* B,
                     int64_t ldb) {
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = 0; i < m; ++i) B[j + i * ldb] = A[i + j * lda];
  return RRF_OK;
}
int randutv_run(hipStream_t, int64_t, int64_t, const double*, int64_t, int64_t, int, uint64_t,
                double*, double*, double*, void*, size_t, bool, int, int*, int64_t,
                const EarlyStop*, bool) { RRF_STUB; }
int powerurv_run(hipStream_t, int64_t, int64_t, const double*, int64_t, int64_t, int, uint64_t,
                 double*, double*, double*, void*, size_t, bool, int) { RRF_STUB; }
int rsvd_run(hipStream_t, int64_t, int64_t, const double*, int64_t, int64_t, int, uint64_t,
             double*, int64_t, double*, double*, int64_t, void*, size_t, bool) { RRF_STUB; }
bool randutv_supported(int64_t, int64_t, int64_t) { return false; }
bool powerurv_supported(int64_t, int64_t, int64_t) { return false; }
bool rsvd_supported(int64_t, int64_t, int64_t) { return false; }
size_t randutv_workspace(int64_t, int64_t, int64_t, int, int64_t) { return 0; }
size_t powerurv_workspace(int64_t, int64_t, int64_t, int, int) { return 0; }
size_t rsvd_workspace(int64_t, int64_t, int64_t) { return 0; }
size_t panel_work_bytes(int64_t, int) { return 0; }
size_t gemm_bf16_work_bytes(int64_t, int64_t) { return 0; }
int sketch_uniforms(hipStream_t, uint64_t, uint64_t, int64_t, int64_t, double*, int64_t) {
  RRF_STUB;
}
int householder_panel(hipStream_t, int64_t, int, const double*, int64_t, double*, int64_t,
                      double*, int64_t, double*, int64_t, double*, double*, int64_t, void*,
                      size_t, int*) { RRF_STUB; }
int block_svd(hipStream_t, int, const double*, int64_t, double*, double*, double*, void*, size_t,
              int*) { RRF_STUB; }
int dgemm(hipStream_t, bool, bool, int64_t, int64_t, int64_t, double, const double*, int64_t,
          const double*, int64_t, double, double*, int64_t, double*, size_t) { RRF_STUB; }
int gemm_x3(hipStream_t, bool, bool, int64_t, int64_t, int64_t, double, const double*, int64_t,
            const double*, int64_t, double, double*, int64_t, double*, size_t) { RRF_STUB; }
int gemm_x6(hipStream_t, bool, bool, int64_t, int64_t, int64_t, double, const double*, int64_t,
            const double*, int64_t, double, double*, int64_t, double*, size_t) { RRF_STUB; }
int gemm_bf16_tn(hipStream_t, int64_t, int64_t, int64_t, const uint16_t*, int64_t,
                 const uint16_t*, int64_t, uint16_t*, int64_t, double*, int64_t, void*, size_t) {
  RRF_STUB;
}
int maxabs(hipStream_t, int64_t, int64_t, const double*, int64_t, unsigned long long*) {
  RRF_STUB;
}
int to_bf16(hipStream_t, int64_t, int64_t, const double*, int64_t, const unsigned long long*,
            uint16_t*, int64_t, uint16_t*, int64_t) { RRF_STUB; }
}  // namespace rrf

static void lookups(const char* tag) {
  printf("%s", tag);
  for (int64_t n : {1, 2, 3, 4, 5, 6, 7, 8, 64}) {
    rrf_batched_cfg c{};
    const int s = rrf_batched_config(n, n, RRF_PREC_FP64, &c);
    printf(" %d:%lld,%d,%d,%d", s, (long long)c.b, c.tile_mask, c.leaf, c.tuned);
  }
  printf("\n");
}

int main(int argc, char** argv) {
  if (argc != 5) return 2;
  const char* cache = argv[1];
  const bool workload = strcmp(argv[2], "workload") == 0;
  const bool batched = strcmp(argv[2], "batched") == 0;
  const int64_t count = atoll(argv[3]), hi = atoll(argv[4]);
  std::vector<int64_t> m(count), n(count);
  uint64_t x = 12345;
  for (int64_t j = 0; j < count; ++j) {  // n in [1, hi]; m in [n/2, 2n]: some wide matrices
    x = x * 6364136223846793005ull + 1442695040888963407ull;
    n[j] = 1 + (int64_t)((x >> 33) % (uint64_t)hi);
    x = x * 6364136223846793005ull + 1442695040888963407ull;
    const int64_t lo = n[j] / 2 > 0 ? n[j] / 2 : 1;
    m[j] = lo + (int64_t)((x >> 33) % (uint64_t)(2 * n[j] - lo + 1));
  }
  if (batched) {
    std::vector<double*> A(count), T(count), U(count), V(count);
    std::vector<const double*> Ac(count);
    for (int64_t j = 0; j < count; ++j) {
      void* p = nullptr;
      (void)hipMalloc(&p, 8 * (size_t)(m[j] * n[j] + 2 * m[j] * n[j] + m[j] * m[j] + n[j] * n[j]));
      A[j] = static_cast<double*>(p);
      T[j] = A[j] + m[j] * n[j];
      U[j] = T[j] + m[j] * n[j];
      V[j] = U[j] + m[j] * m[j];
      Ac[j] = A[j];
      (void)rrf::gaussian(nullptr, 7, (uint64_t)j, m[j], n[j], A[j], m[j]);
    }
    for (int call = 0; call < 2; ++call) {
      if (call == 1) unsetenv("RRF_TEST_FAIL");
      const int rc = rrf_randutv_batched(count, m.data(), n.data(), Ac.data(), m.data(), 0, 1, 7,
                                         U.data(), T.data(), V.data(), nullptr);
      printf("batched %d %ld %ld\n", rc, mock_errors(), g_prop_queries);
    }
    for (int64_t j = 0; j < count; ++j) (void)hipFree(A[j]);
    return rrf_release_workspace() == 0 ? 0 : 3;
  }
  const int rc = workload ? rrf_batched_autotune(RRF_PREC_FP64, 1, count, m.data(), n.data(),
                                                 1024, 7, cache, nullptr)
                          : rrf_batched_autotune(RRF_PREC_FP64, 1, count, nullptr, nullptr, hi,
                                                 7, cache, nullptr);
  printf("autotune %d %ld\n", rc, mock_errors());
  if (rc != 0) {
    printf("%s\n", rrf_last_error());
    return 0;
  }
  lookups("tuned");
  const int u = rrf_batched_tune_load(nullptr);
  lookups(u == 0 ? "builtin" : "unload-failed");
  const int l = rrf_batched_tune_load(cache);
  lookups(l == 0 ? "loaded" : "load-failed");
  const int r = rrf_release_workspace();
  return r == 0 ? 0 : 3;
}
