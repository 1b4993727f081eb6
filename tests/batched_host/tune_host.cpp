// Host harness of the batched call's tuning cache (autotune.hip), built with
// the host compiler and linked with the batched driver and its test double
// (mock_kernels.cpp): loads every cache file named on the command line with
// rrf_batched_tune_load and, after each, looks up the configuration of a few
// sizes with rrf_batched_config. The argument NULL unloads the tables (a null
// path); --lookup only looks up (a first lookup loads $RRF_TUNE_CACHE). One
// line per argument:
//   <status> <status:b,tile_mask,leaf,tuned for n = 1, 40, 64, 65, 300, 512, 4096>
// The device reports gfx950, so loaded gfx950 tables are used by lookups.
// The tuning search itself (gaussian batches, timed calls) is not reached:
// its entry points are stubs that fail.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>

#include "driver.hpp"
#include "kernels.hpp"
#include "rrf.h"

hipError_t hipGetDeviceProperties(hipDeviceProp_t* prop, int) {
  memset(prop, 0, sizeof *prop);
  strcpy(prop->gcnArchName, "gfx950:sramecc+:xnack-");
  return hipSuccess;
}
hipError_t hipGetLastError() { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t*) { return hipErrorNotSupported; }
hipError_t hipEventElapsedTime(float*, hipEvent_t, hipEvent_t) { return hipErrorNotSupported; }

namespace rrf {
int gaussian(hipStream_t, uint64_t, uint64_t, int64_t, int64_t, double*, int64_t) {
  return set_error(RRF_E_NOTSUP, "tuning search not available in the host harness");
}
}  // namespace rrf

extern "C" {
void rrf_opts_init(rrf_opts* o) { memset(o, 0, sizeof *o); }
size_t rrf_randutv_batched_workspace_size(int64_t, const int64_t*, const int64_t*, int64_t, int) {
  return 0;
}
int rrf_randutv_batched(int64_t, const int64_t*, const int64_t*, const double* const*,
                        const int64_t*, int64_t, int32_t, uint64_t, double* const*, double* const*,
                        double* const*, const rrf_opts*) {
  return RRF_E_NOTSUP;
}
}

int main(int argc, char** argv) {
  const int64_t ns[] = {1, 40, 64, 65, 300, 512, 4096};
  for (int i = 1; i < argc; ++i) {
    const bool lookup_only = strcmp(argv[i], "--lookup") == 0;
    const int rc =
        lookup_only ? 0 : rrf_batched_tune_load(strcmp(argv[i], "NULL") == 0 ? nullptr : argv[i]);
    printf("%d", rc);
    for (int64_t n : ns) {
      rrf_batched_cfg c{};
      const int s = rrf_batched_config(n, n, RRF_PREC_FP64, &c);
      printf(" %d:%lld,%d,%d,%d", s, (long long)c.b, c.tile_mask, c.leaf, c.tuned);
    }
    printf("\n");
  }
  return 0;
}
