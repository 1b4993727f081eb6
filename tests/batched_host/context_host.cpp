// Host check of allow_dynamic_lds (context.hip), built with the host
// compiler: the HIP calls it makes are stubbed (a current device per thread,
// and a log of every hipFuncSetAttribute call, which fails for more than
// 160 KiB). Eight threads call it concurrently for two kernels on three
// devices with two sizes; then a request beyond the limit fails, leaves the
// kernel's allowance as it was, and a smaller request still succeeds. Prints
// one line per logged call, "<kernel> <device> <bytes>", in call order per
// (kernel, device), then "failed <status>" and "after <status>".
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <mutex>
#include <thread>
#include <tuple>
#include <vector>

#include "common.hpp"
#include "context.hpp"

static thread_local int t_dev = 0;
static std::mutex g_log_mu;
static std::vector<std::tuple<const void*, int, int>> g_log;

hipError_t hipGetDevice(int* d) {
  *d = t_dev;
  return hipSuccess;
}
hipError_t hipSetDevice(int d) {
  t_dev = d;
  return hipSuccess;
}
hipError_t hipFuncSetAttribute(const void* f, hipFuncAttribute attr, int value) {
  if (attr != hipFuncAttributeMaxDynamicSharedMemorySize || value > 160 * 1024)
    return hipErrorInvalidValue;
  std::lock_guard<std::mutex> lk(g_log_mu);
  g_log.emplace_back(f, t_dev, value);
  return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t*, unsigned) { return hipErrorNotSupported; }
hipError_t hipEventCreateWithFlags(hipEvent_t*, unsigned) { return hipErrorNotSupported; }
const char* hipGetErrorString(hipError_t) { return "stub"; }

namespace rrf {
int set_hip_error(hipError_t, const char*, const char*, int) { return RRF_E_HIP; }
int set_error(int status, const char*) { return status; }
}  // namespace rrf

static char k0, k1, k2;  // stand-ins for kernel addresses

int main() {
  std::vector<std::thread> threads;
  for (int t = 0; t < 8; ++t)
    threads.emplace_back([t]() {
      for (int it = 0; it < 2000; ++it) {
        (void)hipSetDevice((t + it) % 3);
        const size_t bytes = (it + t) % 5 == 0 ? 128 * 1024 : 64 * 1024;
        if (rrf::allow_dynamic_lds((it & 1) ? &k1 : &k0, bytes) != 0) printf("unexpected\n");
      }
    });
  for (auto& th : threads) th.join();
  for (const void* k : {(const void*)&k0, (const void*)&k1})
    for (int d = 0; d < 3; ++d)
      for (const auto& [f, dev, v] : g_log)
        if (f == k && dev == d) printf("%d %d %d\n", k == &k0 ? 0 : 1, d, v);
  (void)hipSetDevice(1);
  printf("failed %d\n", rrf::allow_dynamic_lds(&k2, 200 * 1024));
  printf("after %d\n", rrf::allow_dynamic_lds(&k2, 100 * 1024));
  for (const auto& [f, dev, v] : g_log)
    if (f == &k2) printf("2 %d %d\n", dev, v);
  return 0;
}
