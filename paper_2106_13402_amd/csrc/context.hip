// Per-device execution context: the streams and events the drivers use to
// overlap independent work with the critical path. Created on first use
// and kept for the life of the process; every stream has the default
// priority and does not synchronize with the null stream.
#include <map>
#include <mutex>
#include <unordered_map>
#include <utility>

#include "common.hpp"
#include "context.hpp"

namespace rrf {

namespace {
std::mutex g_mu;
std::unordered_map<int, DeviceContext*> g_ctx;
std::mutex g_lds_mu;
std::map<std::pair<const void*, int>, size_t> g_lds;  // (kernel, device) -> bytes allowed
}  // namespace

int allow_dynamic_lds(const void* kernel, size_t bytes) {
  int dev = 0;
  RRF_CHECK_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_lds_mu);
  size_t& allowed = g_lds[{kernel, dev}];
  if (allowed >= bytes) return RRF_OK;
  RRF_CHECK_HIP(
      hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  allowed = bytes;
  return RRF_OK;
}

int device_context(DeviceContext** out) {
  int dev = 0;
  RRF_CHECK_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_ctx.find(dev);
  if (it != g_ctx.end()) {
    *out = it->second;
    return RRF_OK;
  }
  DeviceContext* c = new DeviceContext();
  for (int i = 0; i < kSideStreams; ++i)
    RRF_CHECK_HIP(hipStreamCreateWithFlags(&c->side[i], hipStreamNonBlocking));
  for (int i = 0; i < kCtxEvents; ++i)
    RRF_CHECK_HIP(hipEventCreateWithFlags(&c->ev[i], hipEventDisableTiming));
  g_ctx[dev] = c;
  *out = c;
  return RRF_OK;
}

}  // namespace rrf
