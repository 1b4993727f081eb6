// Per-device execution context: the streams and events the drivers use to
// overlap independent work with the critical path. Created on first use
// and kept for the life of the process; every stream has the default
// priority and does not synchronize with the null stream.
#include <mutex>
#include <unordered_map>

#include "common.hpp"
#include "context.hpp"

namespace rrf {

namespace {
std::mutex g_mu;
std::unordered_map<int, DeviceContext*> g_ctx;
}  // namespace

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
