// Per-device side streams and events (context.hip).
#pragma once

#include <mutex>

#include "common.hpp"

namespace rrf {

constexpr int kSideStreams = 2;
constexpr int kCtxEvents = 16;

struct DeviceContext {
  hipStream_t side[kSideStreams] = {};
  hipEvent_t ev[kCtxEvents] = {};
  std::mutex mu;  // one factorization enqueues on these streams at a time
};

int device_context(DeviceContext** out);

}  // namespace rrf
