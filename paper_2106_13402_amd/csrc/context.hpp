// Per-device side streams and events (context.hip).
#pragma once

#include <mutex>

#include "common.hpp"

namespace rrf {

constexpr int kSideStreams = 2;
constexpr int kSliceStreams = 3;
constexpr int kCtxEvents = 16;

// HIP spreads the streams of a process over a few hardware queues (four by
// default) and a queue runs its kernels one after another. The batched
// driver's slices run on the caller's stream and on `slice`, which are made
// first so that each slice holds a queue of its own when the process has no
// other streams; `side` comes after them.
struct DeviceContext {
  hipStream_t slice[kSliceStreams] = {};
  hipStream_t side[kSideStreams] = {};
  hipEvent_t ev[kCtxEvents] = {};
  std::mutex mu;  // one factorization enqueues on these streams at a time
};

int device_context(DeviceContext** out);

}  // namespace rrf
