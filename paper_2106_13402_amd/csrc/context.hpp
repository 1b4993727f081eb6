// Per-device side streams and events (context.hip).
#pragma once

#include <mutex>

#include "common.hpp"

namespace rrf {

constexpr int kSideStreams = 2;
constexpr int kCtxEvents = 16;

// HIP spreads the streams of a process over a few hardware queues (four by
// default) and a queue runs its kernels one after another. Each queue the
// process holds also costs the single-matrix drivers time (one idle queue
// more made randUTV at n = 16384 about 9% slower), so the context holds few
// streams: the two side streams, made at first use, and `extra`, made when
// the batched driver first runs; that driver's slices run on the caller's
// stream, the side streams and `extra`.
struct DeviceContext {
  hipStream_t side[kSideStreams] = {};
  hipStream_t extra = nullptr;
  hipEvent_t ev[kCtxEvents] = {};
  std::mutex mu;  // one driver enqueues on these streams at a time
};

int device_context(DeviceContext** out);

// Lets `kernel` launch with up to `bytes` of dynamic LDS on the current
// device. hipFuncSetAttribute acts on the current device only, so the
// attribute is set once per (kernel, device), and again when a later call
// asks for more; callable from several host threads at once.
int allow_dynamic_lds(const void* kernel, size_t bytes);

}  // namespace rrf
