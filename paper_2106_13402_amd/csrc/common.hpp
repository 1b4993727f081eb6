// Shared definitions for the rrf HIP library (gfx950 / MI355X).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/rrf.h"

namespace rrf {

typedef double f64x4 __attribute__((ext_vector_type(4)));

// Record a HIP failure for rrf_last_error(); returns RRF_E_HIP.
int set_hip_error(hipError_t e, const char* what, const char* file, int line);
// Record a message for rrf_last_error(); returns the given status.
int set_error(int status, const char* msg);

#define RRF_CHECK_HIP(expr)                                                     \
  do {                                                                          \
    hipError_t rrf_e_ = (expr);                                                 \
    if (rrf_e_ != hipSuccess)                                                   \
      return ::rrf::set_hip_error(rrf_e_, #expr, __FILE__, __LINE__);           \
  } while (0)

#define RRF_TRY(expr)                                                           \
  do {                                                                          \
    int rrf_s_ = (expr);                                                        \
    if (rrf_s_ != RRF_OK) return rrf_s_;                                        \
  } while (0)

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

// Bump allocator over a caller-provided device workspace (256-byte aligned).
struct Arena {
  char* base = nullptr;
  size_t cap = 0;
  size_t used = 0;
  bool counting = false;  // size-query mode: only accumulate `used`
  template <typename T>
  T* take(size_t count) {
    size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
    size_t at = used;
    used += bytes;
    if (counting) return nullptr;
    if (used > cap) return nullptr;
    return reinterpret_cast<T*>(base + at);
  }
};

}  // namespace rrf
