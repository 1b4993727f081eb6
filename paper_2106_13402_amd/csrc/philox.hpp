// Philox4x64-10 and the Box-Muller pair of the sketch Gaussian (device code
// shared by the single and the batched generators).
#pragma once

#include "common.hpp"

namespace rrf {

constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kM1 = 0xCA5A826395121157ull;
constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kW1 = 0xBB67AE8584CAA73Bull;
constexpr double kTwoPi = 6.283185307179586;  // nearest double to 2 pi

__device__ inline void philox4x64_10(uint64_t& x0, uint64_t& x1, uint64_t& x2, uint64_t& x3,
                                     uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += kW0;
      k1 += kW1;
    }
    const uint64_t hi0 = __umul64hi(kM0, x0), lo0 = kM0 * x0;
    const uint64_t hi1 = __umul64hi(kM1, x2), lo1 = kM1 * x2;
    const uint64_t y0 = hi1 ^ x1 ^ k0;
    const uint64_t y2 = hi0 ^ x3 ^ k1;
    x0 = y0;
    x1 = lo1;
    x2 = y2;
    x3 = lo0;
  }
}

// The four uniforms of counter (gr, c, 0, 0) under key (seed, sid), from
// the top 53 bits of each word: u in (0, 1] from words 0 and 2, v in [0, 1)
// from words 1 and 3, in the order (u_a, v_a, u_b, v_b).
__device__ inline void uniforms4(uint64_t seed, uint64_t sid, uint64_t gr, uint64_t c,
                                 double (&u)[4]) {
  uint64_t x0 = gr, x1 = c, x2 = 0, x3 = 0;
  philox4x64_10(x0, x1, x2, x3, seed, sid);
  u[0] = ((double)(x0 >> 11) + 1.0) * 0x1p-53;
  u[1] = (double)(x1 >> 11) * 0x1p-53;
  u[2] = ((double)(x2 >> 11) + 1.0) * 0x1p-53;
  u[3] = (double)(x3 >> 11) * 0x1p-53;
}

// Entries 4 gr .. 4 gr + 3 of column c of the Gaussian of (seed, sid):
// Box-Muller on the uniforms of counter (gr, c, 0, 0).
__device__ inline void gaussian4(uint64_t seed, uint64_t sid, uint64_t gr, uint64_t c,
                                 double (&v)[4]) {
  double u[4];
  uniforms4(seed, sid, gr, c, u);
  const double rho_a = sqrt(-2.0 * log(u[0]));
  const double rho_b = sqrt(-2.0 * log(u[2]));
  const double ta = kTwoPi * u[1], tb = kTwoPi * u[3];
  v[0] = rho_a * cos(ta);
  v[1] = rho_a * sin(ta);
  v[2] = rho_b * cos(tb);
  v[3] = rho_b * sin(tb);
}

}  // namespace rrf
