// The sketch generator on the device: Philox4x64-10 + Box-Muller.
//
// The paper draws G with `randn` (Alg. 1 first step, Alg. 3 inside its loop)
// without fixing a generator. This library fixes a counter-based one so a
// Gaussian matrix is a pure function of (seed, stream, row, column) and is
// generated where it is used, in HBM, with no host involvement:
//   Philox4x64-10 (Salmon et al., SC'11) with key (seed, stream) and counter
//   (row / 4, column, 0, 0); outputs w0..w3 give uniforms
//   u = ((w >> 11) + 1) 2^-53 in (0,1] (w0, w2) and v = (w >> 11) 2^-53 in
//   [0,1) (w1, w3); rho = sqrt(-2 ln u), theta = 2 pi v; rows 4g, 4g+1 take
//   rho_a cos/sin(theta_a), rows 4g+2, 4g+3 take rho_b cos/sin(theta_b).
// One thread produces four consecutive rows of one column (32 contiguous
// bytes), so a wavefront writes 2 KiB of one column.
#include "common.hpp"
#include "kernels.hpp"
#include "trace.hpp"

namespace rrf {

namespace {

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

__global__ __launch_bounds__(256) void gaussian_kernel(uint64_t seed, uint64_t sid, int64_t rows,
                                                       int64_t cols, double* __restrict__ out,
                                                       int64_t ld) {
  const int64_t groups = (rows + 3) / 4;
  const int64_t total = groups * cols;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * 256) {
    const int64_t gr = t % groups;
    const int64_t c = t / groups;
    uint64_t x0 = (uint64_t)gr, x1 = (uint64_t)c, x2 = 0, x3 = 0;
    philox4x64_10(x0, x1, x2, x3, seed, sid);
    const double ua = ((double)(x0 >> 11) + 1.0) * 0x1p-53;
    const double va = (double)(x1 >> 11) * 0x1p-53;
    const double ub = ((double)(x2 >> 11) + 1.0) * 0x1p-53;
    const double vb = (double)(x3 >> 11) * 0x1p-53;
    const double rho_a = sqrt(-2.0 * log(ua));
    const double rho_b = sqrt(-2.0 * log(ub));
    const double ta = kTwoPi * va, tb = kTwoPi * vb;
    double v[4];
    v[0] = rho_a * cos(ta);
    v[1] = rho_a * sin(ta);
    v[2] = rho_b * cos(tb);
    v[3] = rho_b * sin(tb);
    double* col = out + c * ld;
    const int64_t r0 = gr * 4;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (r0 + k < rows) col[r0 + k] = v[k];
  }
}

}  // namespace

int gaussian(hipStream_t st, uint64_t seed, uint64_t stream_id, int64_t rows, int64_t cols,
             double* out, int64_t ld) {
  if (rows <= 0 || cols <= 0) return RRF_OK;
  const int64_t total = ((rows + 3) / 4) * cols;
  int64_t blocks = ceil_div(total, 256);
  if (blocks > 16384) blocks = 16384;
  int tok = trace_begin(st, kTrGaussian, 0.0, 8.0 * rows * cols);
  hipLaunchKernelGGL(gaussian_kernel, dim3((unsigned)blocks), dim3(256), 0, st, seed, stream_id,
                     rows, cols, out, ld);
  trace_end(st, tok);
  RRF_CHECK_HIP(hipGetLastError());
  return RRF_OK;
}

}  // namespace rrf
