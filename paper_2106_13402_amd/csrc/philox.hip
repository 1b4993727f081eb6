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
#include "philox.hpp"
#include "trace.hpp"

namespace rrf {

namespace {

// kUniform: write the four uniforms of each counter instead of the Gaussians
// made from them (rows 4g .. 4g + 3 = u_a, v_a, u_b, v_b).
template <bool kUniform>
__global__ __launch_bounds__(256) void gaussian_kernel(uint64_t seed, uint64_t sid, int64_t rows,
                                                       int64_t cols, double* __restrict__ out,
                                                       int64_t ld) {
  const int64_t groups = (rows + 3) / 4;
  const int64_t total = groups * cols;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * 256) {
    const int64_t gr = t % groups;
    const int64_t c = t / groups;
    double v[4];
    if (kUniform)
      uniforms4(seed, sid, (uint64_t)gr, (uint64_t)c, v);
    else
      gaussian4(seed, sid, (uint64_t)gr, (uint64_t)c, v);
    double* col = out + c * ld;
    const int64_t r0 = gr * 4;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (r0 + k < rows) col[r0 + k] = v[k];
  }
}

}  // namespace

namespace {

template <bool kUniform>
int launch(hipStream_t st, uint64_t seed, uint64_t stream_id, int64_t rows, int64_t cols,
           double* out, int64_t ld) {
  if (rows <= 0 || cols <= 0) return RRF_OK;
  const int64_t total = ((rows + 3) / 4) * cols;
  int64_t blocks = ceil_div(total, 256);
  if (blocks > 16384) blocks = 16384;
  int tok = trace_begin(st, kTrGaussian, 0.0, 8.0 * rows * cols);
  hipLaunchKernelGGL(gaussian_kernel<kUniform>, dim3((unsigned)blocks), dim3(256), 0, st, seed,
                     stream_id, rows, cols, out, ld);
  trace_end(st, tok);
  RRF_CHECK_HIP(hipGetLastError());
  return RRF_OK;
}

}  // namespace

int gaussian(hipStream_t st, uint64_t seed, uint64_t stream_id, int64_t rows, int64_t cols,
             double* out, int64_t ld) {
  return launch<false>(st, seed, stream_id, rows, cols, out, ld);
}

int sketch_uniforms(hipStream_t st, uint64_t seed, uint64_t stream_id, int64_t rows, int64_t cols,
                    double* out, int64_t ld) {
  return launch<true>(st, seed, stream_id, rows, cols, out, ld);
}

}  // namespace rrf
