// Element-wise helpers: identity start for U and V (Alg. 3 first line), the
// copy of A into T, block copies, the diagonal write T(I2,J2) = D, and the
// finiteness check of the input. All are HBM-bound grid-stride loops that
// walk column-major storage with consecutive threads on consecutive rows.
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"
#include "trace.hpp"

namespace rrf {

namespace {

inline unsigned blocks_for(int64_t elems) {
  int64_t b = ceil_div(elems, 256);
  if (b > 16384) b = 16384;
  if (b < 1) b = 1;
  return (unsigned)b;
}

// 2-D launch over a rows x cols column-major block: a workgroup of 256
// threads covers a tile of TR = min(256, rows rounded up to a power of two)
// rows by 256 / TR columns (so short, wide blocks keep every thread busy),
// tiles down the rows in x, across the columns in y with a stride loop. No
// per-element division.
struct Tile2 {
  int tr_log2;  // log2 TR
  dim3 grid;
};

inline Tile2 tile2(int64_t rows, int64_t cols) {
  int lg = 0;
  while ((1 << lg) < rows && lg < 8) ++lg;
  const int64_t tc = 256 >> lg;
  Tile2 t;
  t.tr_log2 = lg;
  t.grid = dim3((unsigned)ceil_div(rows, (int64_t)1 << lg),
                (unsigned)std::min<int64_t>(ceil_div(cols, tc), 65535));
  return t;
}

// Visit every (i, j) of the block with f(i, j).
#define RRF_TILE2_LOOP(rows, cols, lg, body)                                        \
  do {                                                                              \
    const int tr_ = 1 << (lg), tc_ = 256 >> (lg);                                   \
    const int64_t i = (int64_t)blockIdx.x * tr_ + (threadIdx.x & (tr_ - 1));        \
    if (i < (rows))                                                                 \
      for (int64_t j = (int64_t)blockIdx.y * tc_ + (threadIdx.x >> (lg)); j < (cols); \
           j += (int64_t)gridDim.y * tc_) {                                         \
        body;                                                                       \
      }                                                                             \
  } while (0)

__global__ __launch_bounds__(256) void identity_kernel(int64_t rows, int64_t cols, double* X,
                                                       int64_t ld, int lg) {
  RRF_TILE2_LOOP(rows, cols, lg, X[i + j * ld] = (i == j) ? 1.0 : 0.0);
}

__global__ __launch_bounds__(256) void copy_kernel(int64_t rows, int64_t cols,
                                                   const double* __restrict__ S, int64_t lds,
                                                   double* __restrict__ D, int64_t ldd, int lg) {
  RRF_TILE2_LOOP(rows, cols, lg, D[i + j * ldd] = S[i + j * lds]);
}

__global__ __launch_bounds__(256) void fill_kernel(int64_t rows, int64_t cols, double v, double* X,
                                                   int64_t ld, int lg) {
  RRF_TILE2_LOOP(rows, cols, lg, X[i + j * ld] = v);
}

__global__ __launch_bounds__(256) void diag_kernel(int64_t rows, int64_t cols, const double* d,
                                                   double* X, int64_t ld, int lg) {
  RRF_TILE2_LOOP(rows, cols, lg, X[i + j * ld] = (i == j) ? d[i] : 0.0);
}

__global__ __launch_bounds__(256) void fill_u32_kernel(unsigned* p, int64_t count, unsigned v) {
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < count;
       t += (int64_t)gridDim.x * 256)
    p[t] = v;
}

__global__ __launch_bounds__(256) void finite_kernel(int64_t rows, int64_t cols,
                                                     const double* X, int64_t ld, int* status,
                                                     int lg) {
  bool bad = false;
  RRF_TILE2_LOOP(rows, cols, lg, {
    const double v = X[i + j * ld];
    if (!(v - v == 0.0)) bad = true;  // NaN or +-Inf
  });
  if (bad) atomicOr(status, 1);
}

}  // namespace

int set_identity(hipStream_t st, int64_t rows, int64_t cols, double* X, int64_t ld) {
  if (rows <= 0 || cols <= 0) return RRF_OK;
  int tok = trace_begin(st, kTrElementwise, 0.0, 8.0 * rows * cols);
  const Tile2 g = tile2(rows, cols);
  hipLaunchKernelGGL(identity_kernel, g.grid, dim3(256), 0, st, rows, cols, X, ld, g.tr_log2);
  trace_end(st, tok);
  RRF_CHECK_HIP(hipGetLastError());
  return RRF_OK;
}

namespace {
// D(c, r) = S(r, c) through 32 x 32 tiles in LDS (both sides coalesced).
__global__ __launch_bounds__(256) void transpose_kernel(int64_t rows, int64_t cols,
                                                        const double* __restrict__ S, int64_t lds,
                                                        double* __restrict__ D, int64_t ldd) {
  __shared__ double tile[32][33];
  const int64_t r0 = (int64_t)blockIdx.x * 32, c0 = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int j = ty; j < 32; j += 8) {
    const int64_t r = r0 + tx, c = c0 + j;
    if (r < rows && c < cols) tile[j][tx] = S[r + c * lds];
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    const int64_t c = c0 + tx, r = r0 + j;  // D(c, r)
    if (r < rows && c < cols) D[c + r * ldd] = tile[tx][j];
  }
}
}  // namespace

int transpose_matrix(hipStream_t st, int64_t rows, int64_t cols, const double* S, int64_t lds,
                     double* D, int64_t ldd) {
  if (rows <= 0 || cols <= 0) return RRF_OK;
  if (ceil_div(cols, 32) > 65535) return set_error(RRF_E_NOTSUP, "transpose: too many columns");
  int tok = trace_begin(st, kTrElementwise, 0.0, 16.0 * rows * cols);
  hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)ceil_div(rows, 32), (unsigned)ceil_div(cols, 32)),
                     dim3(256), 0, st, rows, cols, S, lds, D, ldd);
  trace_end(st, tok);
  RRF_CHECK_HIP(hipGetLastError());
  return RRF_OK;
}

int thin_q(hipStream_t st, int64_t M, int64_t k, const double* W, int64_t ldw, const double* Tf,
           int64_t ldt, double* Q, int64_t ldq, double* C) {
  RRF_TRY(dgemm(st, false, true, k, k, k, 1.0, Tf, ldt, W, ldw, 0.0, C, k, nullptr, 0));
  RRF_TRY(set_identity(st, M, k, Q, ldq));
  return dgemm(st, false, false, M, k, k, -1.0, W, ldw, C, k, 1.0, Q, ldq, nullptr, 0);
}

bool dgemm_in_place_fits(bool ta, bool tb, int64_t M, int64_t N, const double* A, int64_t lda,
                         const double* B, int64_t ldb, const double* C, int64_t ldc) {
  if (A == C) return !ta && lda == ldc && M >= 128 && N == 128;
  if (B == C) return !tb && ldb == ldc && M == 128 && N >= 128;
  return false;
}

int dgemm_in_place(hipStream_t st, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
                   const double* A, int64_t lda, const double* B, int64_t ldb, double* C,
                   int64_t ldc, double* work, size_t work_elems) {
  if (!dgemm_in_place_fits(ta, tb, M, N, A, lda, B, ldb, C, ldc))
    return set_error(RRF_E_NOTSUP, "dgemm_in_place: shape or aliasing not supported");
  // M, N >= 128 without small tiles: dgemm_shaped takes 128 x 128 tiles
  return dgemm_shaped(st, ta, tb, M, N, K, alpha, A, lda, B, ldb, 0.0, C, ldc, work, work_elems,
                      false, 0);
}

int copy_matrix(hipStream_t st, int64_t rows, int64_t cols, const double* S, int64_t lds,
                double* D, int64_t ldd) {
  if (rows <= 0 || cols <= 0) return RRF_OK;
  int tok = trace_begin(st, kTrElementwise, 0.0, 16.0 * rows * cols);
  const Tile2 g = tile2(rows, cols);
  hipLaunchKernelGGL(copy_kernel, g.grid, dim3(256), 0, st, rows, cols, S, lds, D, ldd, g.tr_log2);
  trace_end(st, tok);
  RRF_CHECK_HIP(hipGetLastError());
  return RRF_OK;
}

int fill_matrix(hipStream_t st, int64_t rows, int64_t cols, double v, double* X, int64_t ld) {
  if (rows <= 0 || cols <= 0) return RRF_OK;
  int tok = trace_begin(st, kTrElementwise, 0.0, 8.0 * rows * cols);
  const Tile2 g = tile2(rows, cols);
  hipLaunchKernelGGL(fill_kernel, g.grid, dim3(256), 0, st, rows, cols, v, X, ld, g.tr_log2);
  trace_end(st, tok);
  RRF_CHECK_HIP(hipGetLastError());
  return RRF_OK;
}

int set_diag(hipStream_t st, int64_t rows, int64_t cols, const double* d, double* X, int64_t ld) {
  if (rows <= 0 || cols <= 0) return RRF_OK;
  int tok = trace_begin(st, kTrElementwise, 0.0, 8.0 * rows * cols);
  const Tile2 g = tile2(rows, cols);
  hipLaunchKernelGGL(diag_kernel, g.grid, dim3(256), 0, st, rows, cols, d, X, ld, g.tr_log2);
  trace_end(st, tok);
  RRF_CHECK_HIP(hipGetLastError());
  return RRF_OK;
}

int fill_u32(hipStream_t st, unsigned* p, int64_t count, unsigned v) {
  if (count <= 0) return RRF_OK;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(blocks_for(count)), dim3(256), 0, st, p, count, v);
  RRF_CHECK_HIP(hipGetLastError());
  return RRF_OK;
}

int check_finite(hipStream_t st, int64_t rows, int64_t cols, const double* X, int64_t ld,
                 int* status) {
  if (rows <= 0 || cols <= 0) return RRF_OK;
  int tok = trace_begin(st, kTrElementwise, 0.0, 8.0 * rows * cols);
  const Tile2 g = tile2(rows, cols);
  hipLaunchKernelGGL(finite_kernel, g.grid, dim3(256), 0, st, rows, cols, X, ld, status,
                     g.tr_log2);
  trace_end(st, tok);
  RRF_CHECK_HIP(hipGetLastError());
  return RRF_OK;
}

}  // namespace rrf
