// Batched building blocks: many small problems per launch.
//
// The batched randUTV factors thousands of small matrices (n up to 512, b up
// to 64) at once, one step of Alg. 3 for all of them per round of launches.
// Each kernel here takes an array of per-problem descriptors in device memory
// and handles every problem in one launch (grid.y or grid.x = problem), so a
// round costs a fixed number of launches whatever the batch size:
//  * gemm_grouped_kernel: C = alpha op(A) op(B) + beta C per problem on the
//    FP64 matrix cores, one workgroup per tile of every problem (a flat grid
//    over all tiles), tile shape chosen per launch by the outputs' width;
//  * elem_kernel: fill / copy / diagonal / identity per problem;
//  * gauss_kernel: the sketch Gaussian of each problem (its own key);
//  * panel_wg_kernel: Householder QR with compact-WY output (Sec. 2.3, the
//    dlarfg rule) of a whole panel by one workgroup, rows resident in LDS.
//    The arithmetic is that of the grid-wide panel kernel with every sum
//    taken inside the workgroup.
#include <algorithm>
#include <climits>
#include <vector>

#include "batched.hpp"
#include "common.hpp"
#include "gemm_tile.hpp"
#include "kernels.hpp"
#include "philox.hpp"
#include "trace.hpp"

namespace rrf {

namespace {

// --- grouped GEMM ----------------------------------------------------------

// One BM x BN tile of one problem per workgroup (the MFMA tile loop of
// gemm_tile.hpp); the workgroup finds its problem by binary search of the
// running tile counts.
template <bool TA, bool TB, int BM, int BN, int GM, int GN, bool VEC>
__global__ __launch_bounds__(tile::kThreads, 2) void gemm_grouped_kernel(
    const GemmDesc* __restrict__ descs, const int* __restrict__ prefix, int count) {
  using TL = tile::Tile<BM, BN, TA, TB, VEC, GM, GN>;
  __shared__ double lds[TL::LDS];
  const int bid = blockIdx.x;
  int lo = 0, hi = count;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (prefix[mid] <= bid) lo = mid;
    else hi = mid;
  }
  const GemmDesc g = descs[lo];
  const int t = bid - prefix[lo];
  const int64_t tiles_m = (g.M + BM - 1) / BM;
  const int64_t i0 = (int64_t)(t % tiles_m) * BM;
  const int64_t j0 = (int64_t)(t / tiles_m) * BN;

  f64x4 acc[TL::MI][TL::NI];
#pragma unroll
  for (int a = 0; a < TL::MI; ++a)
#pragma unroll
    for (int b = 0; b < TL::NI; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  TL::run(acc, lds, g.A, g.lda, g.B, g.ldb, g.M, g.N, i0, j0, 0, g.K);
#pragma unroll
  for (int a = 0; a < TL::MI; ++a) {
    const int64_t gi = TL::row(i0, a);
    if (gi >= g.M) continue;
#pragma unroll
    for (int b = 0; b < TL::NI; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gj = TL::col(j0, b, r);
        if (gj >= g.N) continue;
        double c = g.alpha * acc[a][b][r];
        if (g.beta != 0.0) c += g.beta * g.C[gi + gj * g.ldc];
        g.C[gi + gj * g.ldc] = c;
      }
  }
}

template <int BM, int BN, int GM, int GN, bool VEC>
void launch_grouped(hipStream_t st, bool ta, bool tb, dim3 grid, const GemmDesc* d,
                    const int* prefix, int count) {
  const dim3 block(tile::kThreads);
  if (!ta && !tb)
    hipLaunchKernelGGL((gemm_grouped_kernel<false, false, BM, BN, GM, GN, VEC>), grid, block, 0,
                       st, d, prefix, count);
  else if (ta && !tb)
    hipLaunchKernelGGL((gemm_grouped_kernel<true, false, BM, BN, GM, GN, VEC>), grid, block, 0,
                       st, d, prefix, count);
  else if (!ta && tb)
    hipLaunchKernelGGL((gemm_grouped_kernel<false, true, BM, BN, GM, GN, VEC>), grid, block, 0,
                       st, d, prefix, count);
  else
    hipLaunchKernelGGL((gemm_grouped_kernel<true, true, BM, BN, GM, GN, VEC>), grid, block, 0,
                       st, d, prefix, count);
}

template <bool VEC>
void launch_grouped_tile(hipStream_t st, bool ta, bool tb, int tile, dim3 grid,
                         const GemmDesc* d, const int* prefix, int count) {
  switch (tile) {
    case kTile128x128: launch_grouped<128, 128, 2, 2, VEC>(st, ta, tb, grid, d, prefix, count); break;
    case kTile128x64: launch_grouped<128, 64, 2, 2, VEC>(st, ta, tb, grid, d, prefix, count); break;
    case kTile64x64: launch_grouped<64, 64, 2, 2, VEC>(st, ta, tb, grid, d, prefix, count); break;
    case kTile128x32: launch_grouped<128, 32, 4, 1, VEC>(st, ta, tb, grid, d, prefix, count); break;
    default: launch_grouped<128, 16, 4, 1, VEC>(st, ta, tb, grid, d, prefix, count);
  }
}

// --- elementwise -----------------------------------------------------------

// One workgroup per (problem, group of 8 columns).
__global__ __launch_bounds__(256) void elem_kernel(const ElemDesc* __restrict__ descs) {
  const ElemDesc d = descs[blockIdx.y];
  const int64_t c0 = (int64_t)blockIdx.x * 8;
  for (int64_t c = c0; c < c0 + 8 && c < d.cols; ++c)
    for (int64_t r = threadIdx.x; r < d.rows; r += 256) {
      double v;
      switch (d.op) {
        case kElemFill: v = d.v; break;
        case kElemCopy: v = d.S[r + c * d.lds]; break;
        case kElemDiag: v = (r == c) ? d.S[c] : 0.0; break;
        default: v = (r == c) ? 1.0 : 0.0; break;  // identity
      }
      d.X[r + c * d.ld] = v;
    }
}

// --- Gaussian --------------------------------------------------------------

__global__ __launch_bounds__(256) void gauss_kernel(const GaussDesc* __restrict__ descs) {
  const GaussDesc d = descs[blockIdx.y];
  const int64_t groups = (d.rows + 3) / 4;
  const int64_t total = groups * d.cols;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * 256) {
    const int64_t gr = t % groups, c = t / groups;
    double v[4];
    gaussian4(d.seed, d.sid, (uint64_t)gr, (uint64_t)c, v);
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (gr * 4 + k < d.rows) d.out[gr * 4 + k + c * d.ld] = v[k];
  }
}

// --- Householder panel, one workgroup --------------------------------------

constexpr int kPT = 512;
constexpr int kPMaxK = 64;

__device__ inline int pow2_at_least(int n) {
  int p = 1;
  while (p < n) p <<= 1;
  return p;
}

// Rows of the panel live in LDS (row-major, stride k + 1, one zero row
// after them, the spare column k absorbing the diagonal lane's stores), Tf
// after them. Round j applies H_{j-1} and forms, in the same pass, the Gram
// row of column j with the later columns and the dots v_{j-1}^T v_l for
// column j-1 of Tf; the sums are reduced across the workgroup in LDS.
__global__ __launch_bounds__(kPT) void panel_wg_kernel(const PanelDesc* __restrict__ descs,
                                                       int k) {
  extern __shared__ double smem[];
  __shared__ double red_s[3 * kPMaxK];
  __shared__ double w_s[kPMaxK];
  __shared__ double part[kPT];
  const PanelDesc a = descs[blockIdx.x];
  const int tid = threadIdx.x;
  const int rows = (int)a.M;
  const int L = k + 1;
  double* Ls = smem;
  double* Tl = smem + (size_t)(rows + 1) * L;  // k x k, ld k

  for (int idx = tid; idx < rows * k; idx += kPT) {
    const int r = idx % rows, c = idx / rows;
    Ls[r * L + c] = a.P[r + (int64_t)c * a.ldp];
  }
  for (int c = tid; c < L; c += kPT) Ls[rows * L + c] = 0.0;
  __syncthreads();
  if (a.zero)
    for (int idx = tid; idx < rows * k; idx += kPT) {
      const int r = idx % rows, c = idx / rows;
      a.zero[r + (int64_t)c * a.ldz] = 0.0;
    }

  double tau_prev = 0.0;
  for (int j = 0; j <= k; ++j) {
    const int ns = (j < k) ? (k - j) : 0;
    const int nt = (j >= 2) ? (j - 1) : 0;
    const double twj = (j >= 1 && j < k) ? tau_prev * w_s[j] : 0.0;
    const int nc = ns + nt;
    const int ncp = pow2_at_least(nc);
    const int tpc = kPT / ncp;
    const int ci = tid % ncp, sub = tid / ncp;
    const int jm = (j >= 1) ? j - 1 : 0;
    double acc = 0.0;
    if (ci < nc) {
      const bool gram = ci < ns;
      const int col = gram ? j + ci : ci - ns;
      const int cst = (gram && col == j) ? k : col;
      const double tw = (gram && j >= 1) ? tau_prev * w_s[col] : 0.0;
      if (!gram && sub == 0) acc = Ls[(j - 1) * L + col];  // row j-1 of v_{j-1} is 1
      for (int r = j + sub; r < rows; r += tpc) {
        const double vv = Ls[r * L + jm];
        const double y = Ls[r * L + col] - tw * vv;
        Ls[r * L + cst] = y;
        const double xj = (r == j) ? 0.0 : Ls[r * L + j] - twj * vv;
        acc += (gram ? xj : vv) * y;
      }
    }
    part[tid] = acc;
    __syncthreads();
    if (tid < nc) {
      double s = 0.0;
      for (int u = 0; u < tpc; ++u) s += part[tid + u * ncp];
      if (tid < ns) red_s[j + tid] = s;
      else red_s[2 * k + (tid - ns)] = s;
    }
    if (j < k) {
      for (int c = j + 1 + tid; c < k; c += kPT) red_s[k + c] = Ls[j * L + c];
      for (int r = j + tid; r < rows; r += kPT) {
        double x = Ls[r * L + j];
        if (j >= 1) {
          x -= twj * Ls[r * L + j - 1];
          Ls[r * L + j] = x;
        }
        if (r == j) red_s[k + j] = x;
      }
    }
    __syncthreads();
    // column j-1 of Tf: Tf(i, j-1) = -tau_{j-1} sum_{c=i}^{j-2} Tf(i, c) dots_c
    if (j >= 1) {
      const int jj = j - 1;
      for (int i = tid; i < jj; i += kPT) {
        double s = 0.0;
        for (int c = i; c < jj; ++c) s += Tl[i + c * k] * red_s[2 * k + c];
        Tl[i + jj * k] = -tau_prev * s;
      }
      if (tid == 0) Tl[jj + jj * k] = tau_prev;
    }
    if (j == k) break;
    const double alpha = red_s[k + j];
    const double xn2 = red_s[j];
    double tau, beta, scal;
    if (xn2 == 0.0) {
      tau = 0.0;
      beta = alpha;
      scal = 0.0;
    } else {
      const double nrm = sqrt(alpha * alpha + xn2);
      beta = -copysign(nrm, alpha);
      tau = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    for (int c = j + 1 + tid; c < k; c += kPT) {
      const double w = red_s[k + c] + scal * red_s[c];
      w_s[c] = w;
      if (a.R) a.R[j + (int64_t)c * a.ldr] = red_s[k + c] - tau * w;
    }
    if (tid == 0) {
      a.tau[j] = tau;
      if (a.R) a.R[j + (int64_t)j * a.ldr] = beta;
    }
    if (a.R)
      for (int i = j + 1 + tid; i < k; i += kPT) a.R[i + (int64_t)j * a.ldr] = 0.0;
    for (int r = j + 1 + tid; r < rows; r += kPT) Ls[r * L + j] *= scal;
    tau_prev = tau;
    __syncthreads();
  }
  __syncthreads();
  for (int idx = tid; idx < k * k; idx += kPT) {
    const int i = idx % k, c = idx / k;
    a.Tf[i + (int64_t)c * a.ldt] = (i <= c) ? Tl[i + c * k] : 0.0;
  }
  for (int idx = tid; idx < rows * k; idx += kPT) {
    const int r = idx % rows, c = idx / rows;
    a.W[r + (int64_t)c * a.ldw] = (r < c) ? 0.0 : (r == c ? 1.0 : Ls[r * L + c]);
  }
}

constexpr int64_t kPanelLds = 140 * 1024;
bool g_panel_attr = false;

}  // namespace

// --- host side -------------------------------------------------------------

int64_t panel_wg_max_rows(int k) {
  if (k < 1 || k > kPMaxK) return 0;
  const int64_t avail = kPanelLds / 8 - (int64_t)k * k;
  return avail / (k + 1) - 1;
}

int gemm_grouped(hipStream_t st, bool ta, bool tb, int tile, bool vec, const GemmDesc* d_descs,
                 const int* d_prefix, int count, int64_t total_tiles, double flops) {
  if (count <= 0 || total_tiles <= 0) return RRF_OK;
  if (tile < 0 || tile >= kGemmTiles) return set_error(RRF_E_INTERNAL, "grouped gemm: tile shape");
  if (total_tiles > INT32_MAX) return set_error(RRF_E_NOTSUP, "grouped gemm: too many tiles");
  const dim3 grid((unsigned)total_tiles);
  static const int cls[kGemmTiles] = {kTrGemmGrouped, kTrGemmGrouped128x64, kTrGemmGrouped128x32,
                                      kTrGemmGrouped128x16, kTrGemmGrouped128x128};
  int tok = trace_begin(st, cls[tile], flops, 0.0);
  if (vec) launch_grouped_tile<true>(st, ta, tb, tile, grid, d_descs, d_prefix, count);
  else launch_grouped_tile<false>(st, ta, tb, tile, grid, d_descs, d_prefix, count);
  trace_end(st, tok);
  RRF_CHECK_HIP(hipGetLastError());
  return RRF_OK;
}

int elem_batched(hipStream_t st, const ElemDesc* d_descs, int count, int64_t max_cols) {
  if (count <= 0 || max_cols <= 0) return RRF_OK;
  int tok = trace_begin(st, kTrElementwise, 0.0, 0.0);
  for (int c0 = 0; c0 < count; c0 += 65535) {
    const dim3 grid((unsigned)ceil_div(max_cols, 8), (unsigned)std::min(count - c0, 65535));
    hipLaunchKernelGGL(elem_kernel, grid, dim3(256), 0, st, d_descs + c0);
  }
  trace_end(st, tok);
  RRF_CHECK_HIP(hipGetLastError());
  return RRF_OK;
}

int gauss_batched(hipStream_t st, const GaussDesc* d_descs, int count, int64_t max_elems) {
  if (count <= 0 || max_elems <= 0) return RRF_OK;
  int tok = trace_begin(st, kTrGaussian, 0.0, 0.0);
  const unsigned bx = (unsigned)std::min<int64_t>(ceil_div(ceil_div(max_elems, 4), 256), 64);
  for (int c0 = 0; c0 < count; c0 += 65535) {
    const dim3 grid(bx, (unsigned)std::min(count - c0, 65535));
    hipLaunchKernelGGL(gauss_kernel, grid, dim3(256), 0, st, d_descs + c0);
  }
  trace_end(st, tok);
  RRF_CHECK_HIP(hipGetLastError());
  return RRF_OK;
}

int panel_wg_batched(hipStream_t st, const PanelDesc* d_descs, int count, int k,
                     int64_t max_rows) {
  if (count <= 0) return RRF_OK;
  if (k < 1 || k > kPMaxK || max_rows > panel_wg_max_rows(k))
    return set_error(RRF_E_INTERNAL, "batched panel: shape beyond one workgroup's LDS");
  if (!g_panel_attr) {
    RRF_CHECK_HIP(hipFuncSetAttribute((const void*)panel_wg_kernel,
                                      hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)kPanelLds));
    g_panel_attr = true;
  }
  const size_t lds = ((size_t)(max_rows + 1) * (k + 1) + (size_t)k * k) * 8;
  int tok = trace_begin(st, kTrPanel, 0.0, 0.0);
  hipLaunchKernelGGL(panel_wg_kernel, dim3((unsigned)count), dim3(kPT), lds, st, d_descs, k);
  trace_end(st, tok);
  RRF_CHECK_HIP(hipGetLastError());
  return RRF_OK;
}

}  // namespace rrf
