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

constexpr int kRT = 512;    // most threads of a panel workgroup
constexpr int kPMaxK = 64;  // widest panel

// One halving exchange of the reduce-scatter below (offset O, H values kept),
// then the next; the steps are unrolled at compile time so that every
// register index is static.
template <int H, int O, int K>
__device__ inline void halve(double (&s)[K], int lane) {
  if constexpr (H >= 1) {
    const bool up = (lane & O) != 0;
#pragma unroll
    for (int i = 0; i < H; ++i) {
      const double keep = up ? s[i + H] : s[i];
      const double send = up ? s[i] : s[i + H];
      s[i] = keep + __shfl_xor(send, O, 64);
    }
    halve<H / 2, O / 2, K>(s, lane);
  }
}

// Sum over the 64 lanes of each of K values (K a power of two <= 64):
// halving exchanges leave lane l holding value l / (64 / K).
template <int K>
__device__ inline double wave_reduce_scatter(double (&s)[K], int lane) {
  halve<K / 2, 32, K>(s, lane);
  double v = s[0];
#pragma unroll
  for (int o = 32 / K; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Householder QR of an M x k panel (k <= K) with compact-WY output (Sec. 2.3,
// the dlarfg rule), the panel held in registers: thread t owns rows t,
// t + 512, ... (RPT of them), all K columns. Column j takes one reduction
// of K inner products with the current column j over the rows below j,
//   s_c = sum_{r > j} x_rc x_rj,
// which give at once the norm (c = j), v_j^T A_c for the update of the
// later columns (c > j, with row j published through LDS) and the dots
// v_c^T v_j that extend T_f (c < j). Two barriers per column.
template <int K, int RPT, int NT>
__global__ __launch_bounds__(NT) void panel_reg_kernel(const PanelDesc* __restrict__ descs,
                                                       int k) {
  constexpr int kRW = NT / 64;
  __shared__ double part[kRW][K];
  __shared__ double red[K];
  __shared__ double rowj[2][K];
  __shared__ double Tl[K][K + 1];  // Tl[i][c] = T_f(i, c)
  __shared__ double taus[K];
  const PanelDesc a = descs[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t M = a.M;

  double x[RPT][K];
#pragma unroll
  for (int t = 0; t < RPT; ++t) {
    const int64_t r = tid + (int64_t)t * NT;
#pragma unroll
    for (int c = 0; c < K; ++c) x[t][c] = (r < M && c < k) ? a.P[r + (int64_t)c * a.ldp] : 0.0;
  }
  if (a.zero)
#pragma unroll
    for (int t = 0; t < RPT; ++t) {
      const int64_t r = tid + (int64_t)t * NT;
      if (r < M)
        for (int c = 0; c < k; ++c) a.zero[r + (int64_t)c * a.ldz] = 0.0;
    }

  for (int j = 0; j < k; ++j) {
    double xj[RPT];
#pragma unroll
    for (int t = 0; t < RPT; ++t) {
      double v = 0.0;
#pragma unroll
      for (int c = 0; c < K; ++c) v = (c == j) ? x[t][c] : v;
      xj[t] = v;
    }
    if (tid == j)
#pragma unroll
      for (int c = 0; c < K; ++c) rowj[j & 1][c] = x[0][c];
    // partial sums over this thread's rows, reduced in chunks of at most 32
    // values (fewer live registers)
    constexpr int CH = K < 32 ? K : 32;
#pragma unroll
    for (int c0 = 0; c0 < K; c0 += CH) {
      double s[CH];
#pragma unroll
      for (int c = 0; c < CH; ++c) s[c] = 0.0;
#pragma unroll
      for (int t = 0; t < RPT; ++t) {
        const int64_t r = tid + (int64_t)t * NT;
        const double w = (r > j) ? xj[t] : 0.0;
#pragma unroll
        for (int c = 0; c < CH; ++c) s[c] += x[t][c0 + c] * w;
      }
      const double v = wave_reduce_scatter<CH>(s, lane);
      if (lane % (64 / CH) == 0) part[wave][c0 + lane / (64 / CH)] = v;
    }
    __syncthreads();
    if (tid < K) {
      double acc = 0.0;
#pragma unroll
      for (int w = 0; w < kRW; ++w) acc += part[w][tid];
      red[tid] = acc;
    }
    __syncthreads();
    const double* rj = rowj[j & 1];
    const double alpha = rj[j], xn2 = red[j];
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
    // d_c = v_c^T v_j (c < j) and w_c = v_j^T A_c (c > j), one column at a time
    double vr[RPT];
#pragma unroll
    for (int t = 0; t < RPT; ++t) {
      const int64_t r = tid + (int64_t)t * NT;
      vr[t] = (r > j) ? scal * xj[t] : (r == j ? 1.0 : 0.0);
    }
#pragma unroll
    for (int c = 0; c < K; ++c) {
      const double dwc = rj[c] + scal * red[c];
#pragma unroll
      for (int t = 0; t < RPT; ++t) {
        const int64_t r = tid + (int64_t)t * NT;
        const double upd = x[t][c] - tau * vr[t] * dwc;
        x[t][c] = (c > j) ? upd : (c == j ? ((r > j) ? vr[t] : (r == j ? beta : x[t][c])) : x[t][c]);
      }
    }
    // column j of T_f: T(i, j) = -tau_j sum_{c=i}^{j-1} T(i, c) d_c
    if (tid < j) {
      double acc = 0.0;
      for (int c = tid; c < j; ++c) acc += Tl[tid][c] * (rj[c] + scal * red[c]);
      Tl[tid][j] = -tau * acc;
    } else if (tid == j) {
      Tl[j][j] = tau;
      taus[j] = tau;
    }
  }
  __syncthreads();
  for (int idx = tid; idx < k * k; idx += NT) {
    const int i = idx % k, c = idx / k;
    a.Tf[i + (int64_t)c * a.ldt] = (i <= c) ? Tl[i][c] : 0.0;
  }
  for (int j = tid; j < k; j += NT) a.tau[j] = taus[j];
#pragma unroll
  for (int t = 0; t < RPT; ++t) {
    const int64_t r = tid + (int64_t)t * NT;
    if (r >= M) continue;
#pragma unroll
    for (int c = 0; c < K; ++c)
      if (c < k) a.W[r + (int64_t)c * a.ldw] = (r < c) ? 0.0 : (r == c ? 1.0 : x[t][c]);
    if (a.R && r < k)
#pragma unroll
      for (int c = 0; c < K; ++c)
        if (c < k) a.R[r + (int64_t)c * a.ldr] = (c >= r) ? x[t][c] : 0.0;
  }
}

}  // namespace

// --- host side -------------------------------------------------------------

int64_t panel_wg_max_rows(int k) {
  if (k < 1 || k > kPMaxK) return 0;
  int K = 1;
  while (K < k) K <<= 1;
  // at most 32 register doubles of panel per thread: taller panels are
  // faster split by columns than held at 64 doubles per thread
  return (int64_t)kRT * std::max(1, std::min(32 / K, 8));
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

template <int K, int RPT>
void launch_panel(hipStream_t st, const PanelDesc* d, int count, int k, int nt) {
  if (nt == 256)
    hipLaunchKernelGGL((panel_reg_kernel<K, RPT, 256>), dim3((unsigned)count), dim3(256), 0, st, d,
                       k);
  else
    hipLaunchKernelGGL((panel_reg_kernel<K, RPT, kRT>), dim3((unsigned)count), dim3(kRT), 0, st, d,
                       k);
}

template <int K>
void launch_panel_rows(hipStream_t st, const PanelDesc* d, int count, int k, int rpt, int nt) {
  if constexpr (K <= 64) {
    if (rpt == 1) launch_panel<K, 1>(st, d, count, k, nt);
    if constexpr (2 * K <= 64) if (rpt == 2) launch_panel<K, 2>(st, d, count, k, nt);
    if constexpr (4 * K <= 64) if (rpt == 4) launch_panel<K, 4>(st, d, count, k, nt);
    if constexpr (8 * K <= 64) if (rpt == 8) launch_panel<K, 8>(st, d, count, k, nt);
  }
}

int panel_wg_batched(hipStream_t st, const PanelDesc* d_descs, int count, int k,
                     int64_t max_rows) {
  if (count <= 0) return RRF_OK;
  if (k < 1 || k > kPMaxK || max_rows > panel_wg_max_rows(k))
    return set_error(RRF_E_INTERNAL, "batched panel: shape beyond one workgroup's registers");
  int K = 1;
  while (K < k) K <<= 1;
  // 256 threads when their rows fit in at most 32 register doubles per
  // thread (several panels per CU), else 512
  int nt = 256, rpt = 1;
  while ((int64_t)nt * rpt < max_rows) rpt <<= 1;
  if (K * rpt > 32) {
    nt = kRT;
    rpt = 1;
    while ((int64_t)nt * rpt < max_rows) rpt <<= 1;
  }
  int tok = trace_begin(st, kTrPanel, 0.0, 0.0);
  switch (K) {
    case 1: launch_panel_rows<1>(st, d_descs, count, k, rpt, nt); break;
    case 2: launch_panel_rows<2>(st, d_descs, count, k, rpt, nt); break;
    case 4: launch_panel_rows<4>(st, d_descs, count, k, rpt, nt); break;
    case 8: launch_panel_rows<8>(st, d_descs, count, k, rpt, nt); break;
    case 16: launch_panel_rows<16>(st, d_descs, count, k, rpt, nt); break;
    case 32: launch_panel_rows<32>(st, d_descs, count, k, rpt, nt); break;
    default: launch_panel_rows<64>(st, d_descs, count, k, rpt, nt);
  }
  trace_end(st, tok);
  RRF_CHECK_HIP(hipGetLastError());
  return RRF_OK;
}

}  // namespace rrf
