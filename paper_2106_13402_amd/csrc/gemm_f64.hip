// FP64 GEMM on the gfx950 matrix cores (v_mfma_f64_16x16x4f64).
//
// C = alpha * op(A) * op(B) + beta * C, column-major, op = N or T.
// Every dense contraction of the factorizations (the sketch and power
// products of Alg. 3 / Alg. 1, and the compact-WY applications of Sec. 2.3)
// goes through this kernel.
//
// Design (MI355X first):
//  * 256-thread workgroups (four wave64s in a 2 x 2 grid); a block tile of
//    BM x BN, each wave owning (BM/2) x (BN/2) as 16 x 16 MFMA sub-tiles with
//    the accumulators in AGPRs;
//  * K is walked in BK = 16 slices through two LDS buffers: the global loads
//    of slice t+1 are issued before the matrix cores start on slice t and are
//    written to the other buffer afterwards, one barrier per slice;
//  * LDS layout follows the operand's contiguous dimension in HBM:
//    "mn-major" operands (A for op = N, B for op = T) are stored [k][mn] with
//    a row stride of BM + 16 doubles, "k-major" ones [mn][k] with an odd row
//    stride of BK + 1 doubles. Both the global-to-LDS copy and the MFMA
//    operand fetch (16 lanes x 8 bytes at a fixed k) then spread over
//    distinct banks;
//  * global loads move 16 bytes per lane (two doubles along the contiguous
//    dimension) when the operand base and leading dimension allow it;
//  * the MFMA computes the *transposed* tile, D' = op(B)^T op(A)^T: the
//    instruction puts output row 4*reg + lane/16 and column lane%16 in each
//    lane, so with the operands swapped the 16 lanes of a quarter-wave own 16
//    consecutive rows of one column of C and the stores coalesce;
//  * skinny products (one output dimension = b) split K over gridDim.z into a
//    partial-sum buffer that a second kernel reduces in a fixed order, so
//    results are bitwise reproducible (no floating-point atomics).
#include "common.hpp"
#include "gemm_tile.hpp"
#include "kernels.hpp"
#include "trace.hpp"

namespace rrf {

namespace {

using tile::kBK;
using tile::kThreads;

struct GemmF64Args {
  int64_t M, N, K;
  double alpha, beta;
  const double* A;
  int64_t lda;
  const double* B;
  int64_t ldb;
  double* C;
  int64_t ldc;
  double* P;       // split-K partials: P[z * M * N + i + j * M] (null if no split)
  int64_t kchunk;  // K extent per split (multiple of kBK)
  int tiles_m;
};

template <int BM, int BN, bool TA, bool TB, bool VEC>
__global__ __launch_bounds__(kThreads, 2) void dgemm_mfma_kernel(GemmF64Args g) {
  // op(A) is k-major in HBM when A is transposed; op(B) when B is not.
  using OA = tile::Operand<BM, TA, VEC>;
  using OB = tile::Operand<BN, !TB, VEC>;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int MI = WM / 16, NI = WN / 16;
  __shared__ double lds[2 * (OA::SIZE + OB::SIZE)];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  const int tile = blockIdx.x;
  const int tm = tile % g.tiles_m;
  const int tn = tile / g.tiles_m;
  const int64_t i0 = (int64_t)tm * BM;
  const int64_t j0 = (int64_t)tn * BN;
  const int64_t kbeg = (int64_t)blockIdx.z * g.kchunk;
  const int64_t kend = (kbeg + g.kchunk < g.K) ? kbeg + g.kchunk : g.K;

  const int lr = lane & 15;  // row (mn) of the operand fragment
  const int lk = lane >> 4;  // k of the operand fragment

  // With beta != 0 (and no split) the accumulators start from
  // (beta / alpha) C, read before the K loop so that its latency overlaps
  // the operand loads instead of following the last MFMA; the epilogue then
  // only scales by alpha and stores.
  // (Only with 16-byte operand loads, whose address registers leave room.)
  const bool c_first = VEC && g.P == nullptr && g.beta != 0.0;
  const double cs = c_first ? g.beta / g.alpha : 0.0;
  f64x4 acc[MI][NI];
  const int64_t ci = i0 + wm * WM + lr, cj = j0 + wn * WN + lk;
  if (c_first && i0 + BM <= g.M && j0 + BN <= g.N) {
    // whole tile inside C: one column pointer walked along the columns
    const double* cp = g.C + ci + cj * g.ldc;
#pragma unroll
    for (int ni = 0; ni < NI; ++ni)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
#pragma unroll
        for (int mi = 0; mi < MI; ++mi) acc[mi][ni][r] = cs * cp[mi * 16];
        cp += 4 * g.ldc;
      }
  } else {
#pragma unroll
    for (int mi = 0; mi < MI; ++mi)
#pragma unroll
      for (int ni = 0; ni < NI; ++ni)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t gi = ci + mi * 16, gj = cj + ni * 16 + 4 * r;
          acc[mi][ni][r] = (c_first && gi < g.M && gj < g.N) ? cs * g.C[gi + gj * g.ldc] : 0.0;
        }
  }

  double ra[OA::PER_T];
  double rb[OB::PER_T];

  if (kbeg < kend) {
    OA::load(ra, g.A, g.lda, i0, g.M, kbeg, kend, tid);
    OB::load(rb, g.B, g.ldb, j0, g.N, kbeg, kend, tid);
    OA::store(lds, ra, tid);
    OB::store(lds + OA::SIZE, rb, tid);
    __syncthreads();
    int buf = 0;
    for (int64_t k0 = kbeg; k0 < kend; k0 += kBK) {
      const bool more = k0 + kBK < kend;
      if (more) {
        OA::load(ra, g.A, g.lda, i0, g.M, k0 + kBK, kend, tid);
        OB::load(rb, g.B, g.ldb, j0, g.N, k0 + kBK, kend, tid);
      }
      const double* la = lds + buf * (OA::SIZE + OB::SIZE);
      const double* lb = la + OA::SIZE;
#pragma unroll
      for (int kk = 0; kk < kBK; kk += 4) {
        double af[MI], bf[NI];
#pragma unroll
        for (int mi = 0; mi < MI; ++mi) af[mi] = OA::frag(la, wm * WM + mi * 16 + lr, kk + lk);
#pragma unroll
        for (int ni = 0; ni < NI; ++ni) bf[ni] = OB::frag(lb, wn * WN + ni * 16 + lr, kk + lk);
#pragma unroll
        for (int mi = 0; mi < MI; ++mi)
#pragma unroll
          for (int ni = 0; ni < NI; ++ni)
            acc[mi][ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[ni], af[mi], acc[mi][ni], 0, 0, 0);
      }
      if (more) {
        double* na = lds + (buf ^ 1) * (OA::SIZE + OB::SIZE);
        OA::store(na, ra, tid);
        OB::store(na + OA::SIZE, rb, tid);
      }
      __syncthreads();
      buf ^= 1;
    }
  }

  // Epilogue: lane l, register r holds C(row l%16, col 4r + l/16) of a sub-tile.
  const int64_t MN = g.M * g.N;
#pragma unroll
  for (int mi = 0; mi < MI; ++mi) {
    const int64_t gi = i0 + wm * WM + mi * 16 + lr;
    if (gi >= g.M) continue;
#pragma unroll
    for (int ni = 0; ni < NI; ++ni) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gj = j0 + wn * WN + ni * 16 + 4 * r + lk;
        if (gj >= g.N) continue;
        const double v = acc[mi][ni][r];
        if (g.P) {
          g.P[(int64_t)blockIdx.z * MN + gi + gj * g.M] = v;
        } else {
          double c = g.alpha * v;
          if (!c_first && g.beta != 0.0) c += g.beta * g.C[gi + gj * g.ldc];
          g.C[gi + gj * g.ldc] = c;
        }
      }
    }
  }
}

// C = alpha * sum_z P_z + beta * C over a 2-D grid (rows in x, columns in
// y), partials added in split order.
__global__ __launch_bounds__(256) void splitk_reduce_kernel(int64_t M, int64_t N, int S,
                                                            const double* __restrict__ P,
                                                            double alpha, double beta,
                                                            double* __restrict__ C, int64_t ldc) {
  const int64_t MN = M * N;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= M) return;
  for (int64_t j = blockIdx.y; j < N; j += gridDim.y) {
    const double* p = P + i + j * M;
    double s = 0.0;
    int z = 0;
    // eight loads in flight, added in split order
    for (; z + 8 <= S; z += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = p[(int64_t)(z + u) * MN];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; z < S; ++z) s += p[(int64_t)z * MN];
    double c = alpha * s;
    if (beta != 0.0) c += beta * C[i + j * ldc];
    C[i + j * ldc] = c;
  }
}

__global__ __launch_bounds__(256) void scale_kernel(int64_t M, int64_t N, double beta, double* C,
                                                    int64_t ldc) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= M) return;
  for (int64_t j = blockIdx.y; j < N; j += gridDim.y)
    C[i + j * ldc] = (beta == 0.0) ? 0.0 : beta * C[i + j * ldc];
}

template <int BM, int BN, bool VEC>
hipError_t launch_tile(hipStream_t st, bool ta, bool tb, GemmF64Args& g, int splits) {
  const int64_t tiles = ceil_div(g.M, BM) * ceil_div(g.N, BN);
  g.tiles_m = (int)ceil_div(g.M, BM);
  dim3 grid((unsigned)tiles, 1, (unsigned)splits);
  dim3 block(kThreads);
  if (!ta && !tb) hipLaunchKernelGGL((dgemm_mfma_kernel<BM, BN, false, false, VEC>), grid, block, 0, st, g);
  else if (ta && !tb) hipLaunchKernelGGL((dgemm_mfma_kernel<BM, BN, true, false, VEC>), grid, block, 0, st, g);
  else if (!ta && tb) hipLaunchKernelGGL((dgemm_mfma_kernel<BM, BN, false, true, VEC>), grid, block, 0, st, g);
  else hipLaunchKernelGGL((dgemm_mfma_kernel<BM, BN, true, true, VEC>), grid, block, 0, st, g);
  return hipGetLastError();
}

// Rows of an M x N elementwise pass in x (256 per block), columns in y.
inline dim3 grid_2d(int64_t M, int64_t N) {
  return dim3((unsigned)ceil_div(M, 256), (unsigned)(N < 65535 ? N : 65535));
}

inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace

int dgemm(hipStream_t st, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
          const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
          int64_t ldc, double* work, size_t work_elems) {
  return dgemm_shaped(st, ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, work, work_elems,
                      false, 0);
}

int dgemm_shaped(hipStream_t st, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
                 const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                 double* C, int64_t ldc, double* work, size_t work_elems, bool small_tiles,
                 int want_splits) {
  if (M <= 0 || N <= 0) return RRF_OK;
  if (K <= 0 || alpha == 0.0) {
    if (beta == 1.0) return RRF_OK;
    hipLaunchKernelGGL(scale_kernel, grid_2d(M, N), dim3(256), 0, st, M, N, beta, C, ldc);
    RRF_CHECK_HIP(hipGetLastError());
    return RRF_OK;
  }
  GemmF64Args g{};
  g.M = M; g.N = N; g.K = K;
  g.alpha = alpha; g.beta = beta;
  g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc;
  g.P = nullptr;

  const bool big = !small_tiles && M >= 128 && N >= 128;
  const int BM = big ? 128 : 64, BN = big ? 128 : 64;
  const int64_t tiles = ceil_div(M, BM) * ceil_div(N, BN);
  // Split K when the tiles alone leave resident slots (two workgroups per CU,
  // 512 on the chip) idle: take the split count s <= 16 (at least 256 of K
  // per split, partials within the workspace) that minimises the time in
  // units of one tile's full-K work, ceil(tiles s / 512) / s, the smallest s
  // on ties.
  const int64_t slots = 512;
  int splits = 1;
  if (want_splits > 1) {
    splits = (int)std::min<int64_t>(want_splits, std::max<int64_t>(1, K / kBK));
    while (splits > 1 && (size_t)splits * M * N > work_elems) --splits;
  } else if (tiles < slots && K >= 2 * 256) {
    double best = 1.0;
    for (int64_t s = 2; s <= 16 && K / s >= 256; ++s) {
      if ((size_t)(s * M * N) > work_elems) break;
      const double t = (double)ceil_div(tiles * s, slots) / (double)s;
      if (t < best - 1e-12) {
        best = t;
        splits = (int)s;
      }
    }
  }
  g.kchunk = round_up(ceil_div(K, splits), kBK);
  splits = (int)ceil_div(K, g.kchunk);
  if (splits > 1) g.P = work;
  // 16-byte loads need 16-byte aligned column starts of both operands.
  const bool vec = aligned16(A) && aligned16(B) && (lda % 2 == 0) && (ldb % 2 == 0);

  // Algorithmic traffic: op(A) and op(B) read once, C written (and read when
  // beta != 0); partial sums count against the reduction kernel.
  const double gbytes = 8.0 * ((double)M * K + (double)K * N +
                               (splits > 1 ? 0.0 : (beta != 0.0 ? 2.0 : 1.0) * M * N));
  int tok = trace_begin(st, gemm_trace_class(BM, ta, tb), 2.0 * M * N * K, gbytes);
  hipError_t e;
  if (big) e = vec ? launch_tile<128, 128, true>(st, ta, tb, g, splits)
                   : launch_tile<128, 128, false>(st, ta, tb, g, splits);
  else e = vec ? launch_tile<64, 64, true>(st, ta, tb, g, splits)
               : launch_tile<64, 64, false>(st, ta, tb, g, splits);
  trace_end(st, tok);
  if (e != hipSuccess) return set_hip_error(e, "dgemm launch", __FILE__, __LINE__);
  if (splits > 1) return splitk_reduce(st, M, N, splits, work, alpha, beta, C, ldc);
  return RRF_OK;
}

int splitk_reduce(hipStream_t st, int64_t M, int64_t N, int splits, const double* P, double alpha,
                  double beta, double* C, int64_t ldc) {
  int tok = trace_begin(st, kTrSplitReduce, (double)splits * M * N,
                        8.0 * (splits + (beta != 0.0 ? 2.0 : 1.0)) * M * N);
  hipLaunchKernelGGL(splitk_reduce_kernel, grid_2d(M, N), dim3(256), 0, st, M, N, splits, P,
                     alpha, beta, C, ldc);
  trace_end(st, tok);
  RRF_CHECK_HIP(hipGetLastError());
  return RRF_OK;
}

}  // namespace rrf
