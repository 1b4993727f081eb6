// Split-bfloat16 six-term products of binary64 matrices on the bfloat16
// matrix cores: the update products of the RRF_PREC_BF16_X6 mode.
//
// C = alpha op(A) op(B) + beta C, column-major, op = N or T, A, B and C
// binary64 in HBM. Every operand element x is split while it is staged into
// LDS into three bfloat16 parts of its binary32 rounding:
//   x32 = x rounded to binary32,
//   hi  = x32 rounded to bfloat16,
//   mid = (x32 - hi) rounded to bfloat16,
//   lo  = (x32 - hi - mid) rounded to bfloat16,
// all to nearest, ties to even, each subtraction exact in binary32, so that
// hi + mid + lo = x32 (24 bits in three 8-bit parts). Of the nine products of
// (hi_a + mid_a + lo_a)(hi_b + mid_b + lo_b) the six leading ones are kept,
//   hi hi + hi mid + mid hi + hi lo + lo hi + mid mid,
// each exact in binary32; the dropped mid lo + lo mid + lo lo is below about
// 2^-23 |a| |b| per term, and the binary32 roundings of the operands add
// 2^-24 each. The terms of one K slice (32) are accumulated in binary32 by
// v_mfma_f32_16x16x32_bf16 and every slice's sum is added to a binary64
// accumulator, so the rounding of the binary32 sums grows with the slice,
// not with K. The result is widened for alpha, beta and the store.
//
// Design: 512-thread workgroups (eight wave64s, 4 x 2) on a BM x BN tile of
// C, (BM/4) x (BN/2) per wave in 16 x 16 sub-tiles; K in slices of 32 through
// two LDS buffers (hi, mid and lo of both operands as [mn][k] rows of 32
// bfloat16 plus 8 of padding), the HBM loads of slice t+1 in flight while the
// matrix cores work on slice t. One workgroup per CU (120 KB of LDS).
// Operand staging and the transposed-tile epilogue follow the three-pass
// kernel (gemm_x3.hip). A rank-b update reads its large operand once at
// 32 flop per byte, so six bfloat16 passes (2.5 PFLOP/s / 6 = 417 TFLOP/s
// equivalent) still leave the kernel bound by HBM.
#include "common.hpp"
#include "kernels.hpp"
#include "trace.hpp"

namespace rrf {

namespace {

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 512;
constexpr int kBK = 32;        // K per LDS slice: one MFMA step
constexpr int kLK = kBK + 8;   // LDS row length in bfloat16
constexpr int kParts = 3;

struct X6Args {
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

__device__ inline uint32_t pack_bf16(float a, float b) {
  const f32x2 v = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}
__device__ inline float lo_half(uint32_t w) { return __uint_as_float(w << 16); }
__device__ inline float hi_half(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

// hi, mid and lo words of four consecutive values (two bfloat16 per word).
__device__ inline void split4(const double (&x)[4], uint2& hi, uint2& mid, uint2& lo) {
  float f0 = (float)x[0], f1 = (float)x[1], f2 = (float)x[2], f3 = (float)x[3];
  // hi is the rounding of the binary32 value; without this the compiler may
  // fuse the two roundings into one directly from binary64
  asm volatile("" : "+v"(f0), "+v"(f1), "+v"(f2), "+v"(f3));
  const uint32_t h0 = pack_bf16(f0, f1), h1 = pack_bf16(f2, f3);
  const float r0 = f0 - lo_half(h0), r1 = f1 - hi_half(h0);
  const float r2 = f2 - lo_half(h1), r3 = f3 - hi_half(h1);
  const uint32_t m0 = pack_bf16(r0, r1), m1 = pack_bf16(r2, r3);
  hi = make_uint2(h0, h1);
  mid = make_uint2(m0, m1);
  lo = make_uint2(pack_bf16(r0 - lo_half(m0), r1 - hi_half(m0)),
                  pack_bf16(r2 - lo_half(m1), r3 - hi_half(m1)));
}

// One operand tile, MN x kBK of op(X), staged as groups of four consecutive
// k per thread. KMAJOR: X is contiguous along k in HBM (A for op = T, B for
// op = N).
template <int MN, bool KMAJOR, bool VEC>
struct Stage {
  static constexpr int G = MN * kBK / 4 / kThreads;
  static_assert(G >= 1 && G * 4 * kThreads == MN * kBK, "operand tile shape");

  __device__ static inline void coord(int tid, int j, int& mn, int& kq) {
    const int g = tid + kThreads * j;
    if (KMAJOR) {
      mn = g / (kBK / 4);
      kq = g % (kBK / 4);
    } else {
      mn = g % MN;
      kq = g / MN;
    }
  }
  // Slice [k0, k0 + kBK) of rows/columns [mn0, mn0 + MN); entries beyond
  // mn_end or k_end read as zero.
  __device__ static inline void load(double (&r)[G][4], const double* X, int64_t ld, int64_t mn0,
                                     int64_t mn_end, int64_t k0, int64_t k_end, int tid) {
#pragma unroll
    for (int j = 0; j < G; ++j) {
      int mn, kq;
      coord(tid, j, mn, kq);
      const int64_t gm = mn0 + mn, gk = k0 + 4 * kq;
      const bool row = gm < mn_end;
      if (KMAJOR) {
        const double* p = X + gk + gm * ld;
        if (VEC && row && gk + 4 <= k_end) {
          const double2 a = *reinterpret_cast<const double2*>(p);
          const double2 b = *reinterpret_cast<const double2*>(p + 2);
          r[j][0] = a.x;
          r[j][1] = a.y;
          r[j][2] = b.x;
          r[j][3] = b.y;
        } else {
#pragma unroll
          for (int t = 0; t < 4; ++t) r[j][t] = (row && gk + t < k_end) ? p[t] : 0.0;
        }
      } else {
        const double* p = X + gm + gk * ld;
#pragma unroll
        for (int t = 0; t < 4; ++t) r[j][t] = (row && gk + t < k_end) ? p[t * ld] : 0.0;
      }
    }
  }
  // parts: kParts arrays of MN x kLK bfloat16, `stride` elements apart
  __device__ static inline void store(uint16_t* parts, int stride, const double (&r)[G][4],
                                      int tid) {
#pragma unroll
    for (int j = 0; j < G; ++j) {
      int mn, kq;
      coord(tid, j, mn, kq);
      uint2 h, m, l;
      split4(r[j], h, m, l);
      const int off = mn * kLK + 4 * kq;
      *reinterpret_cast<uint2*>(parts + off) = h;
      *reinterpret_cast<uint2*>(parts + stride + off) = m;
      *reinterpret_cast<uint2*>(parts + 2 * stride + off) = l;
    }
  }
};

template <int BM, int BN, bool TA, bool TB, bool VEC>
__global__ __launch_bounds__(kThreads, 1) void gemm_x6_kernel(X6Args g) {
  using SA = Stage<BM, TA, VEC>;   // op(A) is contiguous along k when A is transposed
  using SB = Stage<BN, !TB, VEC>;  // op(B) when B is not
  constexpr int LA = BM * kLK, LB = BN * kLK;  // bfloat16 per part
  constexpr int BUF = kParts * (LA + LB);
  constexpr int WM = BM / 4, WN = BN / 2, MI = WM / 16, NI = WN / 16;
  static_assert(MI >= 1 && NI >= 1, "wave tile");
  __shared__ __attribute__((aligned(16))) uint16_t lds[2 * BUF];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t i0 = (int64_t)(blockIdx.x % g.tiles_m) * BM;
  const int64_t j0 = (int64_t)(blockIdx.x / g.tiles_m) * BN;
  const int64_t kbeg = (int64_t)blockIdx.z * g.kchunk;
  const int64_t kend = kbeg + g.kchunk < g.K ? kbeg + g.kchunk : g.K;

  double acc[MI][NI][4];
#pragma unroll
  for (int mi = 0; mi < MI; ++mi)
#pragma unroll
    for (int ni = 0; ni < NI; ++ni)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[mi][ni][r] = 0.0;

  if (kbeg < kend) {
    double ra[SA::G][4], rb[SB::G][4];
    SA::load(ra, g.A, g.lda, i0, g.M, kbeg, kend, tid);
    SB::load(rb, g.B, g.ldb, j0, g.N, kbeg, kend, tid);
    SA::store(lds, LA, ra, tid);
    SB::store(lds + kParts * LA, LB, rb, tid);
    __syncthreads();
    int buf = 0;
    for (int64_t k0 = kbeg; k0 < kend; k0 += kBK) {
      const bool more = k0 + kBK < kend;
      if (more) {
        SA::load(ra, g.A, g.lda, i0, g.M, k0 + kBK, kend, tid);
        SB::load(rb, g.B, g.ldb, j0, g.N, k0 + kBK, kend, tid);
      }
      const uint16_t* a0 = lds + buf * BUF;         // hi, mid, lo of A, LA apart
      const uint16_t* b0 = a0 + kParts * LA;        // hi, mid, lo of B, LB apart
      const int frag = (lane & 15) * kLK + 8 * (lane >> 4);
      bf16x8 fa[MI][kParts];
#pragma unroll
      for (int mi = 0; mi < MI; ++mi) {
        const int off = (wm * WM + mi * 16) * kLK + frag;
#pragma unroll
        for (int p = 0; p < kParts; ++p)
          fa[mi][p] = *reinterpret_cast<const bf16x8*>(a0 + p * LA + off);
      }
#pragma unroll
      for (int ni = 0; ni < NI; ++ni) {
        const int off = (wn * WN + ni * 16) * kLK + frag;
        const bf16x8 fbh = *reinterpret_cast<const bf16x8*>(b0 + off);
        const bf16x8 fbm = *reinterpret_cast<const bf16x8*>(b0 + LB + off);
        const bf16x8 fbl = *reinterpret_cast<const bf16x8*>(b0 + 2 * LB + off);
#pragma unroll
        for (int mi = 0; mi < MI; ++mi) {
          // smallest terms first; the transposed tile takes B's fragment first
          f32x4 s = {0.f, 0.f, 0.f, 0.f};
          s = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fbm, fa[mi][1], s, 0, 0, 0);
          s = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fbl, fa[mi][0], s, 0, 0, 0);
          s = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fbh, fa[mi][2], s, 0, 0, 0);
          s = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fbm, fa[mi][0], s, 0, 0, 0);
          s = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fbh, fa[mi][1], s, 0, 0, 0);
          s = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fbh, fa[mi][0], s, 0, 0, 0);
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[mi][ni][r] += (double)s[r];
        }
      }
      if (more) {
        uint16_t* na = lds + (buf ^ 1) * BUF;
        SA::store(na, LA, ra, tid);
        SB::store(na + kParts * LA, LB, rb, tid);
      }
      __syncthreads();
      buf ^= 1;
    }
  }

  // lane l, entry r of sub-tile (mi, ni) holds C(row l % 16, column
  // 4 (l / 16) + r) of that sub-tile
  const int64_t MN = g.M * g.N;
#pragma unroll
  for (int mi = 0; mi < MI; ++mi) {
    const int64_t m = i0 + wm * WM + mi * 16 + (lane & 15);
    if (m >= g.M) continue;
#pragma unroll
    for (int ni = 0; ni < NI; ++ni)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t n = j0 + wn * WN + ni * 16 + 4 * (lane >> 4) + r;
        if (n >= g.N) continue;
        const double v = acc[mi][ni][r];
        if (g.P) {
          g.P[(int64_t)blockIdx.z * MN + m + n * g.M] = v;
        } else {
          double c = g.alpha * v;
          if (g.beta != 0.0) c += g.beta * g.C[m + n * g.ldc];
          g.C[m + n * g.ldc] = c;
        }
      }
  }
}

template <int BM, int BN, bool VEC>
hipError_t launch(hipStream_t st, bool ta, bool tb, X6Args& g, int splits) {
  const int64_t tiles = ceil_div(g.M, BM) * ceil_div(g.N, BN);
  g.tiles_m = (int)ceil_div(g.M, BM);
  const dim3 grid((unsigned)tiles, 1, (unsigned)splits), block(kThreads);
  if (!ta && !tb) hipLaunchKernelGGL((gemm_x6_kernel<BM, BN, false, false, VEC>), grid, block, 0, st, g);
  else if (ta && !tb) hipLaunchKernelGGL((gemm_x6_kernel<BM, BN, true, false, VEC>), grid, block, 0, st, g);
  else if (!ta && tb) hipLaunchKernelGGL((gemm_x6_kernel<BM, BN, false, true, VEC>), grid, block, 0, st, g);
  else hipLaunchKernelGGL((gemm_x6_kernel<BM, BN, true, true, VEC>), grid, block, 0, st, g);
  return hipGetLastError();
}

inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace

int gemm_x6(hipStream_t st, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
            const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
            int64_t ldc, double* work, size_t work_elems) {
  if (M <= 0 || N <= 0) return RRF_OK;
  if (K <= 0 || alpha == 0.0)  // nothing to multiply: C = beta C as the FP64 GEMM does it
    return dgemm(st, ta, tb, M, N, 0, 0.0, A, lda, B, ldb, beta, C, ldc, nullptr, 0);
  X6Args g{};
  g.M = M; g.N = N; g.K = K;
  g.alpha = alpha; g.beta = beta;
  g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc;

  const bool big = (M >= 128 && N >= 128);
  const int BM = big ? 128 : 64, BN = big ? 128 : 64;
  const int64_t tiles = ceil_div(M, BM) * ceil_div(N, BN);
  // K split as in the FP64 GEMM: when the tiles leave CUs idle (one
  // workgroup per CU), the split count s <= 16 (at least 256 of K per split,
  // partials within the workspace) minimising ceil(tiles s / 256) / s.
  const int64_t slots = 256;
  int splits = 1;
  if (tiles < slots && K >= 2 * 256) {
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
  g.P = splits > 1 ? work : nullptr;
  const bool vec = aligned16(A) && aligned16(B) && (lda % 2 == 0) && (ldb % 2 == 0);

  const double gbytes = 8.0 * ((double)M * K + (double)K * N +
                               (splits > 1 ? 0.0 : (beta != 0.0 ? 2.0 : 1.0) * M * N));
  int tok = trace_begin(st, big ? kTrGemmX6 : kTrGemmX6Small, 2.0 * M * N * K, gbytes);
  hipError_t e;
  if (big) e = vec ? launch<128, 128, true>(st, ta, tb, g, splits)
                   : launch<128, 128, false>(st, ta, tb, g, splits);
  else e = vec ? launch<64, 64, true>(st, ta, tb, g, splits)
               : launch<64, 64, false>(st, ta, tb, g, splits);
  trace_end(st, tok);
  if (e != hipSuccess) return set_hip_error(e, "gemm_x6 launch", __FILE__, __LINE__);
  if (splits > 1) return splitk_reduce(st, M, N, splits, work, alpha, beta, C, ldc);
  return RRF_OK;
}

}  // namespace rrf
