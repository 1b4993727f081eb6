// Mixed-precision sketch of randUTV: bfloat16 inputs, FP32 accumulation.
//
// The sketch of Alg. 3, Y = (T22^T T22)^q T22^T G, only has to capture the
// dominant right singular subspace of T22; the QR of Y and every update of
// T, U and V stay in FP64. In the mixed mode
//  * T22 is scaled by a power of two 2^-e (max|T22| 2^-e in [0.5, 1)) and
//    rounded to bfloat16 twice, as Tb (M x N) and its transpose Tbt (N x M),
//    so that both products of the power iteration read their operand along
//    the inner dimension;
//  * G is rounded as it is (standard normal values are in range);
//  * every product is a "TN" GEMM C = A^T B with both operands contiguous
//    along the inner dimension K, on the bfloat16 matrix cores
//    (v_mfma_f32_16x16x32_bf16), FP32 accumulation, split over K with the
//    partials summed in a fixed order;
//  * between products each column of the FP32 result is scaled by its own
//    power of two (max in [0.5, 1)) and rounded to bfloat16; positive column
//    scalings commute with the products and leave the column space of Y
//    unchanged, they only keep the values inside the binary32 range;
//  * the last product is widened to FP64 exactly.
// Rounding is to nearest, ties to even, directly from the source format.
//
// The products stream T22 in bfloat16 (2 bytes per element per product)
// instead of FP64 (8 bytes, and FP64 matrix-core rates), so the sketch is
// HBM-bound at b <= 256.
#include <algorithm>
#include <climits>
#include <cfloat>

#include "batched.hpp"
#include "common.hpp"
#include "context.hpp"
#include "kernels.hpp"
#include "trace.hpp"

namespace rrf {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// --- rounding --------------------------------------------------------------

// binary64 -> bfloat16 bits, round to nearest even, directly (no binary32
// step). The leading bit's exponent is clamped at -126, below which the
// quantum is 2^-133 (gradual underflow). Inputs here are pre-scaled to
// magnitudes below 1, so there is no overflow.
__device__ inline uint16_t bf16_from_f64(double x) {
  if (x == 0.0) return (uint16_t)(__double_as_longlong(x) >> 48);  // keeps the sign
  int lead = ilogb(x);
  if (lead < -126) lead = -126;
  const double q = rint(scalbn(x, 7 - lead));  // integer multiple of the quantum
  const float r = (float)scalbn(q, lead - 7);  // exact: at most 8 significant bits
  return (uint16_t)(__float_as_uint(r) >> 16);
}

// binary32 -> bfloat16 bits, round to nearest even (finite inputs).
__device__ inline uint16_t bf16_from_f32(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// 2^-e with m 2^-e in [0.5, 1) (frexp convention); 1 for m = 0.
__device__ inline double pow2_scale(double m) {
  if (!(m > 0.0)) return 1.0;
  int e;
  frexp(m, &e);
  return ldexp(1.0, -e);
}

// --- max|X| ----------------------------------------------------------------

// word = max over X of |x| as binary64 bits (non-negative doubles order like
// their bit patterns). The word must be zero at launch. Blocks take 256 rows
// and stride over the columns, so one atomic per block (a few thousand per
// matrix) reaches the word.
__global__ __launch_bounds__(256) void maxabs_kernel(int64_t rows, int64_t cols,
                                                     const double* __restrict__ X, int64_t ld,
                                                     unsigned long long* word) {
  __shared__ double red[4];
  // each thread takes two consecutive rows (one 16-byte load when X and ld
  // allow) of four columns per iteration, so eight values are in flight
  const bool pair = ((reinterpret_cast<uintptr_t>(X) & 15u) == 0) && (ld % 2 == 0);
  const int64_t i = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 2;
  double m[4] = {0.0, 0.0, 0.0, 0.0};
  if (i < rows) {
    const bool two = i + 1 < rows;
    const int64_t step = gridDim.y;
    int64_t j = blockIdx.y;
    for (; j + 3 * step < cols; j += 4 * step) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double* p = X + i + (j + u * step) * ld;
        if (pair && two) {
          const double2 v = *reinterpret_cast<const double2*>(p);
          m[u] = fmax(m[u], fmax(fabs(v.x), fabs(v.y)));
        } else {
          m[u] = fmax(m[u], fabs(p[0]));
          if (two) m[u] = fmax(m[u], fabs(p[1]));
        }
      }
    }
    for (; j < cols; j += step) {
      const double* p = X + i + j * ld;
      m[0] = fmax(m[0], fabs(p[0]));
      if (two) m[0] = fmax(m[0], fabs(p[1]));
    }
  }
  double mm = fmax(fmax(m[0], m[1]), fmax(m[2], m[3]));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mm = fmax(mm, __shfl_xor(mm, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mm;
  __syncthreads();
  if (threadIdx.x == 0) {
    mm = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    if (mm > 0.0) atomicMax(word, (unsigned long long)__double_as_longlong(mm));
  }
}

// X *= s or X /= s with s = pow2_scale(max|X|) from `word`: multiplication
// by a power of two, exact for every entry in the normal range.
__global__ __launch_bounds__(256) void scale_pow2_kernel(int64_t rows, int64_t cols, double* X,
                                                         int64_t ld,
                                                         const unsigned long long* word,
                                                         bool inverse, int guard_exp) {
  const double s0 = pow2_scale(__longlong_as_double((long long)*word));
  // guarded: only a max|X| with binary exponent beyond +-guard_exp is scaled
  if (guard_exp > 0 && s0 >= ldexp(1.0, -guard_exp) && s0 <= ldexp(1.0, guard_exp)) return;
  const double s = inverse ? 1.0 / s0 : s0;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= rows) return;
  for (int64_t j = blockIdx.y; j < cols; j += gridDim.y) X[i + j * ld] *= s;
}

// --- ||X||_F for the early stop of randUTV ---------------------------------

// parts[blockIdx] = sum of (s x)^2 over rows [256 bx, 256 bx + 256) and the
// columns bx.y, bx.y + gridDim.y, ...; s = pow2_scale of the max in `word`
// (a bound on |X|, so no square overflows). Fixed-order sums throughout.
__global__ __launch_bounds__(256) void sumsq_kernel(int64_t rows, int64_t cols,
                                                    const double* __restrict__ X, int64_t ld,
                                                    const unsigned long long* word,
                                                    double* __restrict__ parts) {
  __shared__ double red[4];
  const double s = pow2_scale(__longlong_as_double((long long)*word));
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double acc = 0.0;
  if (i < rows)
    for (int64_t j = blockIdx.y; j < cols; j += gridDim.y) {
      const double v = X[i + j * ld] * s;
      acc = fma(v, v, acc);
    }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0)
    parts[blockIdx.x + (int64_t)blockIdx.y * gridDim.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// out = sqrt(sum of parts) / s.
__global__ __launch_bounds__(256) void sumsq_finish_kernel(const double* __restrict__ parts,
                                                           int count,
                                                           const unsigned long long* word,
                                                           double* out) {
  __shared__ double red[4];
  const double s = pow2_scale(__longlong_as_double((long long)*word));
  double acc = 0.0;
  for (int k = threadIdx.x; k < count; k += 256) acc += parts[k];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) *out = sqrt((red[0] + red[1]) + (red[2] + red[3])) / s;
}

// --- binary64 -> bfloat16, optionally scaled and transposed ----------------

// out (rows x cols, ld ldo) = bf16(X * s), outT (cols x rows, ld ldot) its
// transpose when non-null; s = pow2_scale(max) from `word` when non-null,
// else 1. Rows [rows, ldo) of out and [cols, ldot) of outT are zero-filled so
// that 16-byte loads along the inner dimension never need a ragged edge.
// 64 x 64 tiles; thread (q, g) converts rows 4q..4q+3 of columns g, g+16,
// g+32, g+48 (two 16-byte loads and one 8-byte store per column), and the
// transpose goes through LDS to be stored the same way. ldo and ldot are
// multiples of 8, so the 8-byte stores are aligned.
__global__ __launch_bounds__(256) void to_bf16_kernel(int64_t rows, int64_t cols,
                                                      const double* __restrict__ X, int64_t ld,
                                                      const unsigned long long* word,
                                                      uint16_t* __restrict__ out, int64_t ldo,
                                                      uint16_t* __restrict__ outT, int64_t ldot) {
  __shared__ uint16_t tile[64][68];  // [column][row]
  const double s = word ? pow2_scale(__longlong_as_double((long long)*word)) : 1.0;
  const int64_t r0 = (int64_t)blockIdx.x * 64, c0 = (int64_t)blockIdx.y * 64;
  const int q = threadIdx.x & 15, g = threadIdx.x >> 4;
  const bool vec = ((reinterpret_cast<uintptr_t>(X) & 15u) == 0) && (ld % 2 == 0);
  const int64_t r = r0 + 4 * q;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int cc = g + 16 * u;
    const int64_t c = c0 + cc;
    double x[4] = {0.0, 0.0, 0.0, 0.0};
    if (c < cols) {
      const double* p = X + r + c * ld;
      if (vec && r + 3 < rows) {
        const double2 a = *reinterpret_cast<const double2*>(p);
        const double2 b = *reinterpret_cast<const double2*>(p + 2);
        x[0] = a.x; x[1] = a.y; x[2] = b.x; x[3] = b.y;
      } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) x[t] = (r + t < rows) ? p[t] : 0.0;
      }
    }
    uint16_t h[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) h[t] = (c < cols && r + t < rows) ? bf16_from_f64(x[t] * s) : 0;
    if (r < ldo && c < cols) {
      const uint2 w = make_uint2((uint32_t)h[0] | ((uint32_t)h[1] << 16),
                                 (uint32_t)h[2] | ((uint32_t)h[3] << 16));
      *reinterpret_cast<uint2*>(out + r + c * ldo) = w;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) tile[cc][4 * q + t] = h[t];
  }
  if (!outT) return;
  __syncthreads();
  // outT(c, rr) = X(rr, c): thread (q, g) stores columns 4q..4q+3 of rows
  // g, g+16, g+32, g+48 of outT's tile
  const int64_t c = c0 + 4 * q;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int rr = g + 16 * u;
    const int64_t rw = r0 + rr;
    if (rw >= rows || c >= ldot) continue;
    uint16_t h[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) h[t] = (c + t < cols) ? tile[4 * q + t][rr] : (uint16_t)0;
    const uint2 w = make_uint2((uint32_t)h[0] | ((uint32_t)h[1] << 16),
                               (uint32_t)h[2] | ((uint32_t)h[3] << 16));
    *reinterpret_cast<uint2*>(outT + c + rw * ldot) = w;
  }
}

// --- C = A^T B on the bfloat16 matrix cores --------------------------------

constexpr int kBM = 128, kBN = 128, kBK = 64;
constexpr int kLK = kBK + 8;  // LDS row length in bfloat16 (16-byte pad)
constexpr int kThreads = 256;

struct GemmBf16Args {
  int64_t M, N, K;
  const uint16_t* A;  // K x M, ld lda (multiple of 8), rows [K, lda) zero
  int64_t lda;
  const uint16_t* B;  // K x N, ld ldb (multiple of 8), rows [K, ldb) zero
  int64_t ldb;
  float* P;           // partials: P[z * M * N + m + n * M]
  int64_t kchunk;     // multiple of kBK
  int tiles_m;
};

// Loads the 128 x 64 slice (rows mn0.., inner k0..) of a K-contiguous
// operand as 16-byte chunks: 1024 chunks, four per thread.
__device__ inline void load_slice(uint4 (&reg)[4], const uint16_t* X, int64_t ld, int64_t mn0,
                                  int64_t mn_end, int64_t k0, int64_t k_end, int tid) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int c = tid + kThreads * i;
    const int row = c >> 3, part = c & 7;
    const int64_t mn = mn0 + row, k = k0 + part * 8;
    if (mn < mn_end && k < k_end)
      reg[i] = *reinterpret_cast<const uint4*>(X + k + mn * ld);
    else
      reg[i] = make_uint4(0, 0, 0, 0);
  }
}

__device__ inline void store_slice(uint16_t* lds, const uint4 (&reg)[4], int tid) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int c = tid + kThreads * i;
    const int row = c >> 3, part = c & 7;
    *reinterpret_cast<uint4*>(lds + row * kLK + part * 8) = reg[i];
  }
}

__global__ __launch_bounds__(kThreads, 2) void gemm_bf16_tn_kernel(GemmBf16Args g) {
  __shared__ __attribute__((aligned(16))) uint16_t lds[2][(kBM + kBN) * kLK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;  // 2 x 2 waves of 64 x 64
  const int tm = blockIdx.x % g.tiles_m, tn = blockIdx.x / g.tiles_m;
  const int64_t m0 = (int64_t)tm * kBM, n0 = (int64_t)tn * kBN;
  const int64_t kbeg = (int64_t)blockIdx.z * g.kchunk;
  const int64_t kend = std::min(kbeg + g.kchunk, g.K);
  // 16-byte chunks exist up to the zero-padded end of the inner dimension
  const int64_t kpad = (g.K + 7) & ~(int64_t)7;
  const int64_t kload_end = std::min(kbeg + g.kchunk, kpad);

  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  if (kbeg < kend) {
    uint4 ra[4], rb[4];
    load_slice(ra, g.A, g.lda, m0, g.M, kbeg, kload_end, tid);
    load_slice(rb, g.B, g.ldb, n0, g.N, kbeg, kload_end, tid);
    store_slice(lds[0], ra, tid);
    store_slice(lds[0] + kBM * kLK, rb, tid);
    __syncthreads();
    int buf = 0;
    for (int64_t k0 = kbeg; k0 < kend; k0 += kBK) {
      const bool more = k0 + kBK < kend;
      if (more) {
        load_slice(ra, g.A, g.lda, m0, g.M, k0 + kBK, kload_end, tid);
        load_slice(rb, g.B, g.ldb, n0, g.N, k0 + kBK, kload_end, tid);
      }
      const uint16_t* la = lds[buf];
      const uint16_t* lb = lds[buf] + kBM * kLK;
#pragma unroll
      for (int ks = 0; ks < kBK; ks += 32) {
        bf16x8 af[4], bfr[4];
        // lane l: row l % 16 of the 16 x 32 operand, inner 8 (l / 16) .. + 7
#pragma unroll
        for (int i = 0; i < 4; ++i)
          af[i] = *reinterpret_cast<const bf16x8*>(
              la + (wm * 64 + i * 16 + (lane & 15)) * kLK + ks + 8 * (lane >> 4));
#pragma unroll
        for (int j = 0; j < 4; ++j)
          bfr[j] = *reinterpret_cast<const bf16x8*>(
              lb + (wn * 64 + j * 16 + (lane & 15)) * kLK + ks + 8 * (lane >> 4));
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
      }
      if (more) {
        store_slice(lds[buf ^ 1], ra, tid);
        store_slice(lds[buf ^ 1] + kBM * kLK, rb, tid);
      }
      __syncthreads();
      buf ^= 1;
    }
  }
  // lane l, register r holds D(row 4 (l / 16) + r, column l % 16) of a sub-tile
  float* P = g.P + (int64_t)blockIdx.z * g.M * g.N;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t n = n0 + wn * 64 + j * 16 + (lane & 15);
      if (n >= g.N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + r;
        if (m < g.M) P[m + n * g.M] = acc[i][j][r];
      }
    }
  }
}

// --- sum of the split partials, then per-column bfloat16 or FP64 ----------

// One workgroup per column n: s = sum_z P_z(:, n) in split order, kept in
// LDS when it fits (else in `col`, a global column buffer), then either
// out16(:, n) = bf16(s pow2_scale(max|s|)) with rows [M, ld16) zeroed, or
// out64(:, n) = s widened.
constexpr int kColThreads = 1024;
constexpr int64_t kColLds = 32768;  // floats of the column kept in LDS

__global__ __launch_bounds__(kColThreads) void reduce_columns_kernel(
    int64_t M, int64_t N, int S, const float* __restrict__ P, uint16_t* __restrict__ out16,
    int64_t ld16, double* __restrict__ out64, int64_t ld64, float* __restrict__ col) {
  extern __shared__ float sc[];
  __shared__ float red[kColThreads];
  const int64_t n = blockIdx.x;
  const int tid = threadIdx.x;
  const bool in_lds = M <= kColLds;
  float* c = in_lds ? sc : col + n * M;
  float m = 0.f;
  for (int64_t i = tid; i < M; i += kColThreads) {
    float s = 0.f;
    for (int z = 0; z < S; ++z) s += P[(int64_t)z * M * N + i + n * M];
    c[i] = s;
    m = fmaxf(m, fabsf(s));
  }
  if (out64) {
    for (int64_t i = tid; i < M; i += kColThreads) out64[i + n * ld64] = (double)c[i];
    return;
  }
  red[tid] = m;
  __syncthreads();
  for (int w = kColThreads / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] = fmaxf(red[tid], red[tid + w]);
    __syncthreads();
  }
  const float s = (float)pow2_scale((double)red[0]);
  for (int64_t i = tid; i < ld16; i += kColThreads)
    out16[i + n * ld16] = (i < M) ? bf16_from_f32(c[i] * s) : (uint16_t)0;
}

// --- batched forms (the mixed sketch of the batched randUTV) ---------------

// One workgroup per (problem, 256-row block): max over its rows and all
// columns, one atomic per workgroup.
__global__ __launch_bounds__(256) void maxabs_batched_kernel(const MaxDesc* __restrict__ descs) {
  __shared__ double red[4];
  const MaxDesc d = descs[blockIdx.y];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if ((int64_t)blockIdx.x * 256 >= d.rows) return;
  double m = 0.0;
  if (i < d.rows)
    for (int64_t j = 0; j < d.cols; ++j) m = fmax(m, fabs(d.X[i + j * d.ld]));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    if (m > 0.0) atomicMax(d.word, (unsigned long long)__double_as_longlong(m));
  }
}

// to_bf16_kernel per problem: blockIdx.x walks the problem's 64 x 64 tiles
// (rows up to max(rows, ldo), columns up to max(cols, ldot)).
__global__ __launch_bounds__(256) void to_bf16_batched_kernel(const Bf16Desc* __restrict__ descs) {
  __shared__ uint16_t tile[64][65];
  const Bf16Desc d = descs[blockIdx.y];
  const int64_t R = d.rows > d.ldo ? d.rows : d.ldo;
  const int64_t C = d.outT ? (d.cols > d.ldot ? d.cols : d.ldot) : d.cols;
  const int64_t tr = (R + 63) / 64;
  if ((int64_t)blockIdx.x >= tr * ((C + 63) / 64)) return;
  const double s = d.word ? pow2_scale(__longlong_as_double((long long)*d.word)) : 1.0;
  const int64_t r0 = (int64_t)(blockIdx.x % tr) * 64, c0 = (int64_t)(blockIdx.x / tr) * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int cc = ty; cc < 64; cc += 4) {
    const int64_t r = r0 + tx, c = c0 + cc;
    uint16_t v = 0;
    if (r < d.rows && c < d.cols) v = bf16_from_f64(d.X[r + c * d.ld] * s);
    if (r < d.ldo && c < d.cols) d.out[r + c * d.ldo] = v;
    tile[cc][tx] = v;
  }
  if (!d.outT) return;
  __syncthreads();
  for (int rr = ty; rr < 64; rr += 4) {
    const int64_t c = c0 + tx, r = r0 + rr;
    if (c < d.ldot && r < d.rows) d.outT[c + r * d.ldot] = (c < d.cols) ? tile[tx][rr] : (uint16_t)0;
  }
}

// 128 x 32 output tiles of every problem (4 waves of 32 x 32, 2 x 2 blocks of
// v_mfma_f32_16x16x32_bf16), K in slices of 64 through double-buffered LDS;
// the workgroup finds its problem by binary search of the running tile counts.
constexpr int kGBM = 128, kGBN = 32;

__global__ __launch_bounds__(kThreads) void gemm_bf16_grouped_kernel(
    const Bf16GemmDesc* __restrict__ descs, const int* __restrict__ prefix, int count) {
  __shared__ __attribute__((aligned(16))) uint16_t lds[2][(kGBM + kGBN) * kLK];
  const int bid = blockIdx.x;
  int lo = 0, hi = count;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (prefix[mid] <= bid) lo = mid;
    else hi = mid;
  }
  const Bf16GemmDesc g = descs[lo];
  const int t = bid - prefix[lo];
  const int64_t tiles_m = (g.M + kGBM - 1) / kGBM;
  const int64_t m0 = (int64_t)(t % tiles_m) * kGBM, n0 = (int64_t)(t / tiles_m) * kGBN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;  // 4 x 1 waves
  const int64_t kpad = (g.K + 7) & ~(int64_t)7;

  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  // A: 128 x 64 slice = 1024 chunks of 16 bytes (four per thread); B: 32 x 64
  // = 256 chunks (one per thread)
  auto load = [&](uint4 (&ra)[4], uint4& rb, int64_t k0) {
    load_slice(ra, g.A, g.lda, m0, g.M, k0, kpad, tid);
    const int row = tid >> 3, part = tid & 7;
    const int64_t n = n0 + row, k = k0 + part * 8;
    rb = (n < g.N && k < kpad) ? *reinterpret_cast<const uint4*>(g.B + k + n * g.ldb)
                               : make_uint4(0, 0, 0, 0);
  };
  auto store = [&](int buf, const uint4 (&ra)[4], const uint4& rb) {
    store_slice(lds[buf], ra, tid);
    const int row = tid >> 3, part = tid & 7;
    *reinterpret_cast<uint4*>(lds[buf] + kGBM * kLK + row * kLK + part * 8) = rb;
  };
  if (g.K > 0) {
    uint4 ra[4], rb;
    load(ra, rb, 0);
    store(0, ra, rb);
    __syncthreads();
    int buf = 0;
    for (int64_t k0 = 0; k0 < g.K; k0 += kBK) {
      const bool more = k0 + kBK < g.K;
      if (more) load(ra, rb, k0 + kBK);
      const uint16_t* la = lds[buf];
      const uint16_t* lb = lds[buf] + kGBM * kLK;
#pragma unroll
      for (int ks = 0; ks < kBK; ks += 32) {
        bf16x8 af[2], bfr[2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
          af[i] = *reinterpret_cast<const bf16x8*>(
              la + (wave * 32 + i * 16 + (lane & 15)) * kLK + ks + 8 * (lane >> 4));
#pragma unroll
        for (int j = 0; j < 2; ++j)
          bfr[j] = *reinterpret_cast<const bf16x8*>(
              lb + (j * 16 + (lane & 15)) * kLK + ks + 8 * (lane >> 4));
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
      }
      if (more) store(buf ^ 1, ra, rb);
      __syncthreads();
      buf ^= 1;
    }
  }
  // lane l, register r holds D(row 4 (l / 16) + r, column l % 16) of a sub-tile
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int64_t n = n0 + j * 16 + (lane & 15);
      if (n >= g.N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = m0 + wave * 32 + i * 16 + 4 * (lane >> 4) + r;
        if (m >= g.M) continue;
        if (g.out64) g.out64[m + n * g.ld64] = (double)acc[i][j][r];
        else g.P[m + n * g.ldp] = acc[i][j][r];
      }
    }
}

// One workgroup per (problem, column): the column's max, its power of two,
// the scaled bfloat16 column with rows [M, ld16) zero.
__global__ __launch_bounds__(256) void round_columns_batched_kernel(
    const RoundDesc* __restrict__ descs) {
  __shared__ float red[4];
  const RoundDesc d = descs[blockIdx.y];
  const int64_t n = blockIdx.x;
  if (n >= d.N) return;
  const float* c = d.P + n * d.ldp;
  float m = 0.f;
  for (int64_t i = threadIdx.x; i < d.M; i += 256) m = fmaxf(m, fabsf(c[i]));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  const float s = (float)pow2_scale((double)fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3])));
  for (int64_t i = threadIdx.x; i < d.ld16; i += 256)
    d.out16[i + n * d.ld16] = (i < d.M) ? bf16_from_f32(c[i] * s) : (uint16_t)0;
}

}  // namespace

int maxabs(hipStream_t st, int64_t rows, int64_t cols, const double* X, int64_t ld,
           unsigned long long* word) {
  RRF_TRY(fill_u32(st, reinterpret_cast<unsigned*>(word), 2, 0u));
  if (rows <= 0 || cols <= 0) return RRF_OK;
  dim3 grid((unsigned)ceil_div(rows, 512), (unsigned)std::min<int64_t>(cols, 64));
  int tok = trace_begin(st, kTrElementwise, 0.0, 8.0 * rows * cols);
  hipLaunchKernelGGL(maxabs_kernel, grid, dim3(256), 0, st, rows, cols, X, ld, word);
  trace_end(st, tok);
  RRF_CHECK_HIP(hipGetLastError());
  return RRF_OK;
}

int frob_norm(hipStream_t st, int64_t rows, int64_t cols, const double* X, int64_t ld,
              const unsigned long long* word, double* parts, int max_parts, double* out) {
  if (rows <= 0 || cols <= 0) return fill_matrix(st, 1, 1, 0.0, out, 1);
  const int64_t gx = ceil_div(rows, 256);
  if (gx > max_parts) return set_error(RRF_E_NOTSUP, "frob_norm: too many rows");
  const int64_t gy = std::max<int64_t>(1, std::min<int64_t>(cols, max_parts / gx));
  int tok = trace_begin(st, kTrElementwise, 0.0, 8.0 * rows * cols);
  hipLaunchKernelGGL(sumsq_kernel, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, st, rows, cols,
                     X, ld, word, parts);
  hipLaunchKernelGGL(sumsq_finish_kernel, dim3(1), dim3(256), 0, st, (const double*)parts,
                     (int)(gx * gy), word, out);
  trace_end(st, tok);
  RRF_CHECK_HIP(hipGetLastError());
  return RRF_OK;
}

int scale_pow2(hipStream_t st, int64_t rows, int64_t cols, double* X, int64_t ld,
               const unsigned long long* word, bool inverse, int guard_exp) {
  if (rows <= 0 || cols <= 0) return RRF_OK;
  const dim3 grid((unsigned)ceil_div(rows, 256), (unsigned)std::min<int64_t>(cols, 65535));
  int tok = trace_begin(st, kTrElementwise, 0.0, 16.0 * rows * cols);
  hipLaunchKernelGGL(scale_pow2_kernel, grid, dim3(256), 0, st, rows, cols, X, ld, word, inverse,
                     guard_exp);
  trace_end(st, tok);
  RRF_CHECK_HIP(hipGetLastError());
  return RRF_OK;
}

int to_bf16(hipStream_t st, int64_t rows, int64_t cols, const double* X, int64_t ld,
            const unsigned long long* word, uint16_t* out, int64_t ldo, uint16_t* outT,
            int64_t ldot) {
  if (rows <= 0 || cols <= 0) return RRF_OK;
  const int64_t R = std::max(rows, ldo), C = outT ? std::max(cols, ldot) : cols;
  dim3 grid((unsigned)ceil_div(R, 64), (unsigned)ceil_div(C, 64));
  int tok = trace_begin(st, kTrElementwise, 0.0, (8.0 + (outT ? 4.0 : 2.0)) * rows * cols);
  hipLaunchKernelGGL(to_bf16_kernel, grid, dim3(256), 0, st, rows, cols, X, ld, word, out, ldo,
                     outT, ldot);
  trace_end(st, tok);
  RRF_CHECK_HIP(hipGetLastError());
  return RRF_OK;
}

size_t gemm_bf16_work_bytes(int64_t M, int64_t N) {
  return (size_t)16 * M * N * sizeof(float) + (size_t)M * N * sizeof(float) + 256;
}

namespace {
// Split of K as for the FP64 GEMM: fill the 512 resident slots, at least 256
// of K per split, at most 16 splits.
int bf16_splits(int64_t M, int64_t N, int64_t K) {
  const int64_t tiles = ceil_div(M, kBM) * ceil_div(N, kBN);
  int splits = 1;
  if (tiles < 512 && K >= 512) {
    double best = 1.0;
    for (int64_t s = 2; s <= 16 && K / s >= 256; ++s) {
      const double t = (double)ceil_div(tiles * s, 512) / (double)s;
      if (t < best - 1e-12) {
        best = t;
        splits = (int)s;
      }
    }
  }
  const int64_t kchunk = round_up(ceil_div(std::max<int64_t>(K, 1), splits), kBK);
  return (int)std::max<int64_t>(1, ceil_div(K, kchunk));
}
}  // namespace

size_t gemm_bf16_work_bytes_k(int64_t M, int64_t N, int64_t K) {
  return (size_t)bf16_splits(M, N, K) * M * N * sizeof(float) +
         (M > kColLds ? (size_t)M * N * sizeof(float) : 0) + 256;
}

int gemm_bf16_tn(hipStream_t st, int64_t M, int64_t N, int64_t K, const uint16_t* A,
                 int64_t lda, const uint16_t* B, int64_t ldb, uint16_t* out16, int64_t ld16,
                 double* out64, int64_t ld64, void* work, size_t work_bytes) {
  if (M <= 0 || N <= 0) return RRF_OK;
  if ((lda & 7) || (ldb & 7) || (reinterpret_cast<uintptr_t>(A) & 15) ||
      (reinterpret_cast<uintptr_t>(B) & 15))
    return set_error(RRF_E_INTERNAL, "bf16 gemm: operands must be 16-byte aligned");
  if (work_bytes < gemm_bf16_work_bytes_k(M, N, K) || work == nullptr)
    return set_error(RRF_E_NOMEM, "bf16 gemm: workspace too small");
  const int64_t tiles_m = ceil_div(M, kBM), tiles = tiles_m * ceil_div(N, kBN);
  int splits = bf16_splits(M, N, K);
  GemmBf16Args g{};
  g.M = M; g.N = N; g.K = K;
  g.A = A; g.lda = lda; g.B = B; g.ldb = ldb;
  g.kchunk = round_up(ceil_div(std::max<int64_t>(K, 1), splits), kBK);
  splits = (int)std::max<int64_t>(1, ceil_div(K, g.kchunk));
  g.tiles_m = (int)tiles_m;
  float* P = reinterpret_cast<float*>(work);
  float* col = P + (size_t)splits * M * N;
  g.P = P;
  int tok = trace_begin(st, kTrGemmBf16, 2.0 * M * N * K, 2.0 * ((double)M * K + (double)K * N) +
                                                             4.0 * splits * M * N);
  hipLaunchKernelGGL(gemm_bf16_tn_kernel, dim3((unsigned)tiles, 1, (unsigned)splits),
                     dim3(kThreads), 0, st, g);
  trace_end(st, tok);
  RRF_CHECK_HIP(hipGetLastError());
  RRF_TRY(allow_dynamic_lds((const void*)reduce_columns_kernel, kColLds * sizeof(float)));
  const size_t lds = M <= kColLds ? (size_t)M * sizeof(float) : 0;
  tok = trace_begin(st, kTrSplitReduce, (double)splits * M * N,
                    4.0 * splits * M * N + (out64 ? 8.0 : 2.0) * M * N);
  hipLaunchKernelGGL(reduce_columns_kernel, dim3((unsigned)N), dim3(kColThreads), lds, st, M, N,
                     splits, P, out16, ld16, out64, ld64, col);
  trace_end(st, tok);
  RRF_CHECK_HIP(hipGetLastError());
  return RRF_OK;
}

int maxabs_batched(hipStream_t st, const MaxDesc* d, int count, int64_t max_rows) {
  if (count <= 0 || max_rows <= 0) return RRF_OK;
  int tok = trace_begin(st, kTrElementwise, 0.0, 0.0);
  for (int c0 = 0; c0 < count; c0 += 65535) {
    const dim3 grid((unsigned)ceil_div(max_rows, 256), (unsigned)std::min(count - c0, 65535));
    hipLaunchKernelGGL(maxabs_batched_kernel, grid, dim3(256), 0, st, d + c0);
  }
  trace_end(st, tok);
  RRF_CHECK_HIP(hipGetLastError());
  return RRF_OK;
}

int to_bf16_batched(hipStream_t st, const Bf16Desc* d, int count, int64_t max_tiles) {
  if (count <= 0 || max_tiles <= 0) return RRF_OK;
  int tok = trace_begin(st, kTrElementwise, 0.0, 0.0);
  for (int c0 = 0; c0 < count; c0 += 65535) {
    const dim3 grid((unsigned)max_tiles, (unsigned)std::min(count - c0, 65535));
    hipLaunchKernelGGL(to_bf16_batched_kernel, grid, dim3(256), 0, st, d + c0);
  }
  trace_end(st, tok);
  RRF_CHECK_HIP(hipGetLastError());
  return RRF_OK;
}

int gemm_bf16_grouped(hipStream_t st, const Bf16GemmDesc* d, const int* d_prefix, int count,
                      int64_t total_tiles, double flops) {
  if (count <= 0 || total_tiles <= 0) return RRF_OK;
  if (total_tiles > INT32_MAX) return set_error(RRF_E_NOTSUP, "bf16 grouped gemm: too many tiles");
  int tok = trace_begin(st, kTrGemmBf16, flops, 0.0);
  hipLaunchKernelGGL(gemm_bf16_grouped_kernel, dim3((unsigned)total_tiles), dim3(kThreads), 0, st,
                     d, d_prefix, count);
  trace_end(st, tok);
  RRF_CHECK_HIP(hipGetLastError());
  return RRF_OK;
}

int round_columns_batched(hipStream_t st, const RoundDesc* d, int count, int64_t max_cols) {
  if (count <= 0 || max_cols <= 0) return RRF_OK;
  int tok = trace_begin(st, kTrSplitReduce, 0.0, 0.0);
  for (int c0 = 0; c0 < count; c0 += 65535) {
    const dim3 grid((unsigned)max_cols, (unsigned)std::min(count - c0, 65535));
    hipLaunchKernelGGL(round_columns_batched_kernel, grid, dim3(256), 0, st, d + c0);
  }
  trace_end(st, tok);
  RRF_CHECK_HIP(hipGetLastError());
  return RRF_OK;
}

}  // namespace rrf
