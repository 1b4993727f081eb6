// Householder QR of a panel through CholeskyQR (Sec. 2.3's panel
// factorization, computed another way).
//
// The column-exchange panel kernel pays one grid-wide exchange per column, a
// latency that no row count amortises. Here the panel's orthonormal factor
// comes from CholeskyQR2: two passes of Gram matrix, Cholesky factor and
// multiplication by the factor's inverse (the second pass restores the
// orthogonality the first loses to rounding), and the Householder
// reflectors of that factor are recovered by an LU factorization without
// pivoting of its top k x k block minus a sign matrix:
//
//   Q(0:k, :) - S = L U,  S = diag(s_i),  s_i = -sign of the i-th pivot,
//   W = [L; Q(k:M, :) U^-1],  Tf = -U S L^-T,  R = S R2 R1,
//
// so that I - W Tf W^T has Q's columns (times S) as its first k columns and
// the reflectors follow the dlarfg sign rule. The tall products run on the
// FP64 matrix cores (dgemm_shaped); the k x k steps run in one 512-thread
// workgroup each, every thread holding an 8 x 4 tile of the
// (identity-padded) 128 x 128 matrix in registers, over 4 x 4 blocks with
// one or two barriers per block. When the first pass leaves the second
// pass's Gram matrix within 1e-11 of I, that pass takes first-order factors
// instead of factorizing.
//
// When a pass meets a Cholesky pivot at or below its threshold (the panel is
// ill conditioned or rank deficient, or holds a NaN or an infinity) a device
// flag is raised, the later small kernels return at once, and the
// column-exchange
// kernel, launched conditionally after them, factors the untouched panel; it
// returns at once when the flag is clear. The panel P is therefore never
// written before that launch: W must not overlap P, and the in-place clear
// of `zero` is done after the flag is known.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <type_traits>

#include "common.hpp"
#include "context.hpp"
#include "kernels.hpp"
#include "trace.hpp"

namespace rrf {

namespace {

constexpr int kCqThreads = 512;
constexpr int kTC = 4;       // columns of a thread's tile (8 rows x 4 columns)
constexpr int kCqMax = 128;  // columns
constexpr int kLdm = kCqMax + 1;
constexpr size_t kCqLds = ((size_t)kCqMax * kLdm + 16 * kCqMax) * sizeof(double);
constexpr int kGramMaxSplits = 64;
constexpr int64_t kCholMinRows = 1024;
constexpr int kCholMinCols = 16;
// Smallest pivot accepted in the second pass. Its Gram matrix is that of
// the first pass's output, orthonormal to about u cond(P)^2; a pivot below
// 1/4 means that the first pass lost so much orthogonality (cond(P) beyond
// about 1e7) that the second no longer restores it to rounding, and the
// panel goes to the column kernel instead.
constexpr double kPass2Tol = 0.25;
// Largest |G2 - I| entry for which the second pass takes the first-order
// factors instead of the Cholesky factorization (see cholinv_kernel).
constexpr double kPass2Near = 1e-11;

struct CholArgs {
  int k;
  const double* G;    // k x k, ld k
  double tol;         // smallest accepted pivot
  double near;        // > 0: first-order factors when every |G - I| entry is at most this
  double* R;          // k x k upper triangular factor, ld k
  double* Ri;         // its inverse, ld k
  int* flag;
};

struct ReconArgs {
  int k;
  const double* Q;    // orthonormal factor, top k x k block used, ld ldq
  int64_t ldq;
  const double* Rc;   // Cholesky R of the panel (k x k, ld k; null when R is not wanted)
  double* W;          // top k x k block of the reflectors, ld ldw
  int64_t ldw;
  double* Ui;         // U^-1, k x k, ld k
  double* Tf;
  int64_t ldt;
  double* tau;
  double* R;
  int64_t ldr;
  const int* flag;
};

__device__ inline int flag_value(const int* f) {
  return __hip_atomic_load(const_cast<int*>(f), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The identity-padded 128 x 128 matrix in 8 x 4 tiles, one per thread:
// wave w holds rows 64 (w >> 2) .. +63 and columns 32 (w & 3) .. +31, so
// that whole waves skip the steps whose trailing region misses them.
struct TileIx {
  int ti, tj, r0, c0;  // tile row and column; first row and column
  int R0, R1, C0, C1;  // rows and columns of the wave
  __device__ explicit TileIx(int t) {
    const int w = t >> 6, lane = t & 63;
    ti = 8 * (w >> 2) + (lane >> 3);
    tj = 8 * (w & 3) + (lane & 7);
    r0 = 8 * ti;
    c0 = kTC * tj;
    R0 = 64 * (w >> 2);
    R1 = R0 + 63;
    C0 = 32 * (w & 3);
    C1 = C0 + 31;
  }
};

template <int J>
using Int = std::integral_constant<int, J>;

// f(Int<0>), f(Int<1>): the two 4-row blocks of a thread's 8-row tile, so
// that the rows a step touches are compile-time indices of the register
// tiles.
template <class F>
__device__ __forceinline__ void each_half_up(F&& f) {
  f(Int<0>{});
  f(Int<1>{});
}
template <class F>
__device__ __forceinline__ void each_half_down(F&& f) {
  f(Int<1>{});
  f(Int<0>{});
}

// The algorithms below run over 4 x 4 blocks: block b covers rows and
// columns 4b .. 4b+3, which are rows 4*JB .. 4*JB+3 of tile row b / 2
// (JB = b & 1) and the whole of tile column b. In the Cholesky and LU
// factorizations wave 0 factors the diagonal block and publishes the
// block's rows (and columns) of the factors in LDS, then the waves that
// meet the trailing region update their tiles (two barriers per block); in
// the triangular inverse and solve the threads holding the block's rows
// transform them with the diagonal block and publish them, then the waves
// concerned update (one barrier per block).

// X = U^-1 for U upper triangular in LDS (row stride kLdm): X starts as I;
// from the last block up, X(B, :) <- U_BB^-1 X(B, :) by the rows of block B,
// then X(r, :) -= U(r, B) X(B, :) for the rows r above B.
__device__ void upper_inverse(double (&X)[8][kTC], const double* Ml, double* vb, int k,
                              const TileIx& ix) {
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int c = 0; c < kTC; ++c) X[i][c] = (ix.r0 + i == ix.c0 + c) ? 1.0 : 0.0;
  for (int jt = (k - 1) >> 3; jt >= 0; --jt) {
    each_half_down([&](auto jc) {
      constexpr int JB = decltype(jc)::value;
      constexpr int RB = 4 * JB;
      const int j0 = 8 * jt + RB;
      if (j0 >= k) return;
      double* rb = vb + JB * 4 * kCqMax;
      if (ix.ti == jt) {
        // the block's upper triangle, inverted by back substitution
        double u[4][4];
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
          for (int q = p; q < 4; ++q) u[p][q] = Ml[(j0 + p) * kLdm + j0 + q];
        double d[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) d[p] = 1.0 / u[p][p];
#pragma unroll
        for (int c = 0; c < kTC; ++c) {
          double x[4];
#pragma unroll
          for (int p = 3; p >= 0; --p) {
            double v = X[RB + p][c];
#pragma unroll
            for (int q = p + 1; q < 4; ++q) v = fma(-u[p][q], x[q], v);
            x[p] = v * d[p];
          }
#pragma unroll
          for (int p = 0; p < 4; ++p) {
            X[RB + p][c] = x[p];
            rb[p * kCqMax + ix.c0 + c] = x[p];
          }
        }
      }
      __syncthreads();
      // rows above the block (factor 0 for the others) in the columns from
      // the block on (X is upper triangular); other waves have nothing to do
      if (ix.R0 >= j0 || ix.C1 < j0) return;
      double y[4][kTC];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int c = 0; c < kTC; ++c) y[q][c] = rb[q * kCqMax + ix.c0 + c];
      double uf[8][4];
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) uf[i][q] = Ml[(ix.r0 + i) * kLdm + j0 + q];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const bool above = ix.ti < jt || (ix.ti == jt && i < RB);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double f = above ? uf[i][q] : 0.0;
#pragma unroll
          for (int c = 0; c < kTC; ++c) X[i][c] = fma(-f, y[q][c], X[i][c]);
        }
      }
    });
  }
}

// Cholesky factor R (R^T R = G) and R^-1 in one workgroup.
__global__ __launch_bounds__(kCqThreads) void cholinv_kernel(CholArgs a) {
  extern __shared__ double lds[];
  double* Ml = lds;
  double* vb = lds + kCqMax * kLdm;
  if (flag_value(a.flag) != 0) return;
  const int t = threadIdx.x;
  const TileIx ix(t);
  const int k = a.k;
  if (a.near > 0.0) {
    // G = I + E with every |E_ij| <= near (the second pass of a well
    // conditioned panel): R = I + F, F the upper triangle of E with its
    // diagonal halved, satisfies R^T R = G + F^T F, and I - F is R^-1 up to
    // F^2; with near = 1e-11 and k <= 128 both residuals are below 2e-18,
    // under the rounding of the exact factorization. (NaN compares false
    // and takes the factorization below, which reports it.)
    bool near = true;
    for (int e = t; e < k * k; e += kCqThreads) {
      const int r = e % k, cc = e / k;
      near = near && fabs(a.G[e] - (r == cc ? 1.0 : 0.0)) <= a.near;
    }
    if (__syncthreads_and(near)) {
      for (int e = t; e < k * k; e += kCqThreads) {
        const int r = e % k, cc = e / k;
        const double g = a.G[e];
        const double f = cc > r ? g : (cc == r ? 0.5 * (g - 1.0) : 0.0);
        a.R[e] = (r == cc ? 1.0 : 0.0) + f;
        a.Ri[e] = (r == cc ? 1.0 : 0.0) - f;
      }
      return;
    }
  }

  double A[8][kTC];
  bool finite = true;
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int c = 0; c < kTC; ++c) {
      const int r = ix.r0 + i, cc = ix.c0 + c;
      double v = (r == cc) ? 1.0 : 0.0;
      if (r < k && cc < k) {
        v = a.G[r + (int64_t)cc * k];
        finite = finite && isfinite(v);
      }
      A[i][c] = v;
    }
  if (__syncthreads_or(!finite)) {
    if (t == 0) *a.flag = 1;
    return;
  }
  // right-looking blocked Cholesky of the upper triangle, two barriers per
  // 4 x 4 block. The block's rows (published in LDS by the step before) go
  // to wave 0, which factors the diagonal block and forms the block's rows
  // of R in every column from the block on; then every wave whose tiles meet
  // the trailing upper triangle applies the rank-4 update (A is symmetric,
  // so R(B, r) is also the factor of row r), the owners of the block's rows
  // keep R, and the owners of the next block's rows publish them.
  double* rb = vb;                 // the block's rows (4 x 128)
  double* rr = vb + 4 * kCqMax;    // the block's rows of R (4 x 128)
  __shared__ int bad;
  if (t == 0) bad = 0;
  if (ix.ti == 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < kTC; ++c) rb[q * kCqMax + ix.c0 + c] = A[q][c];
  }
  __syncthreads();
  bool failed = false;
  for (int jt = 0; jt <= (k - 1) >> 3 && !failed; ++jt) {
    each_half_up([&](auto jc) {
      constexpr int JB = decltype(jc)::value;
      constexpr int RB = 4 * JB;           // the block's rows in tile row jt
      constexpr int RN = 4 - RB;           // the next block's rows in its tile row
      const int b = 2 * jt + JB;
      const int j0 = 4 * b;
      if (failed || j0 >= k) return;
      if (t < 64) {
        double r[4][4], dinv[4], blk[4][4];
        bool ok = true;
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
          for (int q = p; q < 4; ++q) blk[p][q] = rb[p * kCqMax + j0 + q];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
#pragma unroll
          for (int q = p; q < 4; ++q) {
            double v = blk[p][q];
#pragma unroll
            for (int m = 0; m < p; ++m) v = fma(-r[m][p], r[m][q], v);
            if (q == p) {
              ok = ok && (v > a.tol);
              const double rs = 1.0 / sqrt(v);
              r[p][p] = v * rs;
              dinv[p] = rs;
            } else {
              r[p][q] = v * dinv[p];
            }
          }
        }
        if (!ok && t == 0) bad = 1;
        double col[2][4];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int q = 0; q < 4; ++q) col[h][q] = rb[q * kCqMax + t + 64 * h];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int cc = t + 64 * h;
          if (cc > j0 + 3) {
            double x[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              double v = col[h][q];
#pragma unroll
              for (int m = 0; m < q; ++m) v = fma(-r[m][q], x[m], v);
              x[q] = v * dinv[q];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) rr[q * kCqMax + cc] = x[q];
          }
        }
        if (t == 0) {  // the diagonal block of R
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int m = 0; m < 4; ++m) rr[q * kCqMax + j0 + m] = (m >= q) ? r[q][m] : 0.0;
        }
      }
      __syncthreads();
      if (bad) {
        failed = true;
        return;
      }
      const bool update = ix.R1 > j0 + 3 && ix.C1 > j0 + 3 && ix.R0 <= ix.C1;
      const bool keep = ix.R0 <= j0 && j0 <= ix.R1 && ix.C1 >= j0;
      if (update || keep) {
        double z[4][kTC];
        const bool cols_right = ix.tj > b;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int c = 0; c < kTC; ++c) {
            const double v = rr[q * kCqMax + ix.c0 + c];
            z[q][c] = cols_right ? v : 0.0;
          }
        if (update) {
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            const bool below = ix.ti > jt || (ix.ti == jt && i >= RB + 4);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const double v = rr[q * kCqMax + ix.r0 + i];
              const double wq = below ? v : 0.0;
#pragma unroll
              for (int c = 0; c < kTC; ++c) A[i][c] = fma(-wq, z[q][c], A[i][c]);
            }
          }
        }
        if (ix.ti == jt && ix.tj >= b) {
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int c = 0; c < kTC; ++c) A[RB + q][c] = rr[q * kCqMax + ix.c0 + c];
        }
        // the next block's rows
        if (ix.ti == jt + (JB == 1 ? 1 : 0)) {
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int c = 0; c < kTC; ++c) rb[q * kCqMax + ix.c0 + c] = A[RN + q][c];
        }
      }
      __syncthreads();
    });
  }
  if (failed) {
    if (t == 0) *a.flag = 1;
    return;
  }

  // R to LDS (upper, zero below) and to global
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int c = 0; c < kTC; ++c) {
      const int r = ix.r0 + i, cc = ix.c0 + c;
      const double v = (cc >= r) ? A[i][c] : 0.0;
      Ml[r * kLdm + cc] = v;
      if (r < k && cc < k) a.R[r + (int64_t)cc * k] = v;
    }
  __syncthreads();
  double X[8][kTC];
  upper_inverse(X, Ml, vb, k, ix);
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int c = 0; c < kTC; ++c) {
      const int r = ix.r0 + i, cc = ix.c0 + c;
      if (r < k && cc < k) a.Ri[r + (int64_t)cc * k] = (cc >= r) ? X[i][c] : 0.0;
    }
}

// Reflectors from the orthonormal factor: LU of Q1 - S (each sign chosen
// when the elimination reaches its pivot, as dlarfg chooses it), U^-1, Tf,
// R.
__global__ __launch_bounds__(kCqThreads) void recon_kernel(ReconArgs a) {
  extern __shared__ double lds[];
  double* Ml = lds;
  double* vb = lds + kCqMax * kLdm;  // 16 x 128 exchange rows after the matrix
  double* cb = vb + 8 * kCqMax;      // its second half
  __shared__ double sg[kCqMax];
  if (flag_value(a.flag) != 0) return;
  const int t = threadIdx.x;
  const TileIx ix(t);
  const int k = a.k;
  if (t < kCqMax) sg[t] = 0.0;

  double A[8][kTC];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int c = 0; c < kTC; ++c) {
      const int r = ix.r0 + i, cc = ix.c0 + c;
      A[i][c] = (r < k && cc < k) ? a.Q[r + cc * a.ldq] : (r == cc ? 1.0 : 0.0);
    }

  // blocked LU without pivoting of Q1 - S, two barriers per 4 x 4 block:
  // the sign s_j = -sign(a_jj) of the current diagonal entry is subtracted
  // when step j is reached, so every pivot has magnitude >= 1. The block's
  // rows and columns (published in LDS by the step before) go to wave 0,
  // which factors the diagonal block and forms the block's rows of U in
  // every column right of it and the multipliers of every row below it;
  // then the waves whose tiles meet the trailing block update, the owners of
  // the block's columns and rows keep L and U, and the owners of the next
  // block's rows and columns publish them.
  double* rbk = vb;                 // the block's rows (4 x 128)
  double* cbk = vb + 4 * kCqMax;    // the block's columns (4 x 128)
  double* ur = vb + 8 * kCqMax;     // U(B, c), c right of the block
  double* lc = vb + 12 * kCqMax;    // L(r, B), r below the block
  __shared__ double dblk[16];
  if (ix.ti == 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < kTC; ++c) rbk[q * kCqMax + ix.c0 + c] = A[q][c];
  }
  if (ix.tj == 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int i = 0; i < 8; ++i) cbk[q * kCqMax + ix.r0 + i] = A[i][q];
  }
  __syncthreads();
  for (int jt = 0; jt <= (k - 1) >> 3; ++jt) {
    each_half_up([&](auto jc) {
      constexpr int JB = decltype(jc)::value;
      constexpr int RB = 4 * JB;
      constexpr int RN = 4 - RB;
      const int b = 2 * jt + JB;
      const int j0 = 4 * b;
      if (j0 >= k) return;
      if (t < 64) {
        double d[4][4], sgn[4], pinv[4];
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
          for (int q = 0; q < 4; ++q) d[p][q] = rbk[p * kCqMax + j0 + q];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          sgn[p] = d[p][p] >= 0.0 ? -1.0 : 1.0;
          d[p][p] -= sgn[p];
          pinv[p] = 1.0 / d[p][p];
#pragma unroll
          for (int m = p + 1; m < 4; ++m) {
            d[m][p] *= pinv[p];
#pragma unroll
            for (int q = p + 1; q < 4; ++q) d[m][q] = fma(-d[m][p], d[p][q], d[m][q]);
          }
        }
        if (t == 0) {
#pragma unroll
          for (int p = 0; p < 4; ++p) {
            sg[j0 + p] = sgn[p];
#pragma unroll
            for (int q = 0; q < 4; ++q) dblk[p * 4 + q] = d[p][q];
          }
        }
        double rowv[2][4], colv[2][4];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            rowv[h][q] = rbk[q * kCqMax + t + 64 * h];
            colv[h][q] = cbk[q * kCqMax + t + 64 * h];
          }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int cc = t + 64 * h;
          if (cc > j0 + 3) {
            // U(B, cc) = L_BB^-1 A(B, cc)
            double x[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              double v = rowv[h][q];
#pragma unroll
              for (int m = 0; m < q; ++m) v = fma(-d[q][m], x[m], v);
              x[q] = v;
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) ur[q * kCqMax + cc] = x[q];
            // L(cc, B) = A(cc, B) U_BB^-1 for the row cc below the block
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              double v = colv[h][q];
#pragma unroll
              for (int m = 0; m < q; ++m) v = fma(-x[m], d[m][q], v);
              x[q] = v * pinv[q];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) lc[q * kCqMax + cc] = x[q];
          }
        }
      }
      __syncthreads();
      const bool update = ix.R1 > j0 + 3 && ix.C1 > j0 + 3;
      const bool cols_own = ix.C0 <= j0 && j0 <= ix.C1 && ix.R1 >= j0;
      const bool rows_own = ix.R0 <= j0 && j0 <= ix.R1 && ix.C1 > j0 + 3;
      if (update || cols_own || rows_own) {
        const bool cols_right = ix.tj > b;
        double u[4][kTC];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int c = 0; c < kTC; ++c) {
            const double v = ur[q * kCqMax + ix.c0 + c];
            u[q][c] = cols_right ? v : 0.0;
          }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const bool below = ix.ti > jt || (ix.ti == jt && i >= RB + 4);
          const bool in = ix.ti == jt && i >= RB && i < RB + 4;
          double l[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const double v = lc[q * kCqMax + ix.r0 + i];
            l[q] = below ? v : 0.0;
          }
          if (update) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
              for (int c = 0; c < kTC; ++c) A[i][c] = fma(-l[q], u[q][c], A[i][c]);
          }
          if (ix.tj == b) {
            // the block's columns: multipliers below it, its LU in it
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const double blk = dblk[((i - RB) & 3) * 4 + q];
              A[i][q] = below ? l[q] : (in ? blk : A[i][q]);
            }
          }
        }
        if (ix.ti == jt && cols_right) {
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int c = 0; c < kTC; ++c) A[RB + q][c] = u[q][c];
        }
        // the next block's rows and columns
        if (ix.ti == jt + (JB == 1 ? 1 : 0)) {
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int c = 0; c < kTC; ++c) rbk[q * kCqMax + ix.c0 + c] = A[RN + q][c];
        }
        if (ix.tj == b + 1) {
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int i = 0; i < 8; ++i) cbk[q * kCqMax + ix.r0 + i] = A[i][q];
        }
      }
      __syncthreads();
    });
  }

  // LU to LDS; L (unit lower) is the top block of W
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int c = 0; c < kTC; ++c) {
      const int r = ix.r0 + i, cc = ix.c0 + c;
      Ml[r * kLdm + cc] = A[i][c];
      if (r < k && cc < k) a.W[r + cc * a.ldw] = r > cc ? A[i][c] : (r == cc ? 1.0 : 0.0);
    }
  __syncthreads();

  double X[8][kTC];
  upper_inverse(X, Ml, vb, k, ix);
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int c = 0; c < kTC; ++c) {
      const int r = ix.r0 + i, cc = ix.c0 + c;
      if (r < k && cc < k) a.Ui[r + (int64_t)cc * k] = (cc >= r) ? X[i][c] : 0.0;
    }

  // Y = Tf^T from L Y = -S U^T by blocked forward substitution (Y lower
  // triangular): Y(B, :) <- L_BB^-1 Y(B, :), then Y(r, :) -= L(r, B) Y(B, :)
  // for the rows r below B
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int c = 0; c < kTC; ++c) {
      const int r = ix.r0 + i, m = ix.c0 + c;
      X[i][c] = (m <= r && r < k) ? -sg[r] * Ml[m * kLdm + r] : 0.0;
    }
  for (int jt = 0; jt <= (k - 1) >> 3; ++jt) {
    each_half_up([&](auto jc) {
      constexpr int JB = decltype(jc)::value;
      constexpr int RB = 4 * JB;
      const int j0 = 8 * jt + RB;
      if (j0 >= k) return;
      double* rb = cb + JB * 4 * kCqMax;  // free once the LU is done
      if (ix.ti == jt) {
        double lb[4][4];
#pragma unroll
        for (int p = 1; p < 4; ++p)
#pragma unroll
          for (int q = 0; q < p; ++q) lb[p][q] = Ml[(j0 + p) * kLdm + j0 + q];
#pragma unroll
        for (int c = 0; c < kTC; ++c) {
          double x[4];
#pragma unroll
          for (int p = 0; p < 4; ++p) {
            double v = X[RB + p][c];
#pragma unroll
            for (int q = 0; q < p; ++q) v = fma(-lb[p][q], x[q], v);
            x[p] = v;
          }
#pragma unroll
          for (int p = 0; p < 4; ++p) {
            X[RB + p][c] = x[p];
            rb[p * kCqMax + ix.c0 + c] = x[p];
          }
        }
      }
      __syncthreads();
      // rows below the block in the columns up to its end (Y is lower
      // triangular); other waves have nothing to do
      if (ix.R1 <= j0 + 3 || ix.C0 > j0 + 3) return;
      double y[4][kTC];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int c = 0; c < kTC; ++c) y[q][c] = rb[q * kCqMax + ix.c0 + c];
      double lf[8][4];
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) lf[i][q] = Ml[(ix.r0 + i) * kLdm + j0 + q];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const bool below = ix.ti > jt || (ix.ti == jt && i >= RB + 4);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double f = below ? lf[i][q] : 0.0;
#pragma unroll
          for (int c = 0; c < kTC; ++c) X[i][c] = fma(-f, y[q][c], X[i][c]);
        }
      }
    });
  }
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int c = 0; c < kTC; ++c) {
      const int r = ix.r0 + i, m = ix.c0 + c;
      if (r < k && m < k) {
        a.Tf[m + r * a.ldt] = (m <= r) ? X[i][c] : 0.0;
        if (m == r) a.tau[r] = X[i][c];
      }
    }
  if (a.R != nullptr) {
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
      for (int c = 0; c < kTC; ++c) {
        const int r = ix.r0 + i, cc = ix.c0 + c;
        if (r < k && cc < k)
          a.R[r + cc * a.ldr] = (cc >= r) ? sg[r] * a.Rc[r + (int64_t)cc * k] : 0.0;
      }
  }
}

// Z (rows x cols) = 0 unless the flag is raised (the fallback then clears it).
__global__ __launch_bounds__(256) void zero_if_ok_kernel(int64_t rows, int64_t cols, double* Z,
                                                         int64_t ldz, const int* flag) {
  if (flag_value(flag) != 0) return;
  const int64_t r = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
  if (r >= rows) return;
  for (int64_t c = (int64_t)blockIdx.y * 4 + (threadIdx.x >> 6); c < cols; c += 4 * gridDim.y)
    Z[r + c * ldz] = 0.0;
}

int set_attrs() {
  RRF_TRY(allow_dynamic_lds((const void*)cholinv_kernel, kCqLds));
  return allow_dynamic_lds((const void*)recon_kernel, kCqLds);
}

int gram_splits(int64_t M) { return (int)std::min<int64_t>(kGramMaxSplits, std::max<int64_t>(1, M / 256)); }

struct CqLayout {
  int* flag;
  char* rest;      // everything after the flag (the fallback's workspace starts here)
  double *S1, *G, *Ri, *Rc, *Ra, *Rb, *Ui, *part;
  size_t part_elems;
  size_t bytes;    // of the CholeskyQR buffers after the flag
};

CqLayout cq_layout(void* work, int64_t M, int k) {
  CqLayout L{};
  char* base = static_cast<char*>(work);
  L.flag = reinterpret_cast<int*>(base);
  char* p = base + 256;
  L.rest = p;
  auto take = [&](size_t elems) {
    double* q = reinterpret_cast<double*>(p);
    p += round_up((int64_t)(elems * sizeof(double)), 256);
    return q;
  };
  const size_t kk = (size_t)k * k;
  L.S1 = take((size_t)M * k);
  L.G = take(kk);
  L.Ri = take(kk);
  L.Rc = take(kk);
  L.Ra = take(kk);
  L.Rb = take(kk);
  L.Ui = take(kk);
  L.part_elems = (size_t)gram_splits(M) * kk;
  L.part = take(L.part_elems);
  L.bytes = (size_t)(p - L.rest);
  return L;
}

int launch_cholinv(hipStream_t st, int k, const double* G, double tol, double near, double* R,
                   double* Ri, int* flag) {
  CholArgs a{k, G, tol, near, R, Ri, flag};
  int tok = trace_begin(st, kTrCholInv, (2.0 / 3.0) * k * (double)k * k, 8.0 * 3.0 * k * k);
  hipLaunchKernelGGL(cholinv_kernel, dim3(1), dim3(kCqThreads), kCqLds, st, a);
  trace_end(st, tok);
  RRF_CHECK_HIP(hipGetLastError());
  return RRF_OK;
}

bool disjoint(const double* a, int64_t lda, const double* b, int64_t ldb, int64_t M, int k) {
  const uintptr_t a0 = (uintptr_t)a, a1 = (uintptr_t)(a + (k - 1) * lda + M);
  const uintptr_t b0 = (uintptr_t)b, b1 = (uintptr_t)(b + (k - 1) * ldb + M);
  return a1 <= b0 || b1 <= a0;
}

}  // namespace

bool cholqr_enabled() {
  const char* e = getenv("RRF_PANEL_COLUMN");
  return !(e && e[0] == '1');
}

bool cholqr_panel_ok(int64_t M, int k, const double* P, int64_t ldp, const double* W,
                     int64_t ldw) {
  return k >= kCholMinCols && k <= kCqMax && M >= kCholMinRows && M >= k &&
         disjoint(P, ldp, W, ldw, M, k);
}

size_t cholqr_work_bytes(int64_t M, int k) {
  if (k < kCholMinCols || k > kCqMax || M < kCholMinRows || M < k) return 0;
  return 256 + cq_layout(nullptr, M, k).bytes;
}

int cholqr_panel(hipStream_t st, int64_t M, int k, const double* P, int64_t ldp, double* W,
                 int64_t ldw, double* R, int64_t ldr, double* Tf, int64_t ldt, double* tau,
                 double* zero, int64_t ldz, void* work, size_t work_bytes, int* status) {
  if (!cholqr_panel_ok(M, k, P, ldp, W, ldw))
    return set_error(RRF_E_NOTSUP, "CholeskyQR panel: shape or aliasing not supported");
  const CqLayout L = cq_layout(work, M, k);
  if (work == nullptr || work_bytes < 256 + L.bytes)
    return set_error(RRF_E_NOMEM, "CholeskyQR panel: workspace too small");
  const size_t fb_bytes = work_bytes - 256;  // the fallback's workspace, after the flag
  RRF_TRY(set_attrs());
  RRF_TRY(fill_u32(st, reinterpret_cast<unsigned*>(L.flag), 1, 0u));
  const int gs = gram_splits(M);
  const bool want_r = (R != nullptr);

  // pass 1: P -> W
  RRF_TRY(dgemm_shaped(st, true, false, k, k, M, 1.0, P, ldp, P, ldp, 0.0, L.G, k, L.part,
                       L.part_elems, true, gs));
  RRF_TRY(launch_cholinv(st, k, L.G, 0.0, 0.0, L.Ra, L.Ri, L.flag));
  RRF_TRY(dgemm_shaped(st, false, false, M, k, k, 1.0, P, ldp, L.Ri, k, 0.0, W, ldw, nullptr,
                       0, true, 1));
  // pass 2: W -> S1, the orthonormal factor
  RRF_TRY(dgemm_shaped(st, true, false, k, k, M, 1.0, W, ldw, W, ldw, 0.0, L.G, k, L.part,
                       L.part_elems, true, gs));
  RRF_TRY(launch_cholinv(st, k, L.G, kPass2Tol, kPass2Near, L.Rc, L.Ri, L.flag));
  RRF_TRY(dgemm_shaped(st, false, false, M, k, k, 1.0, W, ldw, L.Ri, k, 0.0, L.S1, M, nullptr,
                       0, true, 1));
  if (want_r)
    RRF_TRY(dgemm_shaped(st, false, false, k, k, k, 1.0, L.Rc, k, L.Ra, k, 0.0, L.Rb, k,
                         nullptr, 0, true, 1));

  // reflectors: top block of W, U^-1, Tf, tau, R; then W(k:M, :) = Q(k:M, :) U^-1
  ReconArgs ra{};
  ra.k = k;
  ra.Q = L.S1;
  ra.ldq = M;
  ra.Rc = want_r ? L.Rb : nullptr;
  ra.W = W;
  ra.ldw = ldw;
  ra.Ui = L.Ui;
  ra.Tf = Tf;
  ra.ldt = ldt;
  ra.tau = tau;
  ra.R = R;
  ra.ldr = ldr;
  ra.flag = L.flag;
  int tok = trace_begin(st, kTrPanelRecon, 2.0 * k * (double)k * k, 8.0 * 4.0 * k * k);
  hipLaunchKernelGGL(recon_kernel, dim3(1), dim3(kCqThreads), kCqLds, st, ra);
  trace_end(st, tok);
  RRF_CHECK_HIP(hipGetLastError());
  if (M > k)
    RRF_TRY(dgemm_shaped(st, false, false, M - k, k, k, 1.0, L.S1 + k, M, L.Ui, k, 0.0, W + k,
                         ldw, nullptr, 0, true, 1));
  if (zero) {
    const unsigned gy = (unsigned)std::min<int64_t>(ceil_div(k, 4), 8);
    hipLaunchKernelGGL(zero_if_ok_kernel, dim3((unsigned)ceil_div(M, 64), gy), dim3(256), 0, st,
                       M, (int64_t)k, zero, ldz, L.flag);
    RRF_CHECK_HIP(hipGetLastError());
  }
  // the column-exchange kernel, which returns at once unless the flag is raised
  return panel_launch_if(st, M, k, P, ldp, W, ldw, R, ldr, Tf, ldt, tau, zero, ldz, L.rest,
                         fb_bytes, status, L.flag);
}

}  // namespace rrf
