// Left singular vectors and singular values of one small square matrix
// (k <= 256): the SVD of the R factor of randUTV_boosted's sample matrix
// (Sec. 4.2, method b), where only W_Y = Q_Y U_R is needed.
//
// One-sided (Hestenes) Jacobi on the columns of A = R: plane rotations make
// the columns of A V mutually orthogonal, and then A V = U diag(sigma), so
// U is the normalised columns and V never has to be formed. A 256 x 256
// matrix does not fit in one workgroup's LDS, so the columns are cut into
// blocks of 32 and the iteration is a block Jacobi:
//  * an outer sweep pairs the nb blocks round-robin (circle method, nb - 1
//    rounds of nb / 2 disjoint block pairs); each round is one launch with
//    one 1024-thread workgroup per block pair, which loads the pair's (up to)
//    64 columns into LDS, orthogonalises all of them among themselves with
//    up to kInner inner sweeps of the scalar one-sided Jacobi (the rotation
//    and threshold of the block SVD kernel; one half-wave per column pair, so
//    the 32 pairs of an inner round run together), and writes them back;
//  * every workgroup that rotates raises the flag of its outer sweep; the
//    host enqueues a fixed number of outer sweeps and every launch of a sweep
//    whose predecessor raised no flag returns at once, so there is no host
//    synchronisation and no unbounded loop;
//  * a finishing workgroup takes the column norms, orders them descending
//    (stable in column index), normalises the columns and completes the
//    columns of zero norm to an orthonormal basis.
// Column signs are left as the iteration leaves them (the Householder
// reflectors of W_Y(:, 1:b), and everything built from W_Y, do not depend on
// them).
#include <cfloat>

#include "common.hpp"
#include "context.hpp"
#include "kernels.hpp"
#include "trace.hpp"

namespace rrf {

namespace {

constexpr int kThreads = 1024;
constexpr int kWaves = kThreads / 64;
constexpr int kCB = 32;        // columns per block
constexpr int kMaxK = 256;
constexpr int kInner = 2;      // inner sweeps per block-pair meeting
constexpr int kMaxOuter = 40;  // outer sweeps enqueued

struct RoundArgs {
  int k;
  int nb;      // blocks, even (the last may be empty)
  int round;   // 0 .. nb - 2
  int sweep;
  double* A;   // k x k, ld k
  unsigned* rot;  // kMaxOuter flags
};

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the 32 lanes of a half-wave (xor offsets below 32 stay inside it).
__device__ inline double half_sum(double v) {
#pragma unroll
  for (int off = 16; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Columns [c0, c1) of block b.
__device__ inline void block_cols(int b, int k, int& c0, int& c1) {
  c0 = b * kCB;
  c1 = c0 + kCB < k ? c0 + kCB : k;
  if (c0 > k) c0 = k;
}

__global__ __launch_bounds__(kThreads) void block_round_kernel(RoundArgs a) {
  extern __shared__ double lds[];  // 2 kCB columns of k rows, ld k
  __shared__ int rotated, inner_rot;
  if (a.sweep > 0 && a.rot[a.sweep - 1] == 0) return;  // converged
  const int tid = threadIdx.x;
  const int hl = tid & 31, half = tid >> 5;  // one column pair per half-wave
  const int k = a.k;
  // circle method: position 0 holds block 0, positions 1..nb-1 rotate
  const int w = blockIdx.x;
  const int pa = w, pb = a.nb - 1 - w;
  auto at = [&](int pos) { return pos == 0 ? 0 : 1 + (pos - 1 + a.round) % (a.nb - 1); };
  int p0, p1, q0, q1;
  block_cols(at(pa), k, p0, p1);
  block_cols(at(pb), k, q0, q1);
  const int np = p1 - p0, nq = q1 - q0, nc = np + nq;
  if (nc < 2) return;
  // load: LDS column j < np is A(:, p0 + j), then the q block
  for (int idx = tid; idx < nc * k; idx += kThreads) {
    const int r = idx % k, j = idx / k;
    const int c = j < np ? p0 + j : q0 + (j - np);
    lds[idx] = a.A[r + (size_t)c * k];
  }
  if (tid == 0) rotated = 0;
  __syncthreads();
  const int ne = nc + (nc & 1);
  const double tol = DBL_EPSILON * fmax(sqrt((double)k), 8.0);
  for (int sweep = 0; sweep < kInner; ++sweep) {
    if (tid == 0) inner_rot = 0;
    __syncthreads();
    for (int round = 0; round < ne - 1; ++round) {
      for (int pi = half; pi < ne / 2; pi += kThreads / 32) {
        int p, q;
        if (pi == 0) {
          p = round;
          q = ne - 1;
        } else {
          p = (round + pi) % (ne - 1);
          q = (round - pi + ne - 1) % (ne - 1);
        }
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        if (q >= nc) continue;
        double* ap = lds + (size_t)p * k;
        double* aq = lds + (size_t)q * k;
        double app = 0.0, aqq = 0.0, apq = 0.0;
        for (int r = hl; r < k; r += 32) {
          const double x = ap[r], y = aq[r];
          app += x * x;
          aqq += y * y;
          apq += x * y;
        }
        app = half_sum(app);
        aqq = half_sum(aqq);
        apq = half_sum(apq);
        if (apq != 0.0 && fabs(apq) > tol * sqrt(app) * sqrt(aqq)) {
          const double zeta = (aqq - app) / (2.0 * apq);
          double t;
          if (fabs(zeta) > 1e150) t = 0.5 / zeta;
          else t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + t * t);
          const double s = c * t;
          for (int r = hl; r < k; r += 32) {
            const double x = ap[r], y = aq[r];
            ap[r] = c * x - s * y;
            aq[r] = s * x + c * y;
          }
          if (hl == 0) {
            rotated = 1;
            inner_rot = 1;
          }
        }
      }
      __syncthreads();
    }
    if (inner_rot == 0) break;  // this block pair is orthogonal
    __syncthreads();
  }
  for (int idx = tid; idx < nc * k; idx += kThreads) {
    const int r = idx % k, j = idx / k;
    const int c = j < np ? p0 + j : q0 + (j - np);
    a.A[r + (size_t)c * k] = lds[idx];
  }
  if (tid == 0 && rotated) atomicOr(a.rot + a.sweep, 1u);
}

// sigma_j = ||A(:, j)||, descending (stable), U = A(:, perm) / sigma, columns
// of zero norm completed by the coordinate vector least covered so far,
// orthogonalised twice. Flags non-convergence in status bit 2.
__global__ __launch_bounds__(kThreads) void left_finish_kernel(int k, const double* A, double* U,
                                                               double* d, const unsigned* rot,
                                                               int* status) {
  __shared__ double sig[kMaxK];
  __shared__ int perm[kMaxK];
  __shared__ double coef[kMaxK];
  __shared__ int pick;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0 && rot[kMaxOuter - 1] != 0) atomicOr(status, 2);
  for (int c = wave; c < k; c += kWaves) {
    double s = 0.0;
    for (int r = lane; r < k; r += 64) {
      const double x = A[r + (size_t)c * k];
      s += x * x;
    }
    s = wave_sum(s);
    if (lane == 0) sig[c] = sqrt(s);
  }
  __syncthreads();
  for (int c = tid; c < k; c += kThreads) {
    int rank = 0;
    const double sc = (sig[c] == sig[c]) ? sig[c] : -1.0;
    for (int i = 0; i < k; ++i) {
      const double si = (sig[i] == sig[i]) ? sig[i] : -1.0;
      rank += (si > sc) || (si == sc && i < c);
    }
    perm[rank] = c;
  }
  __syncthreads();
  const double tiny = DBL_MIN * (double)k;
  for (int idx = tid; idx < k * k; idx += kThreads) {
    const int r = idx % k, pos = idx / k;
    const int c = perm[pos];
    U[(size_t)pos * k + r] = (sig[c] > tiny) ? A[r + (size_t)c * k] / sig[c] : 0.0;
  }
  for (int pos = tid; pos < k; pos += kThreads) d[pos] = sig[perm[pos]];
  __syncthreads();
  for (int pos = 0; pos < k; ++pos) {
    if (sig[perm[pos]] > tiny) continue;
    for (int i = tid; i < k; i += kThreads) {
      double s = 0.0;
      for (int c = 0; c < pos; ++c) {
        const double x = U[(size_t)c * k + i];
        s += x * x;
      }
      coef[i] = s;
    }
    __syncthreads();
    if (tid == 0) {
      int best = 0;
      for (int i = 1; i < k; ++i)
        if (coef[i] < coef[best]) best = i;
      pick = best;
    }
    __syncthreads();
    const int ip = pick;
    double* u = U + (size_t)pos * k;
    for (int r = tid; r < k; r += kThreads) {
      double s = (r == ip) ? 1.0 : 0.0;
      for (int c = 0; c < pos; ++c) s -= U[(size_t)c * k + r] * U[(size_t)c * k + ip];
      u[r] = s;
    }
    __syncthreads();
    for (int c = tid; c < pos; c += kThreads) {
      double s = 0.0;
      for (int r = 0; r < k; ++r) s += U[(size_t)c * k + r] * u[r];
      coef[c] = s;
    }
    __syncthreads();
    for (int r = tid; r < k; r += kThreads) {
      double s = u[r];
      for (int c = 0; c < pos; ++c) s -= U[(size_t)c * k + r] * coef[c];
      u[r] = s;
    }
    __syncthreads();
    if (wave == 0) {
      double s = 0.0;
      for (int r = lane; r < k; r += 64) s += u[r] * u[r];
      s = wave_sum(s);
      if (lane == 0) coef[0] = 1.0 / sqrt(s);
    }
    __syncthreads();
    const double inv = coef[0];
    for (int r = tid; r < k; r += kThreads) u[r] *= inv;
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void copy_square_kernel(int k, const double* B, int64_t ldb,
                                                          double* A) {
  for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < (int64_t)k * k;
       idx += (int64_t)gridDim.x * 256) {
    const int64_t r = idx % k, c = idx / k;
    A[idx] = B[r + c * ldb];
  }
}

}  // namespace

size_t left_svd_work_bytes(int k) {
  if (k < 1 || k > kMaxK) return 0;
  return (size_t)round_up((int64_t)k * k * 8, 256) + 256;
}

int left_svd(hipStream_t st, int k, const double* B, int64_t ldb, double* U, double* d, void* work,
             size_t work_bytes, int* status) {
  if (k < 1 || k > kMaxK) return set_error(RRF_E_NOTSUP, "left_svd: needs 1 <= k <= 256");
  if (work == nullptr || work_bytes < left_svd_work_bytes(k))
    return set_error(RRF_E_NOMEM, "left_svd: workspace too small");
  double* A = reinterpret_cast<double*>(work);
  unsigned* rot = reinterpret_cast<unsigned*>(reinterpret_cast<char*>(work) +
                                              round_up((int64_t)k * k * 8, 256));
  const size_t lds = (size_t)2 * kCB * k * sizeof(double);
  RRF_TRY(allow_dynamic_lds((const void*)block_round_kernel, 2 * kCB * kMaxK * sizeof(double)));
  int tok = trace_begin(st, kTrJacobi, 0.0, 0.0);
  RRF_TRY(fill_u32(st, rot, kMaxOuter, 0u));
  hipLaunchKernelGGL(copy_square_kernel, dim3((unsigned)ceil_div((int64_t)k * k, 256)), dim3(256),
                     0, st, k, B, ldb, A);
  const int nblk = (int)ceil_div(k, kCB);
  const int nb = nblk + (nblk & 1);
  if (nblk > 1) {
    for (int sw = 0; sw < kMaxOuter; ++sw)
      for (int r = 0; r < nb - 1; ++r) {
        RoundArgs ra{k, nb, r, sw, A, rot};
        hipLaunchKernelGGL(block_round_kernel, dim3((unsigned)(nb / 2)), dim3(kThreads), lds, st,
                           ra);
      }
  } else {
    // one block: a single meeting of the block with the (empty) padding
    // block per sweep
    for (int sw = 0; sw < kMaxOuter; ++sw) {
      RoundArgs ra{k, 2, 0, sw, A, rot};
      hipLaunchKernelGGL(block_round_kernel, dim3(1), dim3(kThreads), lds, st, ra);
    }
  }
  hipLaunchKernelGGL(left_finish_kernel, dim3(1), dim3(kThreads), 0, st, k, (const double*)A, U, d,
                     (const unsigned*)rot, status);
  trace_end(st, tok);
  RRF_CHECK_HIP(hipGetLastError());
  return RRF_OK;
}

}  // namespace rrf
