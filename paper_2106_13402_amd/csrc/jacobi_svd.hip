// SVD of the small k x k diagonal blocks (k <= 256) on one workgroup.
//
// Alg. 3 diagonalizes each b x b block R produced by the panel QR with an
// SVD (and the last trailing block, after its own QR); the paper ships those
// blocks to the host for MAGMA. Here the block never leaves the GPU: a
// one-sided (Hestenes) Jacobi iteration orthogonalizes the columns of
// A_work = R V by plane rotations, accumulating V, so that A_work = Us diag(d)
// with d_j = ||A_work(:, j)||. One-sided Jacobi computes small singular
// values to high relative accuracy, which is what makes T(k,k) ~ sigma_k
// meaningful deep into a decaying spectrum.
//
//  * 1024 threads = 16 wave64s; each round of the round-robin (circle)
//    ordering pairs all k columns disjointly, a wave takes one pair at a
//    time, its lanes stride over the k rows, and the three inner products
//    are butterfly-reduced across the wave;
//  * rotation: zeta = (a_qq - a_pp) / (2 a_pq), t = sign(zeta) /
//    (|zeta| + sqrt(1 + zeta^2)), c = 1/sqrt(1+t^2), s = c t (Rutishauser);
//    a pair is rotated while |a_pq| > max(sqrt(k), 8) eps sqrt(a_pp a_qq)
//    (the rounding level of the wave-tree dot product is ~log2(k) eps, so
//    this converges, and the cosines left keep ||Us^T Us - I|| ~ k eps);
//  * A_work and V live in LDS when 2 k^2 doubles fit; otherwise A_work alone
//    when k^2 do (k <= 128: every inner product and rotation of A_work stays
//    on chip, and V, touched once per rotation, stays in L2), else both in
//    global scratch;
//  * finally: singular values sorted descending (stable in column index),
//    Us = A_work / d, columns with d = 0 completed to an orthonormal basis
//    by projecting the coordinate vector least covered by the columns so
//    far, and each pair (u_j, v_j) signed so that the entry of v_j of largest
//    magnitude is positive (lowest index on ties).
#include <cfloat>

#include "common.hpp"
#include "context.hpp"
#include "kernels.hpp"
#include "trace.hpp"

namespace rrf {

namespace {

constexpr int kThreads = 1024;
constexpr int kWaves = kThreads / 64;
constexpr int kMaxK = 256;
constexpr size_t kLdsBudget = 144 * 1024;
constexpr int kMaxSweeps = 60;

struct SvdArgs {
  int k;           // size of blocks 0 .. count-2
  int k_last;      // size of the last block
  int count;       // number of blocks (one workgroup each)
  int64_t stride;  // elements between consecutive blocks of B, Us, Vs
  int64_t dstride; // elements between consecutive d vectors
  const double* B;
  int64_t ldb;     // leading dimension of each B block (>= its size)
  double* Us;      // each block k x k, ld k
  double* d;
  double* Vs;
  double* gA;  // global scratch: per block 2 k^2 doubles when not in LDS
  int use_lds;  // 2: A_work and V in LDS, 1: A_work in LDS and V in gA, 0: both in gA
  int* status;
  const int* sizes;  // per-block sizes (device), or null
};

// Value of lane (lane ^ 1), (lane ^ 2), (7 - lane) within 8 or (15 - lane)
// within 16 (DPP quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror,
// row_mirror), moved as two 32-bit halves.
template <int kCtrl>
__device__ inline double dpp_move(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, kCtrl, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), kCtrl, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ inline double lane_value(double x, int src) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)b, src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum over the wavefront (all 64 lanes active): within each row of 16 lanes
// by four DPP exchanges, then the four row sums read as scalars and added in
// one order, so every lane gets the same bits.
__device__ inline double wave_sum(double v) {
  v += dpp_move<0xb1>(v);
  v += dpp_move<0x4e>(v);
  v += dpp_move<0x141>(v);
  v += dpp_move<0x140>(v);
  return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

// Singular values, descending order, outputs, completion of Us and the sign
// rule, for a converged block: Aw = A V and Vw = V, columns ldw apart, in
// LDS or global memory; NT threads; the small shared arrays come from the
// kernel.
template <int NT>
__device__ void finish_block(int k, const double* Aw, const double* Vw, int ldw, double* sig,
                             int* perm, double* coef, int& pick, double* Usb, double* Vsb,
                             double* db) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // Column norms = singular values.
  for (int c = wave; c < k; c += (NT / 64)) {
    double s = 0.0;
    for (int r = lane; r < k; r += 64) {
      const double x = Aw[(size_t)c * ldw + r];
      s += x * x;
    }
    s = wave_sum(s);
    if (lane == 0) sig[c] = sqrt(s);
  }
  __syncthreads();
  // Descending order, ties broken by column index. The sort key maps NaN
  // (non-finite input) below every norm, so (key, index) is a strict total
  // order and the ranks always form a permutation of 0..k-1.
  for (int c = tid; c < k; c += NT) {
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
  for (int idx = tid; idx < k * k; idx += NT) {
    const int r = idx % k, pos = idx / k;
    const int c = perm[pos];
    const double sc = sig[c];
    Vsb[(size_t)pos * k + r] = Vw[(size_t)c * ldw + r];
    Usb[(size_t)pos * k + r] = (sc > tiny) ? Aw[(size_t)c * ldw + r] / sc : 0.0;
  }
  for (int pos = tid; pos < k; pos += NT) db[pos] = sig[perm[pos]];
  __syncthreads();

  // Complete Us where d = 0 (these positions come last in the sorted order).
  for (int pos = 0; pos < k; ++pos) {
    if (sig[perm[pos]] > tiny) continue;
    double* U = Usb;
    // coverage of coordinate i by the columns 0..pos-1
    for (int i = tid; i < k; i += NT) {
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
    // u = e_ip - U U(ip,:)^T, then one re-orthogonalization pass.
    double* u = U + (size_t)pos * k;
    for (int r = tid; r < k; r += NT) {
      double s = (r == ip) ? 1.0 : 0.0;
      for (int c = 0; c < pos; ++c) s -= U[(size_t)c * k + r] * U[(size_t)c * k + ip];
      u[r] = s;
    }
    __syncthreads();
    for (int c = tid; c < pos; c += NT) {
      double s = 0.0;
      for (int r = 0; r < k; ++r) s += U[(size_t)c * k + r] * u[r];
      coef[c] = s;
    }
    __syncthreads();
    for (int r = tid; r < k; r += NT) {
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
    for (int r = tid; r < k; r += NT) u[r] *= inv;
    __syncthreads();
  }

  // Sign rule: the entry of v_j of largest magnitude is positive.
  for (int pos = wave; pos < k; pos += (NT / 64)) {
    double best = -1.0;
    int bi = 0;  // stays a valid row even if every entry is NaN
    for (int r = lane; r < k; r += 64) {
      const double x = fabs(Vsb[(size_t)pos * k + r]);
      if (x > best || (x == best && r < bi)) {
        best = x;
        bi = r;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    const bool flip = Vsb[(size_t)pos * k + bi] < 0.0;
    if (flip) {
      for (int r = lane; r < k; r += 64) {
        Vsb[(size_t)pos * k + r] = -Vsb[(size_t)pos * k + r];
        Usb[(size_t)pos * k + r] = -Usb[(size_t)pos * k + r];
      }
    }
  }
}

__global__ __launch_bounds__(kThreads) void jacobi_svd_kernel(SvdArgs a) {
  extern __shared__ double lds[];
  __shared__ double sig[kMaxK];
  __shared__ int perm[kMaxK];
  __shared__ int rotated;
  __shared__ double coef[kMaxK];
  __shared__ int pick;

  const int blk = blockIdx.x;
  const int k = a.sizes ? a.sizes[blk] : ((blk == a.count - 1) ? a.k_last : a.k);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* gbase = a.use_lds == 2 ? nullptr : a.gA + (size_t)blk * 2 * a.k * a.k;
  double* Aw = a.use_lds ? lds : gbase;
  double* Vw = a.use_lds == 2 ? lds + (size_t)k * k : gbase + (size_t)a.k * a.k;
  const double* Bb = a.B + (int64_t)blk * a.stride;
  double* Usb = a.Us + (int64_t)blk * a.stride;
  double* Vsb = a.Vs + (int64_t)blk * a.stride;
  double* db = a.d + (int64_t)blk * a.dstride;

  for (int idx = tid; idx < k * k; idx += kThreads) {
    const int i = idx % k, j = idx / k;
    Aw[idx] = Bb[i + (int64_t)j * a.ldb];
    Vw[idx] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();

  const int kk = k + (k & 1);
  const double tol = DBL_EPSILON * fmax(sqrt((double)k), 8.0);
  bool converged = (k == 1);
  for (int sweep = 0; sweep < kMaxSweeps && !converged; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int round = 0; round < kk - 1; ++round) {
      for (int pi = wave; pi < kk / 2; pi += kWaves) {
        int p, q;
        if (pi == 0) {
          p = round;
          q = kk - 1;
        } else {
          p = (round + pi) % (kk - 1);
          q = (round - pi + kk - 1) % (kk - 1);
        }
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        if (q >= k) continue;
        double* ap = Aw + (size_t)p * k;
        double* aq = Aw + (size_t)q * k;
        double app = 0.0, aqq = 0.0, apq = 0.0;
        for (int r = lane; r < k; r += 64) {
          const double x = ap[r], y = aq[r];
          app += x * x;
          aqq += y * y;
          apq += x * y;
        }
        app = wave_sum(app);
        aqq = wave_sum(aqq);
        apq = wave_sum(apq);
        if (apq != 0.0 && fabs(apq) > tol * sqrt(app) * sqrt(aqq)) {
          const double zeta = (aqq - app) / (2.0 * apq);
          double t;
          if (fabs(zeta) > 1e150) t = 0.5 / zeta;
          else t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + t * t);
          const double s = c * t;
          double* vp = Vw + (size_t)p * k;
          double* vq = Vw + (size_t)q * k;
          for (int r = lane; r < k; r += 64) {
            const double x = ap[r], y = aq[r];
            ap[r] = c * x - s * y;
            aq[r] = s * x + c * y;
            const double u = vp[r], w = vq[r];
            vp[r] = c * u - s * w;
            vq[r] = s * u + c * w;
          }
          if (lane == 0) rotated = 1;
        }
      }
      __syncthreads();
    }
    converged = (rotated == 0);
    __syncthreads();
  }
  if (!converged && tid == 0) atomicOr(a.status, 2);

  finish_block<kThreads>(k, Aw, Vw, k, sig, perm, coef, pick, Usb, Vsb, db);
}

// Blocks of k <= 64 on one wave each: the k/2 disjoint pairs of a round are
// spread over the wave, L = 64 / P lanes per pair (P = k/2 rounded up to a
// power of two), the lanes of a pair striding over the rows and reducing
// their three inner products among themselves. Same rotation, threshold,
// ordering and post-processing as jacobi_svd_kernel; A V and V in LDS with
// columns k + 1 apart (distinct pairs fall on distinct banks).
constexpr int kSmallK = 64;

__global__ __launch_bounds__(64) void jacobi_small_kernel(SvdArgs a) {
  extern __shared__ double lds[];
  __shared__ double sig[kSmallK];
  __shared__ int perm[kSmallK];
  __shared__ double coef[kSmallK];
  __shared__ int pick;

  const int blk = blockIdx.x;
  const int k = a.sizes ? a.sizes[blk] : ((blk == a.count - 1) ? a.k_last : a.k);
  const int lane = threadIdx.x;
  const int ld = k + 1;
  double* Aw = lds;
  double* Vw = lds + (size_t)k * ld;
  const double* Bb = a.B + (int64_t)blk * a.stride;
  double* Usb = a.Us + (int64_t)blk * a.stride;
  double* Vsb = a.Vs + (int64_t)blk * a.stride;
  double* db = a.d + (int64_t)blk * a.dstride;

  for (int idx = lane; idx < k * k; idx += 64) {
    const int i = idx % k, j = idx / k;
    Aw[i + j * ld] = Bb[i + (int64_t)j * a.ldb];
    Vw[i + j * ld] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();

  const int kk = k + (k & 1);
  const int npairs = kk / 2;
  int P = 1;
  while (P < npairs) P <<= 1;
  const int L = 64 / P;
  const int pi = lane / L, sub = lane % L;
  const double tol = DBL_EPSILON * fmax(sqrt((double)k), 8.0);
  bool converged = (k == 1);
  for (int sweep = 0; sweep < kMaxSweeps && !converged; ++sweep) {
    int rot = 0;
    for (int round = 0; round < kk - 1; ++round) {
      int p, q;
      if (pi == 0) {
        p = round;
        q = kk - 1;
      } else {
        p = (round + pi) % (kk - 1);
        q = (round - pi + kk - 1) % (kk - 1);
      }
      if (p > q) {
        const int t = p;
        p = q;
        q = t;
      }
      const bool active = pi < npairs && q < k;
      double* ap = Aw + (size_t)p * ld;
      double* aq = Aw + (size_t)q * ld;
      double app = 0.0, aqq = 0.0, apq = 0.0;
      if (active)
        for (int r = sub; r < k; r += L) {
          const double x = ap[r], y = aq[r];
          app += x * x;
          aqq += y * y;
          apq += x * y;
        }
      for (int off = L / 2; off > 0; off >>= 1) {
        app += __shfl_xor(app, off, 64);
        aqq += __shfl_xor(aqq, off, 64);
        apq += __shfl_xor(apq, off, 64);
      }
      if (active && apq != 0.0 && fabs(apq) > tol * sqrt(app) * sqrt(aqq)) {
        const double zeta = (aqq - app) / (2.0 * apq);
        double t;
        if (fabs(zeta) > 1e150) t = 0.5 / zeta;
        else t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t);
        const double s = c * t;
        double* vp = Vw + (size_t)p * ld;
        double* vq = Vw + (size_t)q * ld;
        for (int r = sub; r < k; r += L) {
          const double x = ap[r], y = aq[r];
          ap[r] = c * x - s * y;
          aq[r] = s * x + c * y;
          const double u = vp[r], w = vq[r];
          vp[r] = c * u - s * w;
          vq[r] = s * u + c * w;
        }
        rot = 1;
      }
      __syncthreads();
    }
    converged = !__any(rot);
  }
  if (!converged && lane == 0) atomicOr(a.status, 2);
  finish_block<64>(k, Aw, Vw, ld, sig, perm, coef, pick, Usb, Vsb, db);
}

// LDS of the one-wave kernel for blocks up to k.
size_t small_lds(int k) { return (size_t)2 * k * (k + 1) * 8; }

int launch_small(hipStream_t st, const SvdArgs& a, int kmax) {
  RRF_TRY(allow_dynamic_lds((const void*)jacobi_small_kernel, small_lds(kSmallK)));
  int tok = trace_begin(st, kTrJacobi, 0.0, 8.0 * 3.0 * kmax * kmax * a.count);
  hipLaunchKernelGGL(jacobi_small_kernel, dim3(a.count), dim3(64), small_lds(kmax), st, a);
  trace_end(st, tok);
  RRF_CHECK_HIP(hipGetLastError());
  return RRF_OK;
}

// The 1024-thread kernel for blocks up to kmax (> kSmallK): A_work and V in
// LDS, A_work only, or neither, by what fits.
int launch_large(hipStream_t st, SvdArgs& a, int kmax, void* work, size_t work_bytes) {
  const size_t both = (size_t)2 * kmax * kmax * 8, one = both / 2;
  a.use_lds = both <= kLdsBudget ? 2 : (one <= kLdsBudget ? 1 : 0);
  if (a.use_lds < 2 && (work == nullptr || work_bytes < both * a.count))
    return set_error(RRF_E_NOMEM, "block svd: workspace too small");
  a.gA = a.use_lds == 2 ? nullptr : reinterpret_cast<double*>(work);
  RRF_TRY(allow_dynamic_lds((const void*)jacobi_svd_kernel, kLdsBudget));
  const size_t lds = a.use_lds == 2 ? both : (a.use_lds == 1 ? one : 0);
  int tok = trace_begin(st, kTrJacobi, 0.0, 8.0 * 3.0 * kmax * kmax * a.count);
  hipLaunchKernelGGL(jacobi_svd_kernel, dim3(a.count), dim3(kThreads), lds, st, a);
  trace_end(st, tok);
  RRF_CHECK_HIP(hipGetLastError());
  return RRF_OK;
}

}  // namespace

size_t block_svd_work_bytes(int k) { return (size_t)2 * k * k * 8 + 256; }

int block_svd_batched(hipStream_t st, int count, int k, int k_last, const double* B, int64_t ldb,
                      int64_t stride, double* Us, double* d, int64_t dstride, double* Vs,
                      void* work, size_t work_bytes, int* status) {
  if (count < 1) return RRF_OK;
  if (k < 1 || k > kMaxK || k_last < 1 || k_last > k)
    return set_error(RRF_E_NOTSUP, "block svd: need 1 <= k_last <= k <= 256");
  if (k <= kSmallK) {
    SvdArgs a{};
    a.k = k;
    a.k_last = k_last;
    a.count = count;
    a.stride = stride;
    a.dstride = dstride;
    a.B = B;
    a.ldb = ldb;
    a.Us = Us;
    a.d = d;
    a.Vs = Vs;
    a.status = status;
    return launch_small(st, a, k);
  }
  SvdArgs a{};
  a.k = k;
  a.k_last = k_last;
  a.count = count;
  a.stride = stride;
  a.dstride = dstride;
  a.B = B;
  a.ldb = ldb;
  a.Us = Us;
  a.d = d;
  a.Vs = Vs;
  a.status = status;
  return launch_large(st, a, k, work, work_bytes);
}

int block_svd_sized(hipStream_t st, int count, int kmax, const int* d_sizes, const double* B,
                    int64_t ldb, int64_t stride, double* Us, double* d, int64_t dstride,
                    double* Vs, void* work, size_t work_bytes, int* status) {
  if (count < 1) return RRF_OK;
  if (kmax < 1 || kmax > kMaxK) return set_error(RRF_E_NOTSUP, "block svd: need k <= 256");
  if (kmax <= kSmallK) {
    SvdArgs a{};
    a.k = kmax;
    a.k_last = kmax;
    a.count = count;
    a.stride = stride;
    a.dstride = dstride;
    a.B = B;
    a.ldb = ldb;
    a.Us = Us;
    a.d = d;
    a.Vs = Vs;
    a.status = status;
    a.sizes = d_sizes;
    return launch_small(st, a, kmax);
  }
  SvdArgs a{};
  a.k = kmax;
  a.k_last = kmax;
  a.count = count;
  a.stride = stride;
  a.dstride = dstride;
  a.B = B;
  a.ldb = ldb;
  a.Us = Us;
  a.d = d;
  a.Vs = Vs;
  a.status = status;
  a.sizes = d_sizes;
  return launch_large(st, a, kmax, work, work_bytes);
}

int block_svd(hipStream_t st, int k, const double* B, int64_t ldb, double* Us, double* d,
              double* Vs, void* work, size_t work_bytes, int* status) {
  return block_svd_batched(st, 1, k, k, B, ldb, 0, Us, d, 0, Vs, work, work_bytes, status);
}

}  // namespace rrf
