// Householder QR of a tall M x k panel (k <= 64) with compact-WY output
// (Sec. 2.3), computed as a tree of small QRs followed by reconstruction of
// the Householder reflectors.
//
// The column-by-column panel needs one grid-wide exchange per column. Here
// the panel is cut into leaf blocks of 256 rows, one per workgroup, and:
//  1. every workgroup factors its leaf in registers (Householder, dlarfg
//     rule): leaf = Q_g [R_g; 0];
//  2. the R factors are combined up a binary tree: the owner of a node
//     factors [R_left; R_right] (two k x k upper triangles) by reflectors
//     [e_j; y_j] whose lower parts y_j are nonzero in rows 0..j only; the
//     left R is the owner's own, the right one arrives from its partner;
//  3. the thin Q of the whole panel is formed top-down: the root starts
//     from E = I_k, each node hands E_right = -Y T E to its partner and keeps
//     E_left = E - T E, and each leaf forms Q_g = [E_g; 0] - V_g T_g V_g1^T E_g
//     (V_g1 = the top k rows of V_g);
//  4. the reflectors of the unblocked Householder QR of the panel are
//     recovered from Q: with S = diag(s_i) chosen on the way so that every
//     pivot has magnitude >= 1, Q_1 - S = L U (no pivoting), and then
//     W = [L; Q_2 U^-1], Tf = -U S L^-T and R = S R_root, so that
//     I - W Tf W^T has first k columns Q S and (I - W Tf W^T) [R; 0] equals
//     the panel. With s_i = -sign of the pivot's diagonal entry this is the
//     factorization the dlarfg sign rule gives (the same W, Tf, R and tau up
//     to rounding), except that a reflector dlarfg leaves as the identity
//     (a zero column below the diagonal) comes back as a true reflection
//     with the matching row of R negated.
// All of it is one cooperative launch: workgroup g owns leaf g and the tree
// nodes above it on its leftmost path; partners exchange R and E through
// device-coherent stores and a flag each, so only the tree's critical path
// (about log2(M / 256) small QRs and triangular products) is serial.
//
// Thread layout everywhere: lane (c, p) = (tid / 8, tid % 8) works on column
// c, rows p + 8 i. Sums over rows are reduced across the 8 lanes of a column
// with a butterfly of shuffles, which gives every lane the same bits.
#include <hip/hip_cooperative_groups.h>

#include <algorithm>

#include "common.hpp"
#include "context.hpp"
#include "kernels.hpp"
#include "trace.hpp"

namespace rrf {

namespace {

constexpr int kThreads = 512;
constexpr int kLeaf = 256;        // rows per leaf
constexpr int kK = 64;            // widest panel
constexpr int kLR = kLeaf / 8;    // leaf rows per lane
constexpr int kNR = kK / 8;       // rows of a k x k block per lane
constexpr int kS = 68;            // LDS row stride of a k x k block
constexpr int kBlk = kK * kS;     // doubles per LDS block
constexpr int kVS = kLeaf + 4;    // LDS stride of a staged leaf column
constexpr int kStage = 16;        // leaf columns staged at once (kStage * kVS <= kBlk)
constexpr int kMaxLeaves = 256;
constexpr int kFlagStride = 16;   // unsigned per flag: one 64-byte line
constexpr long kSpinLimit = 1L << 22;
constexpr size_t kKK = (size_t)kK * kK;  // doubles per global k x k slot

// dynamic LDS: two reflector buffers, tau, signs, four k x k blocks
constexpr size_t kLdsDoubles = 2 * kLeaf + 2 * kK + 4 * (size_t)kBlk;
constexpr size_t kLdsBytes = kLdsDoubles * 8;

struct Args {
  int64_t M;
  int k;
  const double* P;
  int64_t ldp;
  double* W;
  int64_t ldw;
  double* R;
  int64_t ldr;
  double* Tf;
  int64_t ldt;
  double* tau;
  double* zero;
  int64_t ldz;
  int G;              // leaves = workgroups
  int L;              // tree levels, ceil(log2 G)
  unsigned* flagR;    // G flags: the workgroup's R is published
  unsigned* flagE;    // G flags: the workgroup's E has arrived
  unsigned* flagU;    // one flag: U^-1 is published
  double* xR;         // G slots
  double* xE;         // G slots
  double* xU;         // one slot
  double* leafT;      // G slots
  double* nodes;      // 2 slots (Y, T) per tree node
  int* status;
};

__device__ inline void st_dev(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline double ld_dev(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Value of lane (lane ^ 1), (lane ^ 2) or (7 - lane) within each group of 8
// lanes (DPP quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror),
// moved as two 32-bit halves.
template <int kCtrl>
__device__ inline double dpp_move(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, kCtrl, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), kCtrl, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
constexpr int kDppXor1 = 0xb1, kDppXor2 = 0x4e, kDppHalfMirror = 0x141;

// Sum over the 8 lanes of a column group: pairs, then quads, then the two
// quads of the group. Each partial sum is formed from the same two operands
// in every lane that holds it, so every lane gets the same bits.
__device__ inline double red8(double x) {
  x += dpp_move<kDppXor1>(x);
  x += dpp_move<kDppXor2>(x);
  x += dpp_move<kDppHalfMirror>(x);
  return x;
}

// Reflector of (alpha, x) with ||x||^2 = xn2 by the dlarfg rule.
__device__ inline void larfg(double alpha, double xn2, double& tau, double& beta, double& scal) {
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
}

// Make this workgroup's device-coherent stores visible, then raise `flag`.
__device__ inline void publish(unsigned* flag) {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait (bounded) until `flag` is raised; false with status bit 4 on a timeout
// or when another workgroup has failed.
__device__ inline bool wait_flag(const Args& a, const unsigned* flag) {
  int good = 1;
  if (threadIdx.x == 0) {
    long spins = 0;
    while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > kSpinLimit ||
          __hip_atomic_load(a.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
        good = 0;
        atomicOr(a.status, 4);
        break;
      }
    }
  }
  return __syncthreads_and(good) != 0;
}

// Entry j of a column group's distributed register array (index j >> 3 in
// lane p == (j & 7)), summed with zeros from the other lanes: every lane of
// the group gets it (a -0.0 comes back as +0.0).
template <int N>
__device__ inline double pick(const double (&x)[N], int j, int p) {
  double v = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i)
    if (p + 8 * i == j) v = x[i];
  return red8(v);
}

// The same when group j is the only active group of its wavefront (lane
// 9 (j & 7) of the wavefront holds it): read from that lane, sign of zero
// kept.
template <int N>
__device__ inline double pick_owner(const double (&x)[N], int j, int p) {
  double v = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i)
    if (p + 8 * i == j) v = x[i];
  const long long b = __double_as_longlong(v);
  const int src = 9 * (j & 7);
  const int lo = __builtin_amdgcn_readlane((int)b, src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

template <int N>
__device__ inline void put(double (&x)[N], int j, int p, double v) {
#pragma unroll
  for (int i = 0; i < N; ++i)
    if (p + 8 * i == j) x[i] = v;
}

// Row c of the T factor, column jm = j - 1 (called in step j, when the dots
// D(., jm) of reflector jm with the earlier ones are in LDS): lane p holds
// T(c, p + 8 m) in t[m]; T(c, jm) = -tau_jm sum_{c <= u < jm} T(c, u) D(u, jm).
__device__ inline void t_column(double (&t)[kNR], int c, int p, int jm, const double* taus,
                                const double* D) {
  double s = 0.0;
#pragma unroll
  for (int m = 0; m < kNR; ++m) {
    const int u = p + 8 * m;
    if (u >= c && u < jm) s += t[m] * D[u * kS + jm];
  }
  s = red8(s);
  put(t, jm, p, -taus[jm] * s);
}

// Householder QR of the leaf in a[] (rows p + 8 i of column c). On return a[]
// holds R on and above the diagonal and the reflectors below it, taus[] the
// tau_j and t[] row c of the leaf's T. Rows p + 8 i with i >= kNR are >= kK
// and so below every diagonal entry: only the first kNR rows of a lane need
// the comparisons with j.
__device__ void leaf_qr(double (&a)[kLR], double (&t)[kNR], int k, int c, int p, double* vbuf,
                        double* taus, double* D) {
  double s = 0.0;  // ||x||^2 below the diagonal of the next owner's column
  if (c == 0) {
    double s0 = 0.0;
#pragma unroll
    for (int i = 0; i < kLR; ++i)
      if (p + 8 * i > 0) s0 += a[i] * a[i];
    s = red8(s0);
  }
  for (int j = 0; j < k; ++j) {
    double* v = vbuf + (j & 1) * kLeaf;
    if (c == j) {
      double al[kNR];
#pragma unroll
      for (int i = 0; i < kNR; ++i) al[i] = a[i];
      const double alpha = pick_owner(al, j, p);
      double tau, beta, scal;
      larfg(alpha, s, tau, beta, scal);
#pragma unroll
      for (int i = 0; i < kNR; ++i) {
        const int r = p + 8 * i;
        const double vv = r > j ? a[i] * scal : (r == j ? 1.0 : 0.0);
        v[r] = vv;
        a[i] = r > j ? vv : (r == j ? beta : a[i]);
      }
#pragma unroll
      for (int i = kNR; i < kLR; ++i) {
        a[i] *= scal;
        v[p + 8 * i] = a[i];
      }
      if (p == 0) taus[j] = tau;
      put(t, j, p, tau);
    }
    __syncthreads();
    if (c < k && c != j) {
      double d0 = 0.0, d1 = 0.0;
#pragma unroll
      for (int i = 0; i < kLR; i += 2) {
        d0 += v[p + 8 * i] * a[i];
        d1 += v[p + 8 * i + 8] * a[i + 1];
      }
      const double d = red8(d0 + d1);
      if (c > j) {
        const double f = taus[j] * d;
        double s1 = 0.0;
#pragma unroll
        for (int i = 0; i < kNR; ++i) {
          const int r = p + 8 * i;
          a[i] -= f * v[r];
          if (r > j + 1) s1 += a[i] * a[i];
        }
#pragma unroll
        for (int i = kNR; i < kLR; ++i) {
          a[i] -= f * v[p + 8 * i];
          s1 += a[i] * a[i];
        }
        if (c == j + 1) s = red8(s1);
      } else {
        if (p == 0) D[c * kS + j] = d;  // v_c . v_j
        if (c < j - 1) t_column(t, c, p, j - 1, taus, D);
      }
    }
  }
  __syncthreads();
  if (c < k - 1) t_column(t, c, p, k - 1, taus, D);
}

// QR of [R1; R2], two k x k upper triangles: R1 in LDS (row-major, stride
// kS), R2 in b[] (rows p + 8 i of column c). Reflector j is [e_j; y_j] with
// y_j in rows 0..j of the lower block. On return R1s holds the new R, b[]
// holds y_c, taus[] the tau_j and t[] row c of the node's T.
__device__ void node_qr(double (&b)[kNR], double (&t)[kNR], int k, int c, int p, double* R1s,
                        double* vbuf, double* taus, double* D) {
  double s = 0.0;
  if (c == 0) s = red8(p == 0 ? b[0] * b[0] : 0.0);
  for (int j = 0; j < k; ++j) {
    double* y = vbuf + (j & 1) * kLeaf;
    if (c == j) {
      const double alpha = R1s[j * kS + j];
      double tau, beta, scal;
      larfg(alpha, s, tau, beta, scal);
#pragma unroll
      for (int i = 0; i < kNR; ++i) {
        const int r = p + 8 * i;
        const double yy = r <= j ? b[i] * scal : 0.0;
        y[r] = yy;
        b[i] = yy;
      }
      put(t, j, p, tau);
      if (p == 0) {
        taus[j] = tau;
        R1s[j * kS + j] = beta;
      }
    }
    __syncthreads();
    if (c < k && c != j) {
      double d = 0.0;
#pragma unroll
      for (int i = 0; i < kNR; ++i) d += y[p + 8 * i] * b[i];
      d = red8(d);
      if (c > j) {
        const double w = R1s[j * kS + c] + d;
        const double f = taus[j] * w;
        double s1 = 0.0;
#pragma unroll
        for (int i = 0; i < kNR; ++i) {
          const int r = p + 8 * i;
          b[i] -= f * y[r];
          if (r <= j + 1) s1 += b[i] * b[i];
        }
        if (c == j + 1) s = red8(s1);
        if (p == 0) R1s[j * kS + c] = R1s[j * kS + c] - f;
      } else {
        if (p == 0) D[c * kS + j] = d;  // y_c . y_j = v_c . v_j
        if (c < j - 1) t_column(t, c, p, j - 1, taus, D);
      }
    }
  }
  __syncthreads();
  if (c < k - 1) t_column(t, c, p, k - 1, taus, D);
}

// out[i] = sum_{u < k} op(A)(p + 8 i, u) B(u, c), A and B k x k blocks in LDS
// (row-major, stride kS); op(A) = A^T when TA.
template <bool TA>
__device__ inline void lds_mm(const double* A, const double* B, int k, int c, int p,
                              double (&out)[kNR]) {
#pragma unroll
  for (int i = 0; i < kNR; ++i) out[i] = 0.0;
  if (c >= k) return;
  for (int u = 0; u < k; ++u) {
    const double bu = B[u * kS + c];
#pragma unroll
    for (int i = 0; i < kNR; ++i) {
      const int r = p + 8 * i;
      out[i] += (TA ? A[u * kS + r] : A[r * kS + u]) * bu;
    }
  }
}

__device__ inline int node_slot(int G, int l, int g) {
  int off = 0;
  for (int q = 1; q < l; ++q) off += (G + (1 << q) - 1) >> q;
  return off + (g >> l);
}

__global__ __launch_bounds__(kThreads) void tsqr_kernel(Args a) {
  extern __shared__ double smem[];
  double* vbuf = smem;                  // 2 x kLeaf
  double* taus = vbuf + 2 * kLeaf;      // kK
  double* sgn = taus + kK;              // kK
  double* B0 = sgn + kK;                // four k x k blocks
  double* B1 = B0 + kBlk;
  double* B2 = B1 + kBlk;
  double* B3 = B2 + kBlk;

  const int tid = threadIdx.x;
  const int c = tid >> 3, p = tid & 7;
  const int g = blockIdx.x;
  const int k = a.k;
  const int G = a.G;
  const int64_t r0 = (int64_t)g * kLeaf;

  // ---- leaf: load (and clear the source when asked), factor
  double q[kLR];
#pragma unroll
  for (int i = 0; i < kLR; ++i) {
    const int64_t r = r0 + p + 8 * i;
    q[i] = (c < k && r < a.M) ? a.P[r + (int64_t)c * a.ldp] : 0.0;
  }
  if (a.zero && c < k) {
#pragma unroll
    for (int i = 0; i < kLR; ++i) {
      const int64_t r = r0 + p + 8 * i;
      if (r < a.M) a.zero[r + (int64_t)c * a.ldz] = 0.0;
    }
  }
  double t[kNR];
#pragma unroll
  for (int m = 0; m < kNR; ++m) t[m] = 0.0;
  leaf_qr(q, t, k, c, p, vbuf, taus, B1);

  if (G == 1) {
    // one leaf: its factorization is the panel's
    if (c < k) {
#pragma unroll
      for (int m = 0; m < kNR; ++m) {
        const int u = p + 8 * m;
        if (u < k) a.Tf[c + (int64_t)u * a.ldt] = t[m];
      }
      if (p == 0) a.tau[c] = taus[c];
#pragma unroll
      for (int i = 0; i < kLR; ++i) {
        const int64_t r = p + 8 * i;
        if (r < a.M) a.W[r + (int64_t)c * a.ldw] = r > c ? q[i] : (r == c ? 1.0 : 0.0);
        if (a.R && r < k) a.R[r + (int64_t)c * a.ldr] = r <= c ? q[i] : 0.0;
      }
    }
    return;
  }

  // the leaf's T, and its reflectors in the leaf's rows of W (read back to
  // form the leaf's rows of Q)
  if (c < k) {
#pragma unroll
    for (int m = 0; m < kNR; ++m) a.leafT[(size_t)g * kKK + (size_t)c * kK + p + 8 * m] = t[m];
#pragma unroll
    for (int i = 0; i < kLR; ++i) {
      const int r = p + 8 * i;
      if (r0 + r < a.M) a.W[r0 + r + (int64_t)c * a.ldw] = r > c ? q[i] : (r == c ? 1.0 : 0.0);
    }
  }

  // ---- tree: workgroup g owns nodes at levels 1 .. lv (its leftmost path)
  const int lv = (g == 0) ? a.L : __builtin_ctz((unsigned)g);
  if (lv == 0) {
    // odd workgroup: the leaf's R goes to its partner
#pragma unroll
    for (int i = 0; i < kNR; ++i) {
      const int r = p + 8 * i;
      st_dev(a.xR + (size_t)g * kKK + (size_t)r * kK + c, (r <= c && c < k) ? q[i] : 0.0);
    }
    publish(a.flagR + (size_t)g * kFlagStride);
  } else {
#pragma unroll
    for (int i = 0; i < kNR; ++i) {
      const int r = p + 8 * i;
      B0[r * kS + c] = (r <= c && c < k) ? q[i] : 0.0;
    }
    __syncthreads();
    for (int l = 1; l <= lv; ++l) {
      const int partner = g + (1 << (l - 1));
      if (partner >= G) continue;
      if (!wait_flag(a, a.flagR + (size_t)partner * kFlagStride)) return;
      double b[kNR];
#pragma unroll
      for (int i = 0; i < kNR; ++i)
        b[i] = ld_dev(a.xR + (size_t)partner * kKK + (size_t)(p + 8 * i) * kK + c);
#pragma unroll
      for (int m = 0; m < kNR; ++m) t[m] = 0.0;
      node_qr(b, t, k, c, p, B0, vbuf, taus, B1);
      double* slot = a.nodes + (size_t)node_slot(G, l, g) * 2 * kKK;
#pragma unroll
      for (int i = 0; i < kNR; ++i) {
        slot[(size_t)(p + 8 * i) * kK + c] = (c < k) ? b[i] : 0.0;      // Y(r, c)
        slot[kKK + (size_t)c * kK + p + 8 * i] = (c < k) ? t[i] : 0.0;  // T(c, u)
      }
      __syncthreads();
    }
    // the subtree's R: to the partner, or (root) kept for the output in the
    // slot of xR that workgroup 0 never publishes
#pragma unroll
    for (int i = 0; i < kNR; ++i) {
      const int r = p + 8 * i;
      st_dev(a.xR + (size_t)g * kKK + (size_t)r * kK + c, B0[r * kS + c]);
    }
    if (g > 0) publish(a.flagR + (size_t)g * kFlagStride);
  }
  __syncthreads();

  // ---- top-down: E of this workgroup's subtree, then of each node below it
  if (g == 0) {
#pragma unroll
    for (int i = 0; i < kNR; ++i) {
      const int r = p + 8 * i;
      B0[r * kS + c] = (r == c && r < k) ? 1.0 : 0.0;
    }
  } else {
    if (!wait_flag(a, a.flagE + (size_t)g * kFlagStride)) return;
#pragma unroll
    for (int i = 0; i < kNR; ++i) {
      const int r = p + 8 * i;
      B0[r * kS + c] = ld_dev(a.xE + (size_t)g * kKK + (size_t)r * kK + c);
    }
  }
  __syncthreads();
  double o[kNR];
  for (int l = lv; l >= 1; --l) {
    const int partner = g + (1 << (l - 1));
    if (partner >= G) continue;
    const double* slot = a.nodes + (size_t)node_slot(G, l, g) * 2 * kKK;
#pragma unroll
    for (int i = 0; i < kNR; ++i) {
      const int r = p + 8 * i;
      B2[r * kS + c] = slot[(size_t)r * kK + c];         // Y
      B3[r * kS + c] = slot[kKK + (size_t)r * kK + c];   // T
    }
    __syncthreads();
    lds_mm<false>(B3, B0, k, c, p, o);                   // T E
#pragma unroll
    for (int i = 0; i < kNR; ++i) B1[(p + 8 * i) * kS + c] = o[i];
    __syncthreads();
    lds_mm<false>(B2, B1, k, c, p, o);                   // Y T E
#pragma unroll
    for (int i = 0; i < kNR; ++i)
      st_dev(a.xE + (size_t)partner * kKK + (size_t)(p + 8 * i) * kK + c, -o[i]);
    publish(a.flagE + (size_t)partner * kFlagStride);
#pragma unroll
    for (int i = 0; i < kNR; ++i) {
      const int r = p + 8 * i;
      B0[r * kS + c] -= B1[r * kS + c];
    }
    __syncthreads();
  }

  // ---- the leaf's rows of Q: [E; 0] - V (T (V1^T E)), V read back from W
  const int64_t rows = std::min<int64_t>(kLeaf, a.M - r0);  // real rows of the leaf
#pragma unroll
  for (int i = 0; i < kNR; ++i) {
    const int r = p + 8 * i;
    B1[r * kS + c] = (c < k && r < rows) ? a.W[r0 + r + (int64_t)c * a.ldw] : 0.0;  // V1
    B3[r * kS + c] = a.leafT[(size_t)g * kKK + (size_t)r * kK + c];              // T_g
  }
  __syncthreads();
  lds_mm<true>(B1, B0, k, c, p, o);                       // X = V1^T E
#pragma unroll
  for (int i = 0; i < kNR; ++i) B2[(p + 8 * i) * kS + c] = o[i];
  __syncthreads();
  lds_mm<false>(B3, B2, k, c, p, o);                      // Z = T_g X
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kNR; ++i) B1[(p + 8 * i) * kS + c] = o[i];
#pragma unroll
  for (int i = 0; i < kLR; ++i) {
    const int r = p + 8 * i;
    q[i] = (i < kNR && c < k && r < k) ? B0[r * kS + c] : 0.0;
  }
  // columns [cs, cs + kStage) of the leaf's W rows (rows past the panel are
  // zero) into B2, column-major with stride kVS
  auto stage = [&](int cs) {
    for (int idx = tid; idx < kStage * kLeaf; idx += kThreads) {
      const int cc = idx / kLeaf, r = idx % kLeaf;
      B2[cc * kVS + r] =
          (cs + cc < k && r < rows) ? a.W[r0 + r + (int64_t)(cs + cc) * a.ldw] : 0.0;
    }
  };
  for (int cs = 0; cs < k; cs += kStage) {
    __syncthreads();
    stage(cs);
    __syncthreads();
    if (c < k) {
      const int ce = min(cs + kStage, k);
      for (int u = cs; u < ce; ++u) {
        const double z = B1[u * kS + c];
        const double* vc = B2 + (u - cs) * kVS;
#pragma unroll
        for (int i = 0; i < kLR; ++i) q[i] -= vc[p + 8 * i] * z;
      }
    }
  }
  // q[] = the leaf's rows of Q: to W (read back for W = Q U^-1), and
  // workgroup 0 keeps its top k rows
  __syncthreads();
  double lu[kNR];
#pragma unroll
  for (int i = 0; i < kNR; ++i) lu[i] = q[i];
  if (c < k) {
#pragma unroll
    for (int i = 0; i < kLR; ++i) {
      const int r = p + 8 * i;
      if (r < rows) a.W[r0 + r + (int64_t)c * a.ldw] = q[i];
    }
  }

  // ---- workgroup 0: Q1 - S = L U, U^-1, Tf = -U S L^-T, R = S R_root
  if (g == 0) {
    for (int i = 0; i < k; ++i) {
      double* lb = vbuf + (i & 1) * kLeaf;
      if (c == i) {
        const double d = pick(lu, i, p);
        const double si = d >= 0.0 ? -1.0 : 1.0;
        const double piv = d - si;
#pragma unroll
        for (int m = 0; m < kNR; ++m) {
          const int r = p + 8 * m;
          if (r > i) lu[m] = lu[m] / piv;
          if (r == i) lu[m] = piv;
          lb[r] = r > i ? lu[m] : 0.0;
        }
        if (p == 0) sgn[i] = si;
      }
      __syncthreads();
      if (c > i && c < k) {
        const double u = pick(lu, i, p);
#pragma unroll
        for (int m = 0; m < kNR; ++m) {
          const int r = p + 8 * m;
          if (r > i) lu[m] -= lb[r] * u;
        }
      }
    }
    // U -> B2, unit lower L -> B3 (row-major)
#pragma unroll
    for (int m = 0; m < kNR; ++m) {
      const int r = p + 8 * m;
      const bool in = c < k && r < k;
      B2[r * kS + c] = (in && r <= c) ? lu[m] : 0.0;
      B3[r * kS + c] = in ? (r > c ? lu[m] : (r == c ? 1.0 : 0.0)) : 0.0;
    }
    __syncthreads();
    // column c of U^-1 by back substitution, x_r in lane r & 7
#pragma unroll
    for (int m = 0; m < kNR; ++m) o[m] = 0.0;
    if (c < k) {
      for (int r = c; r >= 0; --r) {
        double s = 0.0;
#pragma unroll
        for (int m = 0; m < kNR; ++m) {
          const int u = p + 8 * m;
          if (u > r && u <= c) s += B2[r * kS + u] * o[m];
        }
        s = red8(s);
        put(o, r, p, ((r == c ? 1.0 : 0.0) - s) / B2[r * kS + r]);
      }
    }
    // row c of Tf = X with X L^T = -U S, X upper triangular (t[] holds it)
#pragma unroll
    for (int m = 0; m < kNR; ++m) t[m] = 0.0;
    if (c < k) {
      for (int cc = c; cc < k; ++cc) {
        double s = 0.0;
#pragma unroll
        for (int m = 0; m < kNR; ++m) {
          const int u = p + 8 * m;
          if (u >= c && u < cc) s += t[m] * B3[cc * kS + u];
        }
        s = red8(s);
        put(t, cc, p, -B2[c * kS + cc] * sgn[cc] - s);
      }
    }
    __syncthreads();  // B2 (U) no longer read
    if (c < k) {
#pragma unroll
      for (int m = 0; m < kNR; ++m) {
        const int u = p + 8 * m;
        // U^-1 (column c) to LDS and to the other workgroups
        B1[u * kS + c] = o[m];
        st_dev(a.xU + (size_t)u * kK + c, o[m]);
        if (u < k) {
          a.Tf[c + (int64_t)u * a.ldt] = u >= c ? t[m] : 0.0;
          if (u == c) a.tau[c] = t[m];
          if (a.R)
            a.R[u + (int64_t)c * a.ldr] =
                u <= c ? sgn[u] * ld_dev(a.xR + (size_t)u * kK + c) : 0.0;
        }
      }
    }
    publish(a.flagU);
  } else {
    if (!wait_flag(a, a.flagU)) return;
#pragma unroll
    for (int m = 0; m < kNR; ++m) {
      const int u = p + 8 * m;
      B1[u * kS + c] = ld_dev(a.xU + (size_t)u * kK + c);
    }
  }

  // ---- W = Q U^-1 on the leaf's rows, Q read back from W; workgroup 0's
  // top k rows are L
#pragma unroll
  for (int i = 0; i < kLR; ++i) q[i] = 0.0;
  for (int cs = 0; cs < k; cs += kStage) {
    __syncthreads();
    stage(cs);
    __syncthreads();
    if (c < k) {
      const int ce = min(cs + kStage, c + 1);
      for (int u = cs; u < ce; ++u) {
        const double z = B1[u * kS + c];
        const double* qc = B2 + (u - cs) * kVS;
#pragma unroll
        for (int i = 0; i < kLR; ++i) q[i] += qc[p + 8 * i] * z;
      }
    }
  }
  __syncthreads();  // every read of this leaf's W rows is done
  if (c < k) {
#pragma unroll
    for (int i = 0; i < kLR; ++i) {
      const int r = p + 8 * i;
      if (r < rows) {
        double v = q[i];
        if (g == 0 && r < k) {
          double l = 0.0;
#pragma unroll
          for (int m = 0; m < kNR; ++m)
            if (i == m) l = lu[m];
          v = r > c ? l : (r == c ? 1.0 : 0.0);
        }
        a.W[r0 + r + (int64_t)c * a.ldw] = v;
      }
    }
  }
}

size_t flags_bytes(int G) { return (size_t)round_up((int64_t)(2 * G + 1) * kFlagStride * 4, 256); }
int tree_levels(int G) {
  int L = 0;
  while ((1 << L) < G) ++L;
  return L;
}
int node_count(int G) {
  int n = 0;
  for (int l = 1; (1 << (l - 1)) < G; ++l) n += (G + (1 << l) - 1) >> l;
  return n;
}

}  // namespace

bool tsqr_panel_ok(int64_t M, int k) {
  return k >= 1 && k <= kK && M >= k && ceil_div(M, kLeaf) <= kMaxLeaves;
}

size_t tsqr_work_bytes(int64_t M, int k) {
  if (!tsqr_panel_ok(M, k)) return 0;
  const int G = (int)ceil_div(M, kLeaf);
  const size_t slots = (size_t)3 * G + 1 + (size_t)2 * node_count(G);
  return flags_bytes(G) + slots * kKK * 8;
}

int tsqr_panel(hipStream_t st, int64_t M, int k, const double* P, int64_t ldp, double* W,
               int64_t ldw, double* R, int64_t ldr, double* Tf, int64_t ldt, double* tau,
               double* zero, int64_t ldz, void* work, size_t work_bytes, int* status) {
  if (!tsqr_panel_ok(M, k))
    return set_error(RRF_E_NOTSUP, "tree panel: needs 1 <= k <= 64 and k <= M <= 65536");
  const size_t need = tsqr_work_bytes(M, k);
  if (work == nullptr || work_bytes < need)
    return set_error(RRF_E_NOMEM, "tree panel: workspace too small");
  RRF_TRY(allow_dynamic_lds((const void*)tsqr_kernel, kLdsBytes));
  const int G = (int)ceil_div(M, kLeaf);
  Args a{};
  a.M = M;
  a.k = k;
  a.P = P;
  a.ldp = ldp;
  a.W = W;
  a.ldw = ldw;
  a.R = R;
  a.ldr = ldr;
  a.Tf = Tf;
  a.ldt = ldt;
  a.tau = tau;
  a.zero = zero;
  a.ldz = ldz;
  a.G = G;
  a.L = tree_levels(G);
  unsigned* flags = reinterpret_cast<unsigned*>(work);
  a.flagR = flags;
  a.flagE = flags + (size_t)G * kFlagStride;
  a.flagU = flags + (size_t)2 * G * kFlagStride;
  double* slots = reinterpret_cast<double*>(reinterpret_cast<char*>(work) + flags_bytes(G));
  a.xR = slots;
  a.xE = a.xR + (size_t)G * kKK;
  a.leafT = a.xE + (size_t)G * kKK;
  a.xU = a.leafT + (size_t)G * kKK;
  a.nodes = a.xU + kKK;
  a.status = status;
  // Algorithmic traffic: the panel read once and W written (and the source
  // cleared when asked); flops of the unblocked QR.
  const double pbytes = 8.0 * (double)M * k * (zero ? 3.0 : 2.0);
  const double pflops = 2.0 * (double)M * k * k;
  RRF_TRY(fill_u32(st, flags, (int64_t)(2 * G + 1) * kFlagStride, 0u));
  void* args[] = {&a};
  int tok = trace_begin(st, kTrPanelTsqr, pflops, pbytes);
  hipError_t e = hipLaunchCooperativeKernel((const void*)tsqr_kernel, dim3(G), dim3(kThreads),
                                            args, (unsigned)kLdsBytes, st);
  trace_end(st, tok);
  RRF_CHECK_HIP(e);
  return RRF_OK;
}

}  // namespace rrf
