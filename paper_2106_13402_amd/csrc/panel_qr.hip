// Householder QR of a tall M x k panel with compact-WY output (Sec. 2.3).
//
// Q = H_1 H_2 ... H_k = I - W Tf W^T, H_j = I - tau_j v_j v_j^T, with the
// reflectors chosen by the LAPACK dlarfg rule (beta = -sign(alpha) ||x||,
// tau = (beta - alpha) / beta, v = [1; x / (alpha - beta)], and H = I when
// the sub-column is zero). This is the HQR_full of the sketch Y and of the
// panel T(I2 u I3, J2) in Alg. 3, and the panel step of the blocked HQR used by
// Alg. 1.
//
// A panel is latency-bound: k reflectors in sequence, each needing sums over
// all M rows. MI355X design:
//  * Gw "worker" workgroups (one per CU) own contiguous row blocks of the
//    panel and keep them in LDS, row-major with an odd row stride, for the
//    whole factorization: the panel is read from HBM once and written once;
//  * one grid-wide reduction per column. Round j applies reflector j-1 to
//    the owned rows and, in the same pass over the data, produces every sum
//    the next step needs: the Gram row x^T a_c of the new column x with all
//    later columns (giving ||x||^2 and, once beta is known, all of
//    w = v_j^T A without a second reduction, since v_j = e_j + x/(alpha-beta)),
//    the dot products v_{j-1}^T v_l for column j-1 of Tf, and the owner's
//    copy of row j. Threads are laid out one (or a few) per column, so the
//    sums need no cross-lane reductions;
//  * each worker publishes its partial sums in its slot of a ring of global
//    buffers with device-coherent (write-through) stores, waits for their
//    completion and raises its own flag (one 64-byte line per workgroup);
//    the others poll the flags with a bounded spin and read the slots with
//    device-coherent loads. No cache-wide write-back or invalidation and no
//    contended atomic counter sits between two columns;
//  * every workgroup sums the slots in the same fixed order, spread over all
//    of its threads with the loads in flight together, so all compute
//    bit-identical scalars and results are reproducible run to run;
//  * one extra "coordinator" workgroup owns no rows: it keeps Tf in LDS,
//    builds column j-1 by the forward recurrence
//    Tf(1:j-1, j) = -tau_j Tf(1:j-1, 1:j-1) W^T v_j and writes R, tau and Tf.
//    Workers wait for it only when they are about to reuse a ring buffer, so
//    it may trail them by up to kRing - 2 rounds;
//  * the launch is cooperative so that all workgroups are co-resident.
#include <hip/hip_cooperative_groups.h>

#include <algorithm>
#include <cstdlib>

#include "common.hpp"
#include "context.hpp"
#include "kernels.hpp"
#include "trace.hpp"

namespace rrf {

namespace {

constexpr int kThreads = 512;
constexpr int kMaxCols = 256;
// Widest panel one cooperative launch takes; wider ones are split by columns.
// Each column costs one grid-wide exchange whose partial sums grow with k and
// whose workgroup count grows as the LDS rows per workgroup shrink: at
// M = 16384 a 256-column launch takes 4.9 ms, two 128-column halves with the
// split's GEMMs about 3 ms, while 128 columns in one launch (1.2 ms) beat two
// halves of 64 (1.3 ms).
constexpr int kLaunchCols = 128;
constexpr int64_t kLdsBudget = 140 * 1024;  // dynamic LDS bytes per workgroup
constexpr int kMaxGroups = 256;
constexpr int kRing = 4;                     // slot buffers in flight
constexpr int kFlagStride = 16;              // unsigned per flag: one 64-byte line
constexpr long kSpinLimit = 1L << 22;

struct PanelArgs {
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
  double* red;        // kRing * Gw * slot doubles
  unsigned* flags;    // (Gw + 1) * kFlagStride, zero at launch
  int* status;
  const int* cond;    // when not null: return at once unless *cond != 0
  int Gw;             // worker workgroups; workgroup Gw is the coordinator
  int rows_per;
  int ldl;            // LDS row stride of the row block (k + 1)
  int slot;           // doubles per slot: Gram row, row j, Tf dots (3k, padded)
  int tf_in_lds;      // coordinator keeps Tf in LDS
};

__device__ inline int clampi(int64_t v, int lo, int hi) {
  return (int)(v < lo ? lo : (v > hi ? hi : v));
}

// Device-coherent accesses: written through to, and read from, the level
// that all XCDs share.
__device__ inline void st_dev(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline double ld_dev(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Announce round `epoch` (after this workgroup's slot stores are complete)
// and wait until every worker has announced it and, when coord_epoch > 0, the
// coordinator has announced coord_epoch. Returns false (status bit 4) when a
// spin limit is hit or another workgroup has flagged an error.
__device__ bool announce_and_wait(const PanelArgs& a, unsigned epoch, bool wait,
                                  unsigned coord_epoch) {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  const int tid = threadIdx.x;
  if (tid == 0)
    __hip_atomic_store(a.flags + (size_t)kFlagStride * blockIdx.x, epoch, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  if (!wait) return true;
  int good = 1;
  const int nwait = a.Gw + (coord_epoch > 0 ? 1 : 0);
  if (tid < nwait) {
    const unsigned target = (tid < a.Gw) ? epoch : coord_epoch;
    const unsigned* f = a.flags + (size_t)kFlagStride * tid;
    long spins = 0;
    while (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
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

// Sums over the worker slots: dst[e] = sum_g slot_g[off + e], e < n, in one
// fixed order that depends on n and Gw only, so every workgroup gets
// identical sums. Virtual thread vt takes entry vt % sp (sp = n rounded up
// to a power of two) over the (vt / sp)-th of tpe = kThreads / sp ranges of
// workers, with its loads in flight together; slot_combine adds the tpe
// partials of an entry in range order.
__device__ inline int pow2_at_least(int n) {
  int sp = 1;
  while (sp < n) sp <<= 1;
  return sp;
}

__device__ double slot_partial(const double* base, int slot, int Gw, int off, int n, int vt) {
  const int sp = pow2_at_least(n);
  const int tpe = kThreads / sp;
  const int e = vt % sp, p = vt / sp;
  double acc = 0.0;
  if (e < n) {
    const int g0 = (int)((int64_t)Gw * p / tpe), g1 = (int)((int64_t)Gw * (p + 1) / tpe);
    for (int gb = g0; gb < g1; gb += 32) {
      double v[32];
#pragma unroll
      for (int u = 0; u < 32; ++u)
        v[u] = (gb + u < g1) ? ld_dev(base + (size_t)(gb + u) * slot + off + e) : 0.0;
#pragma unroll
      for (int u = 0; u < 32; ++u) acc += v[u];
    }
  }
  return acc;
}

__device__ inline double slot_combine(int n, int e, const double* part) {
  const int sp = pow2_at_least(n);
  const int tpe = kThreads / sp;
  double s = 0.0;
  for (int u = 0; u < tpe; ++u) s += part[e + u * sp];
  return s;
}

__global__ __launch_bounds__(kThreads) void panel_kernel(PanelArgs a) {
  extern __shared__ double smem[];
  __shared__ double red_s[3 * kMaxCols];
  __shared__ double w_s[kMaxCols];
  __shared__ double part[kThreads];
  __shared__ double part2[kThreads];

  // the same value for every workgroup (written by an earlier launch)
  if (a.cond != nullptr &&
      __hip_atomic_load(const_cast<int*>(a.cond), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
    return;
  const int tid = threadIdx.x;
  const int g = blockIdx.x;
  const bool coord = (g == a.Gw);
  const int k = a.k;
  const int RP = a.rows_per;
  const int L = a.ldl;
  const int64_t r0 = (int64_t)g * RP;
  const int rows = coord ? 0 : (int)((a.M - r0) < RP ? (a.M - r0) : RP);
  double* Ls = smem;  // workers: rows x k (+ zero row, spare column k), stride L
  double* Tl = a.tf_in_lds ? smem : nullptr;  // coordinator: k x k, ld k

  if (!coord) {
    for (int idx = tid; idx < rows * k; idx += kThreads) {
      const int rl = idx % rows, c = idx / rows;
      Ls[rl * L + c] = a.P[(r0 + rl) + (int64_t)c * a.ldp];
    }
    for (int c = tid; c < L; c += kThreads) Ls[rows * L + c] = 0.0;  // zero row
    __syncthreads();
    if (a.zero) {
      for (int idx = tid; idx < rows * k; idx += kThreads) {
        const int rl = idx % rows, c = idx / rows;
        a.zero[(r0 + rl) + (int64_t)c * a.ldz] = 0.0;
      }
    }
  }

  double tau_prev = 0.0;
  for (int j = 0; j <= k; ++j) {
    const int ns = (j < k) ? (k - j) : 0;   // Gram entries s_c, c in [j, k)
    const int nt = (j >= 2) ? (j - 1) : 0;  // Tf dots v_{j-1}^T v_l, l in [0, j-1)
    const unsigned epoch = (unsigned)j + 1;
    const int owner = (j < k) ? (int)(j / RP) : -1;  // worker holding row j
    double* ring = a.red + (size_t)(j % kRing) * a.Gw * a.slot;
    if (!coord) {
      double* slot = ring + (size_t)g * a.slot;
      const int rlj = clampi((int64_t)j - r0, 0, rows);  // first local row >= j
      const int rjl = (g == owner) ? (int)(j - r0) : -1;  // local index of row j
      const double twj = (j >= 1 && j < k) ? tau_prev * w_s[j] : 0.0;
      // (b) one pass over the rows >= j. Lane ci < ns owns column c = j + ci:
      // it applies H_{j-1} (columns c > j; the lane of column j writes into
      // the spare column k, its update is stored in (c)) and accumulates the
      // Gram partial x^T a_c with x = column j below row j after H_{j-1},
      // recomputed on the fly. Lane ci >= ns owns column l = ci - ns < j - 1
      // and accumulates v_{j-1}^T v_l (tw = 0 rewrites the column unchanged).
      // Both kinds run one instruction stream; consecutive lanes take
      // consecutive columns of a row, and tpc lanes share a column over
      // interleaved rows. Rows past the block read and write the zero row.
      const int nc = ns + nt;
      const int ncp = pow2_at_least(nc);
      const int tpc = kThreads / ncp;  // >= 1
      const int ci = tid % ncp, sub = tid / ncp;
      const int jm = (j >= 1) ? j - 1 : 0;
      double acc = 0.0;
      if (ci < nc) {
        const bool gram = ci < ns;
        const int col = gram ? j + ci : ci - ns;
        const int cst = (gram && col == j) ? k : col;
        const double tw = (gram && j >= 1) ? tau_prev * w_s[col] : 0.0;
        // row j-1 of v_{j-1} is the implicit 1
        if (!gram && sub == 0 && (int64_t)j - 1 >= r0 && (int64_t)j - 1 < r0 + rows)
          acc = Ls[(int)(j - 1 - r0) * L + col];
        constexpr int U = 4;
        const int nit = (rows - rlj + U * tpc - 1) / (U * tpc);
        for (int it = 0; it < nit; ++it) {
          const int rb = rlj + sub + it * U * tpc;
          double vv[U], xo[U], yo[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int r = min(rb + u * tpc, rows);
            vv[u] = Ls[r * L + jm];
            xo[u] = Ls[r * L + j];
            yo[u] = Ls[r * L + col];
          }
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int r = min(rb + u * tpc, rows);
            const double y = yo[u] - tw * vv[u];
            Ls[r * L + cst] = y;
            // Gram: x_r (0 on row j itself); Tf dots: v_{j-1}[r]
            const double xj = (r == rjl) ? 0.0 : xo[u] - twj * vv[u];
            acc += (gram ? xj : vv[u]) * y;
          }
        }
      }
      part[tid] = acc;
      __syncthreads();
      // (c) publish: partial sums, row j of the panel (its owner), and column
      // j of H_{j-1} A into LDS.
      if (tid < nc) {
        const double s = slot_combine(nc, tid, part);
        st_dev(slot + ((tid < ns) ? j + tid : 2 * k + (tid - ns)), s);
      }
      if (j < k) {
        if (rjl >= 0)
          for (int c = j + 1 + tid; c < k; c += kThreads) st_dev(slot + k + c, Ls[rjl * L + c]);
        for (int rl = rlj + tid; rl < rows; rl += kThreads) {
          double x = Ls[rl * L + j];
          if (j >= 1) {
            x -= twj * Ls[rl * L + j - 1];
            Ls[rl * L + j] = x;
          }
          if (rl == rjl) st_dev(slot + k + j, x);
        }
      }
      // the last round only feeds the coordinator
      const unsigned ce = (epoch + 2 > (unsigned)kRing) ? epoch + 2 - kRing : 0u;
      if (!announce_and_wait(a, epoch, j < k, ce)) return;
      if (j == k) break;
      // (d) Gram sums and row j, the same order in every workgroup.
      if (tid < ns) red_s[k + j + tid] = ld_dev(ring + (size_t)owner * a.slot + k + j + tid);
      part[tid] = slot_partial(ring, a.slot, a.Gw, j, ns, tid);
      __syncthreads();
      if (tid < ns) red_s[j + tid] = slot_combine(ns, tid, part);
      __syncthreads();
    } else {
      if (!announce_and_wait(a, epoch, true, 0u)) return;
      // (d) the coordinator needs s_j and alpha (for tau_j) and the Tf dots.
      // s_j is summed by the workers' own split of entry 0, so it is
      // bit-identical to theirs.
      const int spg = pow2_at_least(ns);
      if (ns > 0 && tid == 0) red_s[k + j] = ld_dev(ring + (size_t)owner * a.slot + k + j);
      if (ns > 0 && tid < kThreads / spg) part[tid] = slot_partial(ring, a.slot, a.Gw, j, ns, tid * spg);
      part2[tid] = (nt > 0) ? slot_partial(ring, a.slot, a.Gw, 2 * k, nt, tid) : 0.0;
      __syncthreads();
      if (ns > 0 && tid == 0) {
        double sj = 0.0;
        for (int u = 0; u < kThreads / spg; ++u) sj += part[u];
        red_s[j] = sj;
      }
      if (tid < nt) red_s[2 * k + tid] = slot_combine(nt, tid, part2);
      __syncthreads();
      // (e) column j-1 of Tf: Tf(i, j-1) = -tau_{j-1} sum_{c=i}^{j-2} Tf(i, c)
      // dots_c, each dot split over tpi threads and added in range order.
      if (j >= 1) {
        const int jj = j - 1;
        const double* dots = red_s + 2 * k;
        if (jj > 0) {
          const int sp = pow2_at_least(jj);
          const int tpi = kThreads / sp;
          const int i = tid % sp, pi = tid / sp;
          double s = 0.0;
          if (i < jj) {
            const int len = jj - i;
            const int c0 = i + len * pi / tpi, c1 = i + len * (pi + 1) / tpi;
            if (Tl) {
              for (int c = c0; c < c1; ++c) s += Tl[i + c * k] * dots[c];
            } else {
              for (int c = c0; c < c1; ++c) s += a.Tf[i + (int64_t)c * a.ldt] * dots[c];
            }
          }
          part2[tid] = s;
          __syncthreads();
          if (tid < jj) {
            double v = 0.0;
            for (int u = 0; u < tpi; ++u) v += part2[tid + u * sp];
            v = -tau_prev * v;
            if (Tl) Tl[tid + jj * k] = v;
            else a.Tf[tid + (int64_t)jj * a.ldt] = v;
          }
        }
        if (tid == 0) {
          if (Tl) Tl[jj + jj * k] = tau_prev;
          else a.Tf[jj + (int64_t)jj * a.ldt] = tau_prev;
        }
      }
      if (j == k) break;
    }

    // (f) reflector j from alpha = row_j[j] and ||x||^2 = s_j (dlarfg rule);
    // the worker holding row j writes tau_j and row j of R.
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
    if (!coord) {
      const bool own = (g == owner);
      for (int c = j + 1 + tid; c < k; c += kThreads) {
        const double w = red_s[k + c] + scal * red_s[c];
        w_s[c] = w;
        if (own && a.R) a.R[j + (int64_t)c * a.ldr] = red_s[k + c] - tau * w;
      }
      if (own) {
        if (tid == 0) a.tau[j] = tau;
        if (a.R) {
          if (tid == 0) a.R[j + (int64_t)j * a.ldr] = beta;
          for (int i = j + 1 + tid; i < k; i += kThreads) a.R[i + (int64_t)j * a.ldr] = 0.0;
        }
      }
      const int rlx = clampi((int64_t)j + 1 - r0, 0, rows);
      for (int rl = rlx + tid; rl < rows; rl += kThreads) Ls[rl * L + j] *= scal;
    }
    tau_prev = tau;
    __syncthreads();
  }

  __syncthreads();  // the last column of Tf (round k) is complete
  if (coord) {
    // Tf (upper triangular, zero below) to global
    for (int idx = tid; idx < k * k; idx += kThreads) {
      const int i = idx % k, c = idx / k;
      double v = 0.0;
      if (i <= c) v = Tl ? Tl[i + c * k] : a.Tf[i + (int64_t)c * a.ldt];
      a.Tf[i + (int64_t)c * a.ldt] = v;
    }
    return;
  }
  // Explicit unit lower trapezoidal W.
  for (int idx = tid; idx < rows * k; idx += kThreads) {
    const int rl = idx % rows, c = idx / rows;
    const int64_t r = r0 + rl;
    const double v = (r < c) ? 0.0 : (r == c ? 1.0 : Ls[rl * L + c]);
    a.W[r + (int64_t)c * a.ldw] = v;
  }
}

size_t flag_bytes(int Gw) { return (size_t)round_up((int64_t)(Gw + 1) * kFlagStride * 4, 256); }
int slot_doubles(int k) { return (int)round_up((int64_t)3 * k, 32); }

}  // namespace

bool panel_plan(int64_t M, int k, PanelPlan* plan) {
  if (k < 1 || k > kMaxCols || M < k) return false;
  const int64_t L = k + 1;
  const int64_t max_rows = kLdsBudget / (L * 8) - 1;  // one zero row follows the block
  int64_t Gw = ceil_div(M, max_rows);
  if (Gw + 1 > kMaxGroups) return false;
  const int64_t rp = ceil_div(M, Gw);
  Gw = ceil_div(M, rp);
  const bool tf_lds = (int64_t)k * k * 8 <= kLdsBudget;
  plan->G = (int)Gw;
  plan->rows_per = (int)rp;
  plan->lds = (size_t)std::max<int64_t>((rp + 1) * L, tf_lds ? (int64_t)k * k : 0) * 8;
  plan->work = flag_bytes((int)Gw) + (size_t)kRing * Gw * slot_doubles(k) * 8;
  return true;
}

namespace {

int panel_launch(hipStream_t st, int64_t M, int k, const double* P, int64_t ldp, double* W,
                 int64_t ldw, double* R, int64_t ldr, double* Tf, int64_t ldt, double* tau,
                 double* zero, int64_t ldz, void* work, size_t work_bytes, int* status) {
  return panel_launch_if(st, M, k, P, ldp, W, ldw, R, ldr, Tf, ldt, tau, zero, ldz, work,
                         work_bytes, status, nullptr);
}

}  // namespace

// One cooperative launch; the panel must satisfy panel_plan.
int panel_launch_if(hipStream_t st, int64_t M, int k, const double* P, int64_t ldp, double* W,
                    int64_t ldw, double* R, int64_t ldr, double* Tf, int64_t ldt, double* tau,
                    double* zero, int64_t ldz, void* work, size_t work_bytes, int* status,
                    const int* cond) {
  PanelPlan plan;
  if (!panel_plan(M, k, &plan))
    return set_error(RRF_E_NOTSUP, "householder panel: needs 1 <= k <= 256, M >= k and the panel "
                                   "within the LDS of 255 workgroups");
  if (work_bytes < plan.work || work == nullptr)
    return set_error(RRF_E_NOMEM, "householder panel: workspace too small");
  RRF_TRY(allow_dynamic_lds((const void*)panel_kernel, kLdsBudget));
  unsigned* flags = reinterpret_cast<unsigned*>(work);
  PanelArgs a{};
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
  a.red = reinterpret_cast<double*>(reinterpret_cast<char*>(work) + flag_bytes(plan.G));
  a.flags = flags;
  a.status = status;
  a.cond = cond;
  a.Gw = plan.G;
  a.rows_per = plan.rows_per;
  a.ldl = k + 1;
  a.slot = slot_doubles(k);
  a.tf_in_lds = ((int64_t)k * k * 8 <= kLdsBudget) ? 1 : 0;
  // Algorithmic traffic: the panel read once, W written, and the in-place
  // clear of the source panel when requested.
  const double pbytes = 8.0 * (double)M * k * (zero ? 3.0 : 2.0);
  const double pflops = 2.0 * (double)M * k * k;
  RRF_TRY(fill_u32(st, flags, (int64_t)(plan.G + 1) * kFlagStride, 0u));
  void* args[] = {&a};
  int tok = cond ? trace_begin(st, kTrPanelFallback, 0.0, 0.0) : trace_begin(st, kTrPanel, pflops, pbytes);
  hipError_t e = hipLaunchCooperativeKernel((const void*)panel_kernel, dim3(plan.G + 1),
                                            dim3(kThreads), args, (unsigned)plan.lds, st);
  trace_end(st, tok);
  RRF_CHECK_HIP(e);
  return RRF_OK;
}

namespace {

// Largest panel height one launch takes for k columns (0 if none).
int64_t fit_rows(int k) {
  const int64_t max_rows = kLdsBudget / ((int64_t)(k + 1) * 8) - 1;
  return max_rows < 1 ? 0 : max_rows * (kMaxGroups - 1);
}

// Scratch of the split below: Z, T1^T Z and W1^T W2 (k1 x k2 each) and the
// split-K partials of the GEMMs with inner dimension M.
constexpr int kSplitParts = 16;
size_t split_temp_bytes(int k1, int k2) { return (size_t)(3 + kSplitParts) * k1 * k2 * 8; }

// With RRF_PANEL_TREE=1 in the environment the tree panel (panel_tsqr.hip)
// takes every panel of at most kTreeCols columns it can, and wider ones are
// split by columns into halves it takes. It is not the default: measured on
// MI355X it is about half as fast as the kernel above (16384 x 64: 1.0 ms
// against 0.57 ms), its serial chain of one-workgroup QRs (a leaf and one
// node per tree level, about 1 us per column each) and its LDS-bound small
// products costing more than the grid exchanges it removes.
constexpr int kTreeCols = 64;

bool tree_enabled() {
  const char* e = getenv("RRF_PANEL_TREE");
  return e && e[0] == '1';
}

}  // namespace

size_t panel_work_bytes(int64_t Mmax, int k) {
  if (k < 1 || k > kMaxCols || Mmax < k) return 0;
  // every path some M <= Mmax may take, in any mode
  size_t need = tsqr_work_bytes(Mmax, k);
  const int64_t fit = k <= kLaunchCols ? fit_rows(k) : 0;
  if (fit >= k) {
    PanelPlan p;
    if (panel_plan(std::min(Mmax, fit), k, &p)) need = std::max(need, p.work);
  }
  if (Mmax > fit || k > kTreeCols) {
    if (k < 2) return need;
    const int k1 = k / 2, k2 = k - k1;
    const size_t a = panel_work_bytes(Mmax, k1), b = panel_work_bytes(Mmax - k1, k2);
    if (a == 0 || b == 0) return Mmax > fit ? 0 : need;
    need = std::max(need, (size_t)round_up((int64_t)std::max(a, b), 256) + split_temp_bytes(k1, k2));
  }
  // CholeskyQR: its flag, then either its buffers or the fallback's workspace
  const size_t cq = cholqr_work_bytes(Mmax, k);
  if (cq) need = std::max(need + 256, cq);
  return need;
}

// A panel taller than one launch takes is split by columns (recursive
// blocked Householder QR): with P = [P1 P2], P1 = Q1 [R11; 0] with
// Q1 = I - W1 T1 W1^T, then Q1^T P2 = [R12; P2'] and P2' = Q2' R22, and
// Q = Q1 Q2 = I - W T W^T with W = [W1, [0; W2']] and
// T = [T1, -T1 (W1^T W2) T2; 0, T2]. In exact arithmetic these are the
// reflectors of the unblocked factorization.
int householder_panel(hipStream_t st, int64_t M, int k, const double* P, int64_t ldp, double* W,
                      int64_t ldw, double* R, int64_t ldr, double* Tf, int64_t ldt, double* tau,
                      double* zero, int64_t ldz, void* work, size_t work_bytes, int* status) {
  const bool tree = tree_enabled();
  PanelPlan plan;
  if (!tree && cholqr_enabled() && cholqr_panel_ok(M, k, P, ldp, W, ldw) &&
      panel_plan(M, k, &plan))
    return cholqr_panel(st, M, k, P, ldp, W, ldw, R, ldr, Tf, ldt, tau, zero, ldz, work,
                        work_bytes, status);
  if (tree && tsqr_panel_ok(M, k))
    return tsqr_panel(st, M, k, P, ldp, W, ldw, R, ldr, Tf, ldt, tau, zero, ldz, work,
                      work_bytes, status);
  const bool split_for_tree = tree && k > kTreeCols && tsqr_panel_ok(M - k / 2, k - k / 2);
  if (!split_for_tree && k <= kLaunchCols && panel_plan(M, k, &plan))
    return panel_launch(st, M, k, P, ldp, W, ldw, R, ldr, Tf, ldt, tau, zero, ldz, work,
                        work_bytes, status);
  if (k < 2 || M < k)
    return set_error(RRF_E_NOTSUP, "householder panel: shape not supported");
  const int k1 = k / 2, k2 = k - k1;
  const size_t sub = std::max(panel_work_bytes(M, k1), panel_work_bytes(M - k1, k2));
  if (sub == 0) return set_error(RRF_E_NOTSUP, "householder panel: shape not supported");
  const size_t sub_r = (size_t)round_up((int64_t)sub, 256);
  if (work == nullptr || work_bytes < sub_r + split_temp_bytes(k1, k2))
    return set_error(RRF_E_NOMEM, "householder panel: workspace too small");
  double* Z = reinterpret_cast<double*>(reinterpret_cast<char*>(work) + sub_r);
  double* Z2 = Z + (size_t)k1 * k2;
  double* S = Z2 + (size_t)k1 * k2;
  double* split = S + (size_t)k1 * k2;
  const size_t split_elems = (size_t)kSplitParts * k1 * k2;

  // P1 = Q1 [R11; 0]
  RRF_TRY(householder_panel(st, M, k1, P, ldp, W, ldw, R, ldr, Tf, ldt, tau, zero, ldz, work, sub,
                            status));
  // W2 <- Q1^T P2 = P2 - W1 (T1^T (W1^T P2)), then R12 = its first k1 rows
  double* W2 = W + (int64_t)k1 * ldw;
  if (W != P || ldw != ldp) RRF_TRY(copy_matrix(st, M, k2, P + (int64_t)k1 * ldp, ldp, W2, ldw));
  if (zero) RRF_TRY(fill_matrix(st, M, k2, 0.0, zero + (int64_t)k1 * ldz, ldz));
  RRF_TRY(dgemm(st, true, false, k1, k2, M, 1.0, W, ldw, W2, ldw, 0.0, Z, k1, split, split_elems));
  RRF_TRY(dgemm(st, true, false, k1, k2, k1, 1.0, Tf, ldt, Z, k1, 0.0, Z2, k1, nullptr, 0));
  RRF_TRY(dgemm(st, false, false, M, k2, k1, -1.0, W, ldw, Z2, k1, 1.0, W2, ldw, nullptr, 0));
  if (R) {
    RRF_TRY(copy_matrix(st, k1, k2, W2, ldw, R + (int64_t)k1 * ldr, ldr));
    RRF_TRY(fill_matrix(st, k2, k1, 0.0, R + k1, ldr));
  }
  // P2' (rows k1.. of W2, in place) = Q2' R22
  RRF_TRY(householder_panel(st, M - k1, k2, W2 + k1, ldw, W2 + k1, ldw,
                            R ? R + k1 + (int64_t)k1 * ldr : nullptr, ldr,
                            Tf + k1 + (int64_t)k1 * ldt, ldt, tau + k1, nullptr, 0, work, sub,
                            status));
  RRF_TRY(fill_matrix(st, k1, k2, 0.0, W2, ldw));
  // T12 = -T1 (W1^T W2) T2
  RRF_TRY(dgemm(st, true, false, k1, k2, M, 1.0, W, ldw, W2, ldw, 0.0, S, k1, split, split_elems));
  RRF_TRY(dgemm(st, false, false, k1, k2, k1, 1.0, Tf, ldt, S, k1, 0.0, Z, k1, nullptr, 0));
  RRF_TRY(dgemm(st, false, false, k1, k2, k2, -1.0, Z, k1, Tf + k1 + (int64_t)k1 * ldt, ldt, 0.0,
                Tf + (int64_t)k1 * ldt, ldt, nullptr, 0));
  RRF_TRY(fill_matrix(st, k2, k1, 0.0, Tf + k1, ldt));
  return RRF_OK;
}

}  // namespace rrf
