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
//  * each worker publishes its partial sums in a slot of a double-buffered
//    global array and meets the others at a counter barrier (device-scope
//    release/acquire, bounded spin); every workgroup then sums the slots in a
//    fixed order, so all compute bit-identical scalars and results are
//    reproducible run to run;
//  * one extra "coordinator" workgroup owns no rows: it keeps Tf in LDS,
//    builds column j-1 by the forward recurrence
//    Tf(1:j-1, j) = -tau_j Tf(1:j-1, 1:j-1) W^T v_j while the workers move on,
//    and writes R, tau and Tf;
//  * the launch is cooperative so that all workgroups are co-resident.
#include <hip/hip_cooperative_groups.h>

#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"
#include "trace.hpp"

namespace rrf {

namespace {

constexpr int kThreads = 256;
constexpr int kMaxCols = 256;
constexpr int64_t kLdsBudget = 144 * 1024;  // dynamic LDS bytes per workgroup
constexpr int kMaxGroups = 256;
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
  double* red;        // 2 * Gw * slot doubles
  unsigned* counter;  // zero at launch
  int* status;
  int Gw;             // worker workgroups; workgroup Gw is the coordinator
  int rows_per;
  int ldr_lds;        // LDS row stride of the row block (k + 1)
  int slot;           // 3 * k
  int tf_in_lds;      // coordinator keeps Tf in LDS
};

__device__ inline int clampi(int64_t v, int lo, int hi) {
  return (int)(v < lo ? lo : (v > hi ? hi : v));
}

// Counter barrier across the workgroups of a cooperative launch.
// Returns false (and flags status) if the spin limit is hit.
__device__ bool grid_barrier(unsigned* counter, unsigned target, int* status) {
  __shared__ int ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    int good = 1;
    __threadfence();
    atomicAdd(counter, 1u);
    long spins = 0;
    while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > kSpinLimit ||
          __hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
        good = 0;
        atomicOr(status, 4);
        break;
      }
    }
    __threadfence();
    ok = good;
  }
  __syncthreads();
  return ok != 0;
}

// Sum of base[g * stride + idx] over g = 0..G-1 in a fixed association
// (eight interleaved partial sums, combined pairwise), loads unrolled.
__device__ inline double sum_slots(const double* base, size_t stride, int idx, int G) {
  double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int g = 0;
  for (; g + 8 <= G; g += 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) s[u] += base[(size_t)(g + u) * stride + idx];
  }
  for (int u = 0; g < G; ++g, ++u) s[u] += base[(size_t)g * stride + idx];
  return ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

__global__ __launch_bounds__(kThreads) void panel_kernel(PanelArgs a) {
  extern __shared__ double smem[];
  __shared__ double red_s[3 * kMaxCols];
  __shared__ double w_s[kMaxCols];
  __shared__ double part[kThreads];

  const int tid = threadIdx.x;
  const int g = blockIdx.x;
  const bool coord = (g == a.Gw);
  const int k = a.k;
  const int RP = a.rows_per;
  const int L = a.ldr_lds;
  const int64_t r0 = (int64_t)g * RP;
  const int rows = coord ? 0 : (int)((a.M - r0) < RP ? (a.M - r0) : RP);
  double* Ls = smem;                                  // workers: rows x k, stride L
  double* Tl = a.tf_in_lds ? smem : nullptr;          // coordinator: k x k, ld k
  const int G = a.Gw + 1;

  if (!coord) {
    for (int idx = tid; idx < rows * k; idx += kThreads) {
      const int rl = idx % rows, c = idx / rows;
      Ls[rl * L + c] = a.P[(r0 + rl) + (int64_t)c * a.ldp];
    }
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
    double* slot = a.red + ((size_t)(j & 1) * a.Gw + g) * a.slot;
    if (!coord) {
      // (a) column j of H_{j-1} applied to owned rows r >= j.
      const int rlj = clampi((int64_t)j - r0, 0, rows);      // first local row >= j
      if (j >= 1 && j < k && tau_prev != 0.0) {
        const double wj = tau_prev * w_s[j];
        for (int rl = rlj + tid; rl < rows; rl += kThreads)
          Ls[rl * L + j] -= wj * Ls[rl * L + j - 1];
      }
      __syncthreads();
      // (b) one pass over the columns: update the rest of H_{j-1} and form
      // this workgroup's partial sums. Consecutive threads take consecutive
      // columns of a row; tpc threads share a column over interleaved rows.
      const int nc = ns + nt;
      if (nc > 0) {
        int ncp = 1;
        while (ncp < nc) ncp <<= 1;
        const int tpc = kThreads / ncp;  // >= 1
        const int ci = tid % ncp, sub = tid / ncp;
        double acc = 0.0;
        if (ci < nc) {
          if (ci < ns) {
            const int c = j + ci;
            const double tw = (j >= 1 && tau_prev != 0.0) ? tau_prev * w_s[c] : 0.0;
            const int rlx = clampi((int64_t)j + 1 - r0, 0, rows);  // first local row > j
            for (int rl = rlj + sub; rl < rows; rl += tpc) {
              double y = Ls[rl * L + c];
              if (c > j && tw != 0.0) {
                y -= tw * Ls[rl * L + j - 1];
                Ls[rl * L + c] = y;
              }
              if (rl >= rlx) acc += Ls[rl * L + j] * y;
            }
          } else {
            const int l = ci - ns;
            const int rlv = clampi((int64_t)j - 1 - r0, 0, rows);
            for (int rl = rlv + sub; rl < rows; rl += tpc) {
              const double vv = (r0 + rl == j - 1) ? 1.0 : Ls[rl * L + j - 1];
              acc += vv * Ls[rl * L + l];
            }
          }
        }
        part[tid] = acc;
        __syncthreads();
        if (tid < nc) {
          double s = 0.0;
          for (int u = 0; u < tpc; ++u) s += part[tid + u * ncp];
          if (tid < ns) slot[j + tid] = s;
          else slot[2 * k + (tid - ns)] = s;
        }
      }
      // (c) the owner of row j publishes it (after the updates of (b))
      __syncthreads();
      if (j < k && (int64_t)j >= r0 && (int64_t)j < r0 + rows) {
        const int rl = (int)(j - r0);
        for (int c = j + tid; c < k; c += kThreads) slot[k + c] = Ls[rl * L + c];
      }
    }

    if (G > 1) {
      if (!grid_barrier(a.counter, (unsigned)(j + 1) * (unsigned)G, a.status)) return;
    } else {
      __syncthreads();
    }

    // (d) sum the worker slots in a fixed order (every workgroup alike).
    {
      const double* base = a.red + (size_t)(j & 1) * a.Gw * a.slot;
      const int owner = (j < k) ? (int)(j / RP) : 0;
      const int ne = 2 * ns + nt;
      for (int e = tid; e < ne; e += kThreads) {
        int idx;
        double v;
        if (e < ns) {
          idx = j + e;
          v = sum_slots(base, a.slot, idx, a.Gw);
        } else if (e < 2 * ns) {
          idx = k + j + (e - ns);
          v = base[(size_t)owner * a.slot + idx];
        } else {
          idx = 2 * k + (e - 2 * ns);
          v = sum_slots(base, a.slot, idx, a.Gw);
        }
        red_s[idx] = v;
      }
    }
    __syncthreads();

    // (e) coordinator: column j-1 of Tf.
    if (coord && j >= 1) {
      const int jj = j - 1;
      for (int i = tid; i < jj; i += kThreads) {
        double s = 0.0;
        if (Tl) {
          for (int c = i; c < jj; ++c) s += Tl[i + c * k] * red_s[2 * k + c];
        } else {
          for (int c = i; c < jj; ++c) s += a.Tf[i + (int64_t)c * a.ldt] * red_s[2 * k + c];
        }
        const double v = -tau_prev * s;
        if (Tl) Tl[i + jj * k] = v;
        else a.Tf[i + (int64_t)jj * a.ldt] = v;
      }
      if (tid == 0) {
        if (Tl) Tl[jj + jj * k] = tau_prev;
        else a.Tf[jj + (int64_t)jj * a.ldt] = tau_prev;
      }
    }
    if (j == k) break;

    // (f) reflector j from alpha = row_j[j] and ||x||^2 = s_j (dlarfg rule).
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
    for (int c = j + 1 + tid; c < k; c += kThreads) w_s[c] = red_s[k + c] + scal * red_s[c];
    __syncthreads();
    if (coord) {
      if (tid == 0) a.tau[j] = tau;
      if (a.R) {
        if (tid == 0) a.R[j + (int64_t)j * a.ldr] = beta;
        for (int c = j + 1 + tid; c < k; c += kThreads)
          a.R[j + (int64_t)c * a.ldr] = red_s[k + c] - tau * w_s[c];
        for (int i = j + 1 + tid; i < k; i += kThreads) a.R[i + (int64_t)j * a.ldr] = 0.0;
      }
    } else {
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

bool g_attr_set = false;

}  // namespace

bool panel_plan(int64_t M, int k, PanelPlan* plan) {
  if (k < 1 || k > kMaxCols || M < k) return false;
  const int64_t L = k + 1;
  const int64_t max_rows = kLdsBudget / (L * 8);
  int64_t Gw = ceil_div(M, max_rows);
  if (Gw + 1 > kMaxGroups) return false;
  const int64_t rp = ceil_div(M, Gw);
  Gw = ceil_div(M, rp);
  const bool tf_lds = (int64_t)k * k * 8 <= kLdsBudget;
  plan->G = (int)Gw;
  plan->rows_per = (int)rp;
  plan->lds = (size_t)std::max<int64_t>(rp * L, tf_lds ? (int64_t)k * k : 0) * 8;
  plan->work = 256 + (size_t)2 * Gw * 3 * k * 8;
  return true;
}

int householder_panel(hipStream_t st, int64_t M, int k, const double* P, int64_t ldp, double* W,
                      int64_t ldw, double* R, int64_t ldr, double* Tf, int64_t ldt, double* tau,
                      double* zero, int64_t ldz, void* work, size_t work_bytes, int* status) {
  PanelPlan plan;
  if (!panel_plan(M, k, &plan))
    return set_error(RRF_E_NOTSUP, "householder panel: shape outside 1 <= k <= 256, M >= k, "
                                   "M (k + 1) <= 255 * 18432");
  if (work_bytes < plan.work || work == nullptr)
    return set_error(RRF_E_NOMEM, "householder panel: workspace too small");
  if (!g_attr_set) {
    RRF_CHECK_HIP(hipFuncSetAttribute((const void*)panel_kernel,
                                      hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)kLdsBudget));
    g_attr_set = true;
  }
  unsigned* counter = reinterpret_cast<unsigned*>(work);
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
  a.red = reinterpret_cast<double*>(reinterpret_cast<char*>(work) + 256);
  a.counter = counter;
  a.status = status;
  a.Gw = plan.G;
  a.rows_per = plan.rows_per;
  a.ldr_lds = k + 1;
  a.slot = 3 * k;
  a.tf_in_lds = ((int64_t)k * k * 8 <= kLdsBudget) ? 1 : 0;
  // Algorithmic traffic: the panel read once, W written, and the in-place
  // clear of the source panel when requested.
  const double pbytes = 8.0 * (double)M * k * (zero ? 3.0 : 2.0);
  const double pflops = 2.0 * (double)M * k * k;
  RRF_TRY(fill_u32(st, counter, 1, 0u));
  void* args[] = {&a};
  int tok = trace_begin(st, kTrPanel, pflops, pbytes);
  hipError_t e = hipLaunchCooperativeKernel((const void*)panel_kernel, dim3(plan.G + 1),
                                            dim3(kThreads), args, (unsigned)plan.lds, st);
  trace_end(st, tok);
  RRF_CHECK_HIP(e);
  return RRF_OK;
}

}  // namespace rrf
