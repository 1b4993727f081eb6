// Batched randUTV: Alg. 3 on many small matrices of one block size b, the
// same step of every matrix issued together.
//
// Each round of launches carries one stage of step i for all matrices that
// still have that step (grouped GEMMs, one-workgroup panels, batched
// generator and elementwise kernels of batched.hip), so a batch of thousands
// of matrices costs a few hundred launches. The arithmetic per matrix is
// that of randutv.hip: the sketch Y = (T22^T T22)^q T22^T G_i, the panel of
// Y (V_i), X = T(:, J2uJ3) W_v with the columns J2 of T V_i, the panel of
// T(I2uI3, J2) (U_i, R), the fused rank-2b update of T(:, J3); afterwards
// every small SVD in one launch, the block updates of T, and U and V formed
// backward from each matrix's kept reflectors in groups of four steps.
// Panels taller than one workgroup's LDS holds are split by columns (the
// merge of two compact-WY factors, as in householder_panel).
//
// Descriptors of a round are built on the host in pinned memory and copied
// to the device on the stream that runs the round; a ring of slots lets the
// host build the next rounds while the device runs the earlier ones. Large
// batches are cut into up to four slices of about equal work, each driven by
// its own host thread on its own stream, ordered after the caller's stream
// and before its later work: one slice's latency-bound launches (panels,
// small SVDs) overlap another's GEMMs.
#include <algorithm>
#include <climits>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "batched.hpp"
#include "common.hpp"
#include "context.hpp"
#include "driver.hpp"
#include "kernels.hpp"
#include "trace.hpp"

namespace rrf {

namespace {

constexpr int kBGroup = 4;            // steps merged per backward application

// Tunable choices of the plan (set per building thread from the call's
// configuration, see BatchedCfg): the grouped GEMM's allowed tile shapes (a
// bit mask over GemmTile) and the widest panel one launch factors before the
// column split takes over (0: as wide as one workgroup holds).
static_assert(kTileMaskAll == (1 << kGemmTiles) - 1, "every tile shape");
thread_local int t_tile_mask = kTileMaskAll;
thread_local int t_panel_leaf = 0;
constexpr int kSlots = 4;             // descriptor ring
constexpr size_t kDescPerMat = 2048;  // descriptor bytes per matrix and round (bound)

// Per-matrix views into the workspace.
struct Mat {
  int64_t m, n, s;
  const double* A;
  int64_t lda;
  double *U, *T, *V;
  uint64_t seed;
  double *G, *Y, *Z, *XW, *WZ, *S, *X0, *Zl, *WU, *WV, *TU, *TV, *tau, *pt;
  double *TG, *Sx, *Sy, *Zg, *Z2;
  int64_t blk0;  // index of this matrix's first block in the shared R/Us/Vs/d
  // mixed sketch: bfloat16 copies of T22 (and transposed), G, Y, Z (ld a
  // multiple of 8), FP32 products, the max|T22| word
  uint16_t *Tb, *Tbt, *Gb, *Yb, *Zb;
  float* Pf;
  unsigned long long* word;
};

// One round: descriptors packed in `bytes`, launches in `ops` order.
struct Plan {
  enum { kGemm, kElem, kGauss, kPanel, kMax, kBf16, kGemm16, kRound, kCopyIn, kCall };
  struct Op {
    int kind;
    bool ta, tb;
    size_t off;
    int count;
    int64_t aux;
    int k;  // panel width, or the GEMM tile shape
    double flops;
    size_t off2;  // GEMM: running tile counts
    bool vec;     // GEMM: 16-byte loads
    void* dst = nullptr;                    // kCopyIn: aux bytes at off go to dst
    std::function<int(hipStream_t)> fn{};  // kCall: a launch that takes no descriptors
  };
  std::vector<unsigned char> bytes;
  std::vector<Op> ops;

  template <class D>
  size_t put(const std::vector<D>& v) {
    const size_t off = (bytes.size() + 15) & ~(size_t)15;
    bytes.resize(off + v.size() * sizeof(D));
    memcpy(bytes.data() + off, v.data(), v.size() * sizeof(D));
    return off;
  }
  // The tile shape with the least padded work, weighted by how well each
  // shape keeps the matrix cores fed (wider tiles reuse each loaded slice
  // more often).
  // Among the tile shapes the plan allows (64 x 64 always), the one with the
  // least padded work, weighted by how well each shape keeps the matrix cores
  // fed (wider tiles reuse each loaded slice more often).
  static int pick_tile(const std::vector<GemmDesc>& v) {
    static const int order[5] = {kTile128x128, kTile128x64, kTile64x64, kTile128x32, kTile128x16};
    static const double weight[5] = {1.0, 1.1, 1.3, 1.25, 1.5};
    const int mask = t_tile_mask | (1 << kTile64x64);
    int best = kTile64x64;
    double best_cost = -1.0;
    for (int c = 0; c < 5; ++c) {
      const int t = order[c];
      if (!(mask & (1 << t))) continue;
      double area = 0.0;
      for (const auto& g : v)
        area += (double)tile_count(t, g.M, g.N) * tile_rows(t) * tile_cols(t) * (double)g.K;
      const double cost = area * weight[c];
      if (best_cost < 0.0 || cost < best_cost) {
        best = t;
        best_cost = cost;
      }
    }
    return best;
  }
  void gemm(bool ta, bool tb, const std::vector<GemmDesc>& v) {
    if (v.empty()) return;
    const int tile = pick_tile(v);
    std::vector<int> prefix(v.size() + 1, 0);
    double fl = 0.0;
    int64_t total = 0;
    for (size_t i = 0; i < v.size(); ++i) {
      total += tile_count(tile, v[i].M, v[i].N);
      prefix[i + 1] = (int)std::min<int64_t>(total, INT32_MAX);
      fl += 2.0 * v[i].M * v[i].N * v[i].K;
    }
    // 16-byte loads when every operand column starts 16-byte aligned
    bool vec = true;
    for (const auto& g : v)
      vec = vec && ((uintptr_t)g.A % 16 == 0) && ((uintptr_t)g.B % 16 == 0) && g.lda % 2 == 0 &&
            g.ldb % 2 == 0;
    const size_t off = put(v);
    ops.push_back({kGemm, ta, tb, off, (int)v.size(), total, tile, fl, put(prefix), vec});
  }
  void elem(const std::vector<ElemDesc>& v) {
    if (v.empty()) return;
    int64_t cols = 0;
    for (const auto& e : v) cols = std::max(cols, e.cols);
    ops.push_back({kElem, false, false, put(v), (int)v.size(), cols, 0, 0.0, 0, false});
  }
  void gauss(const std::vector<GaussDesc>& v) {
    if (v.empty()) return;
    int64_t el = 0;
    for (const auto& e : v) el = std::max(el, e.rows * e.cols);
    ops.push_back({kGauss, false, false, put(v), (int)v.size(), el, 0, 0.0, 0, false});
  }
  void maxabs(const std::vector<MaxDesc>& v) {
    if (v.empty()) return;
    int64_t rows = 0;
    for (const auto& e : v) rows = std::max(rows, e.rows);
    ops.push_back({kMax, false, false, put(v), (int)v.size(), rows, 0, 0.0, 0, false});
  }
  void bf16(const std::vector<Bf16Desc>& v) {
    if (v.empty()) return;
    int64_t tiles = 0;
    for (const auto& e : v)
      tiles = std::max(tiles, bf16_conv_tiles(e.rows, e.cols, e.ldo, e.outT ? e.ldot : 0));
    ops.push_back({kBf16, false, false, put(v), (int)v.size(), tiles, 0, 0.0, 0, false});
  }
  void gemm16(const std::vector<Bf16GemmDesc>& v) {
    if (v.empty()) return;
    std::vector<int> prefix(v.size() + 1, 0);
    double fl = 0.0;
    int64_t total = 0;
    for (size_t i = 0; i < v.size(); ++i) {
      total += bf16_group_tiles(v[i].M, v[i].N);
      prefix[i + 1] = (int)std::min<int64_t>(total, INT32_MAX);
      fl += 2.0 * v[i].M * v[i].N * v[i].K;
    }
    const size_t off = put(v);
    ops.push_back({kGemm16, false, false, off, (int)v.size(), total, 0, fl, put(prefix), false});
  }
  void round(const std::vector<RoundDesc>& v) {
    if (v.empty()) return;
    int64_t cols = 0;
    for (const auto& e : v) cols = std::max(cols, e.N);
    ops.push_back({kRound, false, false, put(v), (int)v.size(), cols, 0, 0.0, 0, false});
  }
  // device copy of `bytes` host bytes to dst, staged in this round's descriptors
  void copy_in(const void* src, size_t bytes, void* dst) {
    const size_t off = (this->bytes.size() + 15) & ~(size_t)15;
    this->bytes.resize(off + bytes);
    memcpy(this->bytes.data() + off, src, bytes);
    Op o{kCopyIn, false, false, off, 0, (int64_t)bytes, 0, 0.0, 0, false};
    o.dst = dst;
    ops.push_back(std::move(o));
  }
  void call(std::function<int(hipStream_t)> f) {
    Op o{kCall, false, false, 0, 0, 0, 0, 0.0, 0, false};
    o.fn = std::move(f);
    ops.push_back(std::move(o));
  }
  void panel(const std::vector<PanelDesc>& v, int k) {
    if (v.empty()) return;
    int64_t rows = 0;
    for (const auto& e : v) rows = std::max(rows, e.M);
    ops.push_back({kPanel, false, false, put(v), (int)v.size(), rows, k, 0.0, 0, false});
  }
};

// Pinned host slots and device slots of the descriptor ring, kept per device
// between calls (grown, never shrunk).
struct Ring {
  unsigned char* host = nullptr;
  unsigned char* dev = nullptr;
  size_t cap = 0;  // bytes per slot
  hipEvent_t copied[kSlots] = {};
  bool pending[kSlots] = {};
  int slot = 0;
};
std::mutex g_ring_mu;  // one batched call at a time per process

int ring_reserve(Ring& r, size_t cap) {
  if (r.cap >= cap) return RRF_OK;
  for (int s = 0; s < kSlots; ++s)
    if (r.pending[s]) RRF_CHECK_HIP(hipEventSynchronize(r.copied[s]));
  // device slots may still be read by kernels of an asynchronous call
  if (r.dev) RRF_CHECK_HIP(hipDeviceSynchronize());
  if (r.host) RRF_CHECK_HIP(hipHostFree(r.host));
  if (r.dev) RRF_CHECK_HIP(hipFree(r.dev));
  r.host = nullptr;
  r.dev = nullptr;
  r.cap = 0;
  RRF_CHECK_HIP(hipHostMalloc((void**)&r.host, kSlots * cap, hipHostMallocDefault));
  RRF_CHECK_HIP(hipMalloc((void**)&r.dev, kSlots * cap));
  for (int s = 0; s < kSlots; ++s) {
    if (!r.copied[s]) RRF_CHECK_HIP(hipEventCreateWithFlags(&r.copied[s], hipEventDisableTiming));
    r.pending[s] = false;
  }
  r.cap = cap;
  return RRF_OK;
}

// Enqueue the launches of round `p` whose descriptors sit at device address d.
int enqueue_plan(hipStream_t st, const Plan& p, const unsigned char* d) {
  for (const auto& op : p.ops) {
    const void* dd = d + op.off;
    switch (op.kind) {
      case Plan::kGemm:
        RRF_TRY(gemm_grouped(st, op.ta, op.tb, op.k, op.vec, static_cast<const GemmDesc*>(dd),
                             reinterpret_cast<const int*>(d + op.off2), op.count, op.aux,
                             op.flops));
        break;
      case Plan::kElem:
        RRF_TRY(elem_batched(st, static_cast<const ElemDesc*>(dd), op.count, op.aux));
        break;
      case Plan::kGauss:
        RRF_TRY(gauss_batched(st, static_cast<const GaussDesc*>(dd), op.count, op.aux));
        break;
      case Plan::kMax:
        RRF_TRY(maxabs_batched(st, static_cast<const MaxDesc*>(dd), op.count, op.aux));
        break;
      case Plan::kBf16:
        RRF_TRY(to_bf16_batched(st, static_cast<const Bf16Desc*>(dd), op.count, op.aux));
        break;
      case Plan::kGemm16:
        RRF_TRY(gemm_bf16_grouped(st, static_cast<const Bf16GemmDesc*>(dd),
                                  reinterpret_cast<const int*>(d + op.off2), op.count, op.aux,
                                  op.flops));
        break;
      case Plan::kRound:
        RRF_TRY(round_columns_batched(st, static_cast<const RoundDesc*>(dd), op.count, op.aux));
        break;
      case Plan::kCopyIn:
        RRF_CHECK_HIP(hipMemcpyAsync(op.dst, dd, (size_t)op.aux, hipMemcpyDeviceToDevice, st));
        break;
      case Plan::kCall:
        RRF_TRY(op.fn(st));
        break;
      default:
        RRF_TRY(panel_wg_batched(st, static_cast<const PanelDesc*>(dd), op.count, op.k, op.aux));
    }
  }
  return RRF_OK;
}

// Stream round `p` through the next ring slot: its descriptors are copied to
// the slot's device side, then its launches are enqueued on `st`.
int run_plan(hipStream_t st, Ring& r, const Plan& p) {
  if (p.ops.empty()) return RRF_OK;
  if (p.bytes.size() > r.cap)
    return set_error(RRF_E_INTERNAL, "batched randutv: descriptor round exceeds its slot");
  const int s = r.slot;
  r.slot = (r.slot + 1) % kSlots;
  // once the slot's previous copy has completed, its host side is free; its
  // device side is read only by kernels enqueued before the next copy
  if (r.pending[s]) RRF_CHECK_HIP(hipEventSynchronize(r.copied[s]));
  unsigned char* h = r.host + (size_t)s * r.cap;
  unsigned char* d = r.dev + (size_t)s * r.cap;
  if (!p.bytes.empty()) {
    memcpy(h, p.bytes.data(), p.bytes.size());
    RRF_CHECK_HIP(hipMemcpyAsync(d, h, p.bytes.size(), hipMemcpyHostToDevice, st));
  }
  RRF_CHECK_HIP(hipEventRecord(r.copied[s], st));
  r.pending[s] = true;
  return enqueue_plan(st, p, d);
}

// Where a finished round goes: streamed through a ring, or kept for a recording.
using Emit = std::function<int(Plan&)>;

GemmDesc gd(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
            const double* B, int64_t ldb, double beta, double* C, int64_t ldc) {
  return GemmDesc{M, N, K, A, lda, B, ldb, C, ldc, alpha, beta};
}
ElemDesc fill(int64_t rows, int64_t cols, double v, double* X, int64_t ld) {
  return ElemDesc{kElemFill, rows, cols, nullptr, 0, X, ld, v};
}
ElemDesc copy(int64_t rows, int64_t cols, const double* S, int64_t lds, double* X, int64_t ld) {
  return ElemDesc{kElemCopy, rows, cols, S, lds, X, ld, 0.0};
}

// Householder panels of width k for every problem in P, split by columns
// while the tallest does not fit one workgroup: QR of the left k1 columns,
// the right k2 columns updated by the left factor's transpose, QR of their
// lower part, then the merged T_f = [T1, -T1 W1^T W2 T2; 0, T2]. pt[i] is
// problem i's scratch, 3 k1 k2 doubles per level. False when a panel cannot
// be split further.
bool plan_panel(std::vector<Plan>& rounds, const std::vector<PanelDesc>& P,
                const std::vector<double*>& pt, int k) {
  if (P.empty()) return true;
  // one launch holds every panel (each is a chain of k latency-bound column
  // steps, so the launch takes as long as its slowest panel); when any is
  // too tall for one workgroup, all are split
  int64_t maxM = 0;
  for (const auto& p : P) maxM = std::max(maxM, p.M);
  if (maxM <= panel_wg_max_rows(k) && (t_panel_leaf <= 0 || k <= t_panel_leaf)) {
    rounds.emplace_back();
    rounds.back().panel(P, k);
    return true;
  }
  if (k < 2) return false;
  const int k1 = k / 2, k2 = k - k1;
  const size_t lvl = (size_t)3 * k1 * k2;
  std::vector<double*> pt_next(P.size());
  for (size_t i = 0; i < P.size(); ++i) pt_next[i] = pt[i] + lvl;
  if (!plan_panel(rounds, P, pt_next, k1)) return false;  // left half (first k1 columns)

  rounds.emplace_back();
  {
    Plan& a = rounds.back();
    std::vector<ElemDesc> cp, zr, r12;
    std::vector<GemmDesc> g1, g2, g3;
    for (size_t i = 0; i < P.size(); ++i) {
      const PanelDesc& p = P[i];
      double* W2 = p.W + (int64_t)k1 * p.ldw;
      double *Z = pt[i], *Z2 = Z + (size_t)k1 * k2;
      if (p.W != p.P || p.ldw != p.ldp)
        cp.push_back(copy(p.M, k2, p.P + (int64_t)k1 * p.ldp, p.ldp, W2, p.ldw));
      if (p.zero) zr.push_back(fill(p.M, k2, 0.0, p.zero + (int64_t)k1 * p.ldz, p.ldz));
      // A2 <- (I - W1 T1 W1^T)^T A2
      g1.push_back(gd(k1, k2, p.M, 1.0, p.W, p.ldw, W2, p.ldw, 0.0, Z, k1));
      g2.push_back(gd(k1, k2, k1, 1.0, p.Tf, p.ldt, Z, k1, 0.0, Z2, k1));
      g3.push_back(gd(p.M, k2, k1, -1.0, p.W, p.ldw, Z2, k1, 1.0, W2, p.ldw));
      if (p.R) {
        r12.push_back(copy(k1, k2, W2, p.ldw, p.R + (int64_t)k1 * p.ldr, p.ldr));
        r12.push_back(fill(k2, k1, 0.0, p.R + k1, p.ldr));
      }
    }
    a.elem(cp);  // before the clear, which may cover the same block
    a.elem(zr);
    a.gemm(true, false, g1);
    a.gemm(true, false, g2);
    a.gemm(false, false, g3);
    a.elem(r12);
  }
  std::vector<PanelDesc> Q;
  for (const auto& p : P) {
    double* W2 = p.W + (int64_t)k1 * p.ldw;
    Q.push_back(PanelDesc{p.M - k1, W2 + k1, p.ldw, W2 + k1, p.ldw,
                          p.R ? p.R + k1 + (int64_t)k1 * p.ldr : nullptr, p.ldr,
                          p.Tf + k1 + (int64_t)k1 * p.ldt, p.ldt, p.tau + k1, nullptr, 0});
  }
  if (!plan_panel(rounds, Q, pt_next, k2)) return false;  // right half, in place

  rounds.emplace_back();
  Plan& c = rounds.back();
  std::vector<ElemDesc> z2;
  std::vector<GemmDesc> h1, h2, h3;
  for (size_t i = 0; i < P.size(); ++i) {
    const PanelDesc& p = P[i];
    double* W2 = p.W + (int64_t)k1 * p.ldw;
    double *Z = pt[i], *S = Z + (size_t)2 * k1 * k2;
    z2.push_back(fill(k1, k2, 0.0, W2, p.ldw));  // R12 leaves the reflector block
    z2.push_back(fill(k2, k1, 0.0, p.Tf + k1, p.ldt));
    h1.push_back(gd(k1, k2, p.M, 1.0, p.W, p.ldw, W2, p.ldw, 0.0, S, k1));
    h2.push_back(gd(k1, k2, k1, 1.0, p.Tf, p.ldt, S, k1, 0.0, Z, k1));
    h3.push_back(gd(k1, k2, k2, -1.0, Z, k1, p.Tf + k1 + (int64_t)k1 * p.ldt, p.ldt, 0.0,
                    p.Tf + (int64_t)k1 * p.ldt, p.ldt));
  }
  c.elem(z2);
  c.gemm(true, false, h1);
  c.gemm(false, false, h2);
  c.gemm(false, false, h3);
  return true;
}

int64_t panel_levels_doubles(int k) {
  int64_t t = 0;
  for (int kk = k; kk > 1; kk -= kk / 2) t += (int64_t)3 * (kk / 2) * (kk - kk / 2);
  return t;
}

struct Shared {
  int* status = nullptr;  // word 0: device-side failure bits
  double *R = nullptr, *Us = nullptr, *Vs = nullptr, *d = nullptr;
  int* sizes = nullptr;
  void* svd = nullptr;
  size_t svd_bytes = 0;
  int64_t nblocks = 0;
};

// Carve the workspace (or only count its bytes when base is null).
size_t layout(int64_t count, const int64_t* m, const int64_t* n, int64_t b, int precision,
              char* base, Shared* sh, std::vector<Mat>* mats) {
  Arena ar;
  ar.base = base;
  ar.counting = base == nullptr;
  ar.cap = (size_t)-1;
  Shared s;
  s.status = ar.take<int>(64);
  for (int64_t j = 0; j < count; ++j) s.nblocks += ceil_div(n[j], b);
  s.R = ar.take<double>((size_t)s.nblocks * b * b);
  s.Us = ar.take<double>((size_t)s.nblocks * b * b);
  s.Vs = ar.take<double>((size_t)s.nblocks * b * b);
  s.d = ar.take<double>((size_t)s.nblocks * b);
  s.sizes = ar.take<int>((size_t)s.nblocks);
  s.svd_bytes = (size_t)s.nblocks * block_svd_work_bytes((int)b);
  s.svd = ar.take<char>(s.svd_bytes);
  if (sh) *sh = s;
  if (mats) mats->resize(count);
  int64_t blk = 0;
  for (int64_t j = 0; j < count; ++j) {
    const int64_t mj = m[j], nj = n[j], mx = std::max(mj, nj), kb = std::min(b, nj);
    const int64_t st = ceil_div(nj, b), gk = kBGroup * kb;
    Mat x{};
    x.m = mj;
    x.n = nj;
    x.s = st;
    x.blk0 = blk;
    blk += st;
    x.G = ar.take<double>((size_t)mj * kb);
    x.Y = ar.take<double>((size_t)nj * kb);
    x.Z = ar.take<double>((size_t)mj * kb);
    x.XW = ar.take<double>((size_t)mj * 2 * kb);
    x.WZ = ar.take<double>((size_t)nj * 2 * kb);
    x.S = ar.take<double>((size_t)kb * kb);
    x.X0 = ar.take<double>((size_t)mx * kb);
    x.Zl = ar.take<double>((size_t)kb * nj);
    x.WU = ar.take<double>((size_t)mj * nj);
    x.WV = ar.take<double>((size_t)nj * nj);
    x.TU = ar.take<double>((size_t)st * b * b);  // factor of step i at i b^2, ld b
    x.TV = ar.take<double>((size_t)st * b * b);
    x.tau = ar.take<double>((size_t)kb);
    x.pt = ar.take<double>((size_t)panel_levels_doubles((int)kb) + 1);
    x.TG = ar.take<double>((size_t)2 * gk * gk);
    x.Sx = ar.take<double>((size_t)2 * gk * kb);
    x.Sy = ar.take<double>((size_t)2 * gk * kb);
    x.Zg = ar.take<double>((size_t)2 * gk * mx);
    x.Z2 = ar.take<double>((size_t)2 * gk * mx);
    if (precision == RRF_PREC_BF16_SKETCH) {
      const int64_t lm = bf16_ld(mj), ln = bf16_ld(nj);
      x.Tb = ar.take<uint16_t>((size_t)lm * nj);
      x.Tbt = ar.take<uint16_t>((size_t)ln * mj);
      x.Gb = ar.take<uint16_t>((size_t)lm * kb);
      x.Yb = ar.take<uint16_t>((size_t)ln * kb);
      x.Zb = ar.take<uint16_t>((size_t)lm * kb);
      x.Pf = ar.take<float>((size_t)mx * kb);
      x.word = ar.take<unsigned long long>(1);
    }
    if (mats) (*mats)[j] = x;
  }
  return ar.used;
}

// The mixed sketch of step i for the matrices in `js` (as sketch_mixed of
// randutv.hip): T22 scaled by the power of two of its max|.| and rounded to
// bfloat16 with its transpose, G rounded as it is, every product accumulated
// in FP32; the intermediate columns are rescaled by powers of two and
// rounded, the last product is widened to FP64 into Y.
void plan_sketch_bf16(std::vector<Plan>& rounds, std::vector<Mat>& mats,
                      const std::vector<int64_t>& js, int64_t c0, int64_t b, int q) {
  if (js.empty()) return;
  rounds.emplace_back();
  Plan& p = rounds.back();
  std::vector<GaussDesc> g;
  std::vector<ElemDesc> zw;
  std::vector<MaxDesc> mx;
  std::vector<Bf16Desc> cv;
  for (int64_t j : js) {
    Mat& x = mats[j];
    const int64_t Mi = x.m - c0, Ni = x.n - c0;
    const double* T22 = x.T + c0 + c0 * x.m;
    g.push_back(GaussDesc{x.seed, (uint64_t)(c0 / b + 1), Mi, b, x.G, Mi});
    zw.push_back(fill(1, 1, 0.0, reinterpret_cast<double*>(x.word), 1));  // 0.0 has all-zero bits
    mx.push_back(MaxDesc{Mi, Ni, T22, x.m, x.word});
    cv.push_back(Bf16Desc{Mi, Ni, T22, x.m, x.word, x.Tb, bf16_ld(Mi), x.Tbt, bf16_ld(Ni)});
  }
  p.gauss(g);
  p.elem(zw);
  p.maxabs(mx);
  std::vector<Bf16Desc> gc;
  for (int64_t j : js) {
    Mat& x = mats[j];
    const int64_t Mi = x.m - c0;
    gc.push_back(Bf16Desc{Mi, b, x.G, Mi, nullptr, x.Gb, bf16_ld(Mi), nullptr, 0});
  }
  cv.insert(cv.end(), gc.begin(), gc.end());
  p.bf16(cv);
  // Y = T22^T G
  {
    std::vector<Bf16GemmDesc> gm;
    std::vector<RoundDesc> rd;
    for (int64_t j : js) {
      Mat& x = mats[j];
      const int64_t Mi = x.m - c0, Ni = x.n - c0, lm = bf16_ld(Mi), ln = bf16_ld(Ni);
      const bool last = q == 0;
      gm.push_back(Bf16GemmDesc{Ni, b, Mi, x.Tb, lm, x.Gb, lm, last ? nullptr : x.Pf, Ni,
                                last ? x.Y : nullptr, Ni});
      if (!last) rd.push_back(RoundDesc{Ni, b, x.Pf, Ni, x.Yb, ln});
    }
    p.gemm16(gm);
    p.round(rd);
  }
  for (int it = 0; it < q; ++it) {
    const bool last = it == q - 1;
    std::vector<Bf16GemmDesc> gz, gy;
    std::vector<RoundDesc> rz, ry;
    for (int64_t j : js) {
      Mat& x = mats[j];
      const int64_t Mi = x.m - c0, Ni = x.n - c0, lm = bf16_ld(Mi), ln = bf16_ld(Ni);
      // Z = T22 Y = Tbt^T Y, then Y = T22^T Z = Tb^T Z
      gz.push_back(Bf16GemmDesc{Mi, b, Ni, x.Tbt, ln, x.Yb, ln, x.Pf, Mi, nullptr, 0});
      rz.push_back(RoundDesc{Mi, b, x.Pf, Mi, x.Zb, lm});
      gy.push_back(Bf16GemmDesc{Ni, b, Mi, x.Tb, lm, x.Zb, lm, last ? nullptr : x.Pf, Ni,
                                last ? x.Y : nullptr, Ni});
      if (!last) ry.push_back(RoundDesc{Ni, b, x.Pf, Ni, x.Yb, ln});
    }
    p.gemm16(gz);
    p.round(rz);
    p.gemm16(gy);
    p.round(ry);
  }
}

// The loop of Alg. 3 for every matrix, step i of all together.
int run_loop(const Emit& emit, std::vector<Mat>& mats, const Shared& sh, int64_t b, int q,
             int precision, std::vector<std::vector<int64_t>>& ku,
             std::vector<std::vector<int64_t>>& kv) {
  const int64_t bb = b;
  const int64_t count = (int64_t)mats.size();
  std::vector<Plan> rounds;
  int64_t smax = 0;
  for (auto& x : mats) smax = std::max(smax, x.s);
  for (int64_t i = 0; i < smax; ++i) {
    const int64_t c0 = i * b;
    std::vector<int64_t> norm, last;
    for (int64_t j = 0; j < count; ++j) {
      if (i >= mats[j].s) continue;
      (i < mats[j].s - 1 ? norm : last).push_back(j);
    }
    // sketch: Y = T22^T G_i, then q times Z = T22 Y, Y = T22^T Z
    if (precision == RRF_PREC_BF16_SKETCH) {
      plan_sketch_bf16(rounds, mats, norm, c0, b, q);
    } else {
      rounds.emplace_back();
      std::vector<GaussDesc> g;
      std::vector<GemmDesc> y;
      for (int64_t j : norm) {
        Mat& x = mats[j];
        const int64_t Mi = x.m - c0, Ni = x.n - c0;
        g.push_back(GaussDesc{x.seed, (uint64_t)(i + 1), Mi, b, x.G, Mi});
        y.push_back(gd(Ni, b, Mi, 1.0, x.T + c0 + c0 * x.m, x.m, x.G, Mi, 0.0, x.Y, Ni));
      }
      rounds.back().gauss(g);
      rounds.back().gemm(true, false, y);
      for (int it = 0; it < q; ++it) {
        rounds.emplace_back();
        std::vector<GemmDesc> z, yy;
        for (int64_t j : norm) {
          Mat& x = mats[j];
          const int64_t Mi = x.m - c0, Ni = x.n - c0;
          const double* T22 = x.T + c0 + c0 * x.m;
          z.push_back(gd(Mi, b, Ni, 1.0, T22, x.m, x.Y, Ni, 0.0, x.Z, Mi));
          yy.push_back(gd(Ni, b, Mi, 1.0, T22, x.m, x.Z, Mi, 0.0, x.Y, Ni));
        }
        rounds.back().gemm(false, false, z);
        rounds.back().gemm(true, false, yy);
      }
    }
    // V_i: Householder QR of Y (W_v, T_v kept for the backward V)
    {
      std::vector<PanelDesc> P;
      std::vector<double*> pt;
      for (int64_t j : norm) {
        Mat& x = mats[j];
        const int64_t Ni = x.n - c0;
        P.push_back(PanelDesc{Ni, x.Y, Ni, x.WV + c0 + c0 * x.n, x.n, nullptr, 0,
                              x.TV + i * bb * bb, bb, x.tau, nullptr, 0});
        pt.push_back(x.pt);
        kv[j][i] = b;
      }
      if (!plan_panel(rounds, P, pt, (int)b))
        return set_error(RRF_E_NOTSUP, "batched randutv: panel too tall to split");
    }
    // Wr = W_v T_v^T, X = T(:, J2uJ3) W_v, columns J2 of T V_i = T - X Wr^T
    {
      rounds.emplace_back();
      std::vector<GemmDesc> wr, xg, j2;
      for (int64_t j : norm) {
        Mat& x = mats[j];
        const int64_t Ni = x.n - c0;
        const double* Wv = x.WV + c0 + c0 * x.n;
        wr.push_back(gd(Ni, b, b, 1.0, Wv, x.n, x.TV + i * bb * bb, bb, 0.0, x.WZ, x.n));
        xg.push_back(gd(x.m, b, Ni, 1.0, x.T + c0 * x.m, x.m, Wv, x.n, 0.0, x.XW, x.m));
        j2.push_back(gd(x.m, b, b, -1.0, x.XW, x.m, x.WZ, x.n, 1.0, x.T + c0 * x.m, x.m));
      }
      rounds.back().gemm(false, true, wr);
      rounds.back().gemm(false, false, xg);
      rounds.back().gemm(false, true, j2);
    }
    // U_i and R: Householder QR of T(I2uI3, J2), the panel cleared in T; the
    // last block likewise when tall, else copied into R as it is
    {
      std::vector<PanelDesc> P;
      std::vector<double*> pt;
      for (int64_t j : norm) {
        Mat& x = mats[j];
        double* T22 = x.T + c0 + c0 * x.m;
        P.push_back(PanelDesc{x.m - c0, T22, x.m, x.WU + c0 + c0 * x.m, x.m,
                              sh.R + (x.blk0 + i) * bb * bb, bb, x.TU + i * bb * bb, bb, x.tau,
                              T22, x.m});
        pt.push_back(x.pt);
        ku[j][i] = b;
      }
      if (!plan_panel(rounds, P, pt, (int)b))
        return set_error(RRF_E_NOTSUP, "batched randutv: panel too tall to split");
      rounds.emplace_back();
      std::vector<ElemDesc> cp;
      std::vector<PanelDesc> PL;
      std::vector<double*> ptl;
      std::vector<int> lw;
      for (int64_t j : last) {
        Mat& x = mats[j];
        const int64_t Mi = x.m - c0, Ni = x.n - c0;
        double* T22 = x.T + c0 + c0 * x.m;
        double* Rb = sh.R + (x.blk0 + i) * bb * bb;
        if (Mi > Ni) {
          PL.push_back(PanelDesc{Mi, T22, x.m, x.WU + c0 + c0 * x.m, x.m, Rb, bb,
                                 x.TU + i * bb * bb, bb, x.tau, nullptr, 0});
          ptl.push_back(x.pt);
          lw.push_back((int)Ni);
          ku[j][i] = Ni;
        } else {
          cp.push_back(copy(Ni, Ni, T22, x.m, Rb, bb));
        }
      }
      rounds.back().elem(cp);
      // one group of panels per width (the last blocks of a batch may differ)
      std::vector<int> widths(lw);
      std::sort(widths.begin(), widths.end());
      widths.erase(std::unique(widths.begin(), widths.end()), widths.end());
      for (int w : widths) {
        std::vector<PanelDesc> Pw;
        std::vector<double*> ptw;
        for (size_t t = 0; t < PL.size(); ++t)
          if (lw[t] == w) {
            Pw.push_back(PL[t]);
            ptw.push_back(ptl[t]);
          }
        if (!plan_panel(rounds, Pw, ptw, w))
          return set_error(RRF_E_NOTSUP, "batched randutv: panel too tall to split");
      }
    }
    // T(:, J3) <- U_i^T (T(:, J3) - X Wr(J3)^T): with Wl = W_u T_u^T (zero on
    // the rows above c0) and Z^T = T(I2uI3, J3)^T W_u - Wr(J3) (X(I2uI3)^T W_u),
    // one product T(:, J3) -= [X, Wl] [Wr(J3), Z^T]^T
    {
      rounds.emplace_back();
      std::vector<ElemDesc> zf;
      std::vector<GemmDesc> wl, zt, sg, zc, up;
      for (int64_t j : norm) {
        Mat& x = mats[j];
        const int64_t Mi = x.m - c0, c2 = c0 + b, N3 = x.n - c2;
        const double* Wu = x.WU + c0 + c0 * x.m;
        double* Wl = x.XW + x.m * b;
        double* Zt = x.WZ + x.n * b;
        const int64_t z0 = std::max<int64_t>(0, c0 - b);  // rows written by step i-1
        if (c0 > z0) zf.push_back(fill(c0 - z0, b, 0.0, Wl + z0, x.m));
        wl.push_back(gd(Mi, b, b, 1.0, Wu, x.m, x.TU + i * bb * bb, bb, 0.0, Wl + c0, x.m));
        zt.push_back(gd(N3, b, Mi, 1.0, x.T + c0 + c2 * x.m, x.m, Wu, x.m, 0.0, Zt + b, x.n));
        sg.push_back(gd(b, b, Mi, 1.0, x.XW + c0, x.m, Wu, x.m, 0.0, x.S, b));
        zc.push_back(gd(N3, b, b, -1.0, x.WZ + b, x.n, x.S, b, 1.0, Zt + b, x.n));
        up.push_back(gd(x.m, N3, 2 * b, -1.0, x.XW, x.m, x.WZ + b, x.n, 1.0, x.T + c2 * x.m, x.m));
      }
      Plan& p = rounds.back();
      p.elem(zf);
      p.gemm(false, true, wl);
      p.gemm(true, false, zt);
      p.gemm(true, false, sg);
      p.gemm(false, false, zc);
      p.gemm(false, true, up);
    }
    for (auto& p : rounds) RRF_TRY(emit(p));
    rounds.clear();
  }
  return RRF_OK;
}

// Block SVDs, T's diagonal blocks, and the block updates T(I1, J2) Vs and
// Us^T T(J2, J3).
int run_blocks(const Emit& emit, std::vector<Mat>& mats, const Shared& sh, int64_t b) {
  const int64_t bb = b;
  {
    Plan sv;
    sv.call([sh, b, bb](hipStream_t st) {
      return block_svd_sized(st, (int)sh.nblocks, (int)b, sh.sizes, sh.R, bb, bb * bb, sh.Us,
                             sh.d, bb, sh.Vs, sh.svd, sh.svd_bytes, sh.status);
    });
    RRF_TRY(emit(sv));
  }
  int64_t smax = 0;
  for (auto& x : mats) smax = std::max(smax, x.s);
  for (int64_t i = 0; i < smax; ++i) {
    const int64_t c0 = i * b;
    Plan p;
    std::vector<ElemDesc> dg, cb;
    std::vector<GemmDesc> t1, t2;
    for (auto& x : mats) {
      if (i >= x.s) continue;
      const int64_t kb = std::min(b, x.n - c0), c2 = c0 + kb;
      const bool lastb = i == x.s - 1;
      const int64_t g = x.blk0 + i;
      double* T22 = x.T + c0 + c0 * x.m;
      dg.push_back(ElemDesc{kElemDiag, lastb ? x.m - c0 : kb, kb, sh.d + g * bb, 0, T22, x.m, 0.0});
      if (c0 > 0) {
        t1.push_back(gd(c0, kb, kb, 1.0, x.T + c0 * x.m, x.m, sh.Vs + g * bb * bb, kb, 0.0, x.X0,
                        c0));
        cb.push_back(copy(c0, kb, x.X0, c0, x.T + c0 * x.m, x.m));
      }
      if (!lastb) {
        const int64_t N3 = x.n - c2;
        t2.push_back(gd(kb, N3, kb, 1.0, sh.Us + g * bb * bb, kb, x.T + c0 + c2 * x.m, x.m, 0.0,
                        x.Zl, kb));
        cb.push_back(copy(kb, N3, x.Zl, kb, x.T + c0 + c2 * x.m, x.m));
      }
    }
    p.elem(dg);
    p.gemm(false, false, t1);
    p.gemm(true, false, t2);
    p.elem(cb);
    RRF_TRY(emit(p));
  }
  return RRF_OK;
}

// U = H_0 ... H_{s-1} and V likewise, applied to I from the last group of
// kBGroup steps backward (only Q(ca:, ca:) changes), then the rotations of
// their block columns by Us and Vs.
int run_backward(const Emit& emit, std::vector<Mat>& mats, const Shared& sh, int64_t b,
                 const std::vector<std::vector<int64_t>>& ku,
                 const std::vector<std::vector<int64_t>>& kv) {
  const int64_t bb = b;
  struct Job {
    double* Q;
    int64_t N;
    const double* W;
    const double* Tall;
    const std::vector<int64_t>* kbs;
    double *TG, *Sx, *Sy, *Zg, *Z2;
    std::vector<std::pair<int64_t, int64_t>> groups;  // [i0, i1), last group first
  };
  std::vector<Job> jobs;
  for (size_t j = 0; j < mats.size(); ++j) {
    Mat& x = mats[j];
    const int64_t kb = std::min(b, x.n), gk = kBGroup * kb, mx = std::max(x.m, x.n);
    for (int side = 0; side < 2; ++side) {
      double* Q = side == 0 ? x.U : x.V;
      if (!Q) continue;
      Job jb{Q,
             side == 0 ? x.m : x.n,
             side == 0 ? x.WU : x.WV,
             side == 0 ? x.TU : x.TV,
             side == 0 ? &ku[j] : &kv[j],
             x.TG + side * gk * gk,
             x.Sx + side * gk * kb,
             x.Sy + side * gk * kb,
             x.Zg + side * gk * mx,
             x.Z2 + side * gk * mx,
             {}};
      const auto& kbs = *jb.kbs;
      int64_t i1 = (int64_t)kbs.size();
      while (i1 > 0) {
        while (i1 > 0 && kbs[i1 - 1] == 0) --i1;
        if (i1 == 0) break;
        int64_t i0 = std::max<int64_t>(0, i1 - kBGroup);
        for (int64_t t = i1 - 1; t >= i0; --t)
          if (kbs[t] == 0) {
            i0 = t + 1;
            break;
          }
        jb.groups.push_back({i0, i1});
        i1 = i0;
      }
      jobs.push_back(std::move(jb));
    }
  }
  if (jobs.empty()) return RRF_OK;
  {
    Plan p;
    std::vector<ElemDesc> id;
    for (auto& jb : jobs)
      id.push_back(ElemDesc{kElemIdentity, jb.N, jb.N, nullptr, 0, jb.Q, jb.N, 0.0});
    p.elem(id);
    RRF_TRY(emit(p));
  }
  size_t rmax = 0;
  for (auto& jb : jobs) rmax = std::max(rmax, jb.groups.size());
  auto width_of = [](const Job& jb, int64_t i0, int64_t i1) {
    int64_t w = 0;
    for (int64_t u = i0; u < i1; ++u) w += (*jb.kbs)[u];
    return w;
  };
  for (size_t r = 0; r < rmax; ++r) {
    // merged factor T_G of the group, one step per round:
    // T_G(0:p, p:p+k) = -T_G(0:p, 0:p) W_G(:, 0:p)^T W_t T_t, T_G(p:, p:) = T_t
    for (int t = 0; t < kBGroup; ++t) {
      Plan pl;
      std::vector<ElemDesc> zf, cp;
      std::vector<GemmDesc> s1, s2, s3;
      for (auto& jb : jobs) {
        if (r >= jb.groups.size()) continue;
        const auto [i0, i1] = jb.groups[r];
        if (i0 + t >= i1) continue;
        const int64_t width = width_of(jb, i0, i1);
        const int64_t ca = i0 * b, Nq = jb.N - ca, p = t * b, kbi = (*jb.kbs)[i0 + t];
        const double* WG = jb.W + ca + ca * jb.N;
        const double* Ti = jb.Tall + (i0 + t) * bb * bb;
        if (t == 0) zf.push_back(fill(width, width, 0.0, jb.TG, width));
        if (p > 0) {
          s1.push_back(gd(p, kbi, Nq, 1.0, WG, jb.N, WG + p * jb.N, jb.N, 0.0, jb.Sx, p));
          s2.push_back(gd(p, kbi, p, 1.0, jb.TG, width, jb.Sx, p, 0.0, jb.Sy, p));
          s3.push_back(gd(p, kbi, kbi, -1.0, jb.Sy, p, Ti, bb, 0.0, jb.TG + p * width, width));
        }
        cp.push_back(copy(kbi, kbi, Ti, bb, jb.TG + p + p * width, width));
      }
      pl.elem(zf);
      pl.gemm(true, false, s1);
      pl.gemm(false, false, s2);
      pl.gemm(false, false, s3);
      pl.elem(cp);
      RRF_TRY(emit(pl));
    }
    // Q(ca:, ca:) -= W_G (T_G (W_G^T Q(ca:, ca:)))
    Plan pl;
    std::vector<GemmDesc> a1, a2, a3;
    for (auto& jb : jobs) {
      if (r >= jb.groups.size()) continue;
      const auto [i0, i1] = jb.groups[r];
      const int64_t width = width_of(jb, i0, i1);
      const int64_t ca = i0 * b, Nq = jb.N - ca;
      const double* WG = jb.W + ca + ca * jb.N;
      double* Qb = jb.Q + ca + ca * jb.N;
      a1.push_back(gd(width, Nq, Nq, 1.0, WG, jb.N, Qb, jb.N, 0.0, jb.Zg, width));
      a2.push_back(gd(width, Nq, width, 1.0, jb.TG, width, jb.Zg, width, 0.0, jb.Z2, width));
      a3.push_back(gd(Nq, Nq, width, -1.0, WG, jb.N, jb.Z2, width, 1.0, Qb, jb.N));
    }
    pl.gemm(true, false, a1);
    pl.gemm(false, false, a2);
    pl.gemm(false, false, a3);
    RRF_TRY(emit(pl));
  }
  int64_t smax = 0;
  for (auto& x : mats) smax = std::max(smax, x.s);
  for (int64_t i = 0; i < smax; ++i) {
    const int64_t c0 = i * b;
    Plan p;
    std::vector<GemmDesc> g;
    std::vector<ElemDesc> cb;
    for (auto& x : mats) {
      if (i >= x.s) continue;
      const int64_t kb = std::min(b, x.n - c0), gb = x.blk0 + i;
      if (x.U) {
        g.push_back(gd(x.m, kb, kb, 1.0, x.U + c0 * x.m, x.m, sh.Us + gb * bb * bb, kb, 0.0, x.Zg,
                       x.m));
        cb.push_back(copy(x.m, kb, x.Zg, x.m, x.U + c0 * x.m, x.m));
      }
      if (x.V) {
        g.push_back(gd(x.n, kb, kb, 1.0, x.V + c0 * x.n, x.n, sh.Vs + gb * bb * bb, kb, 0.0, x.Z2,
                       x.n));
        cb.push_back(copy(x.n, kb, x.Z2, x.n, x.V + c0 * x.n, x.n));
      }
    }
    p.gemm(false, false, g);
    p.elem(cb);
    RRF_TRY(emit(p));
  }
  return RRF_OK;
}

}  // namespace

int64_t randutv_batched_block(int64_t m, int64_t n) {
  (void)m;
  // measured per n bucket of the 4096-matrix workload (n in [64, 512],
  // m in [n, 2n], q = 1): 16 is fastest up to n = 256, 32 above; 64 never
  // wins (its panels need column splits and its block SVDs are 8x dearer)
  return n <= 256 ? 16 : 32;
}

size_t randutv_batched_workspace(int64_t count, const int64_t* m, const int64_t* n, int64_t b,
                                 int precision) {
  return layout(count, m, n, b, precision, nullptr, nullptr, nullptr);
}

namespace {

// Every round of one slice of the batch, in order: set-up, the loop, the
// block SVDs and updates, and U and V. mats[j].blk0 and sh index the slice's
// own blocks.
int plan_slice(const Emit& emit, std::vector<Mat>& mats, const Shared& sh, const BatchedCfg& cfg,
               int q, int precision) {
  const int64_t b = cfg.b;
  t_tile_mask = cfg.tile_mask;
  t_panel_leaf = cfg.leaf;
  {
    Plan p;
    std::vector<ElemDesc> e;
    for (auto& x : mats) {
      if (x.T != x.A) e.push_back(copy(x.m, x.n, x.A, x.lda, x.T, x.m));
      if (x.U) e.push_back(fill(x.m, x.n, 0.0, x.WU, x.m));  // reflector stores
      if (x.V) e.push_back(fill(x.n, x.n, 0.0, x.WV, x.n));
    }
    p.elem(e);
    RRF_TRY(emit(p));
  }
  {
    std::vector<int> hs((size_t)sh.nblocks);
    for (auto& x : mats)
      for (int64_t i = 0; i < x.s; ++i) hs[x.blk0 + i] = (int)std::min(b, x.n - i * b);
    Plan p;
    p.copy_in(hs.data(), hs.size() * sizeof(int), sh.sizes);
    RRF_TRY(emit(p));
  }
  std::vector<std::vector<int64_t>> ku(mats.size()), kv(mats.size());
  for (size_t j = 0; j < mats.size(); ++j) {
    ku[j].assign(mats[j].s, 0);
    kv[j].assign(mats[j].s, 0);
  }
  RRF_TRY(run_loop(emit, mats, sh, b, q, precision, ku, kv));
  RRF_TRY(run_blocks(emit, mats, sh, b));
  RRF_TRY(run_backward(emit, mats, sh, b, ku, kv));
  return RRF_OK;
}

// One slice streamed through its descriptor ring on `st`.
int run_slice(hipStream_t st, Ring& ring, std::vector<Mat>& mats, const Shared& sh,
              const BatchedCfg& cfg, int q, int precision) {
  RRF_TRY(ring_reserve(ring, std::max(mats.size() * kDescPerMat, (size_t)sh.nblocks * 4) +
                                 (1 << 16)));
  return plan_slice([&](Plan& p) { return run_plan(st, ring, p); }, mats, sh, cfg, q, precision);
}

// A recorded batched call: the descriptors of every round of every slice in
// one resident device buffer, and the launches of each slice captured into a
// HIP graph. A later call with the same shapes replays the graphs; when only
// pointers or seeds differ, the descriptors are rebuilt on the host and
// uploaded into the same buffer first (the rounds and launches depend on the
// shapes alone).
constexpr int kMaxSlices = 4;
constexpr int kMaxRecordings = 8;  // per device, least recently used evicted
struct Recording {
  BatchedCfg cfg{};
  int q = 0, precision = 0, S = 0;
  std::vector<int64_t> m, n, cut;
  uint64_t args = 0;              // hash of the workspace, pointers, ld and seeds
  std::vector<size_t> sizes;      // byte size of every round (layout check)
  std::vector<size_t> offsets;    // device offset of every round
  unsigned char* dev = nullptr;   // resident descriptors
  unsigned char* host = nullptr;  // pinned staging of the last upload
  size_t bytes = 0;
  hipGraphExec_t exec[kMaxSlices] = {};
  hipEvent_t uploaded = nullptr;  // the staging copy has been read
  hipEvent_t done = nullptr;      // the last replay has completed
  uint64_t used = 0;
};

// Per-device resources kept between calls: the slices' descriptor rings, the
// events that order the slices after and before the caller's stream, and the
// recorded calls. Slice 0 runs on the caller's stream, the others on the
// device context's streams.
struct DeviceRes {
  Ring rings[kMaxSlices];
  hipEvent_t done[kMaxSlices] = {};
  hipEvent_t start = nullptr;
  hipEvent_t ring_done = nullptr;  // the last lockstep call's rounds are enqueued up to here
  bool ring_used = false;
  std::vector<Recording*> recs;
  uint64_t clock = 0;
};
std::unordered_map<int, DeviceRes> g_res;

static_assert(kMaxSlices == kSideStreams + 2, "slices on the caller's, side and extra streams");

// The slices' streams of this call (`streams[0]` is the caller's) and the
// events, created on first use; the caller holds `ctx->mu`.
int slice_resources(DeviceRes& r, DeviceContext* ctx, hipStream_t st, hipStream_t* streams) {
  if (!ctx->extra) RRF_CHECK_HIP(hipStreamCreateWithFlags(&ctx->extra, hipStreamNonBlocking));
  if (!r.start) RRF_CHECK_HIP(hipEventCreateWithFlags(&r.start, hipEventDisableTiming));
  if (!r.ring_done) RRF_CHECK_HIP(hipEventCreateWithFlags(&r.ring_done, hipEventDisableTiming));
  streams[0] = st;
  for (int i = 0; i < kSideStreams; ++i) {
    streams[1 + i] = ctx->side[i];
    trace_unmark_stream(ctx->side[i]);  // the batched kernels keep their own classes
  }
  streams[kMaxSlices - 1] = ctx->extra;
  for (int i = 0; i < kMaxSlices; ++i)
    if (!r.done[i]) RRF_CHECK_HIP(hipEventCreateWithFlags(&r.done[i], hipEventDisableTiming));
  return RRF_OK;
}

int free_recording(Recording* r) {
  if (r->done) RRF_CHECK_HIP(hipEventSynchronize(r->done));
  if (r->uploaded) RRF_CHECK_HIP(hipEventSynchronize(r->uploaded));
  for (int i = 0; i < kMaxSlices; ++i)
    if (r->exec[i]) RRF_CHECK_HIP(hipGraphExecDestroy(r->exec[i]));
  if (r->dev) RRF_CHECK_HIP(hipFree(r->dev));
  if (r->host) RRF_CHECK_HIP(hipHostFree(r->host));
  if (r->done) RRF_CHECK_HIP(hipEventDestroy(r->done));
  if (r->uploaded) RRF_CHECK_HIP(hipEventDestroy(r->uploaded));
  delete r;
  return RRF_OK;
}

uint64_t fnv(uint64_t h, uint64_t v) {
  for (int i = 0; i < 8; ++i) {
    h ^= (v >> (8 * i)) & 0xff;
    h *= 1099511628211ull;
  }
  return h;
}

uint64_t args_hash(const std::vector<Mat>& mats, const void* ws) {
  uint64_t h = fnv(1469598103934665603ull, (uintptr_t)ws);
  for (const auto& x : mats) {
    h = fnv(h, (uintptr_t)x.A);
    h = fnv(h, (uint64_t)x.lda);
    h = fnv(h, (uintptr_t)x.U);
    h = fnv(h, (uintptr_t)x.T);
    h = fnv(h, (uintptr_t)x.V);
    h = fnv(h, x.seed);
  }
  return h;
}

struct Slice {
  std::vector<Mat> mats;
  Shared sh;
  int rc = RRF_OK;
  std::string msg;
  std::vector<Plan> plans;  // replay mode: every round, in order
};

// Build every slice's rounds on host threads (one per slice).
int build_plans(int dev, std::vector<Slice>& work, const BatchedCfg& cfg, int q, int precision) {
  std::vector<std::thread> threads;
  for (size_t i = 0; i < work.size(); ++i) {
    threads.emplace_back([&, i]() {
      Slice& w = work[i];
      w.plans.clear();
      hipError_t e = hipSetDevice(dev);
      if (e != hipSuccess) {
        w.rc = set_hip_error(e, "hipSetDevice", __FILE__, __LINE__);
      } else if (!w.mats.empty()) {
        w.rc = plan_slice([&](Plan& p) {
          if (!p.ops.empty()) w.plans.push_back(std::move(p));
          return RRF_OK;
        }, w.mats, w.sh, cfg, q, precision);
      }
      if (w.rc != RRF_OK) w.msg = rrf_last_error();
    });
  }
  for (auto& t : threads) t.join();
  for (auto& w : work)
    if (w.rc != RRF_OK) return set_error(w.rc, w.msg.c_str());
  return RRF_OK;
}

// Concatenated descriptors of every round (256-byte aligned) into `host`.
void pack_plans(const std::vector<Slice>& work, const std::vector<size_t>& offsets,
                unsigned char* host) {
  size_t r = 0;
  for (const auto& w : work)
    for (const auto& p : w.plans) {
      if (!p.bytes.empty()) memcpy(host + offsets[r], p.bytes.data(), p.bytes.size());
      ++r;
    }
}

int record(hipStream_t st, const hipStream_t* streams, std::vector<Slice>& work,
           Recording* rec) {
  size_t total = 0;
  for (const auto& w : work)
    for (const auto& p : w.plans) {
      rec->sizes.push_back(p.bytes.size());
      rec->offsets.push_back(total);
      total += (p.bytes.size() + 255) & ~(size_t)255;
    }
  rec->bytes = std::max<size_t>(total, 256);
  RRF_CHECK_HIP(hipMalloc((void**)&rec->dev, rec->bytes));
  RRF_CHECK_HIP(hipHostMalloc((void**)&rec->host, rec->bytes, hipHostMallocDefault));
  RRF_CHECK_HIP(hipEventCreateWithFlags(&rec->uploaded, hipEventDisableTiming));
  RRF_CHECK_HIP(hipEventCreateWithFlags(&rec->done, hipEventDisableTiming));
  pack_plans(work, rec->offsets, rec->host);
  RRF_CHECK_HIP(hipMemcpyAsync(rec->dev, rec->host, rec->bytes, hipMemcpyHostToDevice, st));
  RRF_CHECK_HIP(hipEventRecord(rec->uploaded, st));
  // capture each slice's launches (nothing runs while capturing; the
  // descriptors are read when the graph is launched). The caller's stream may
  // be the null stream, which cannot capture, so every slice is captured on a
  // context stream; a graph runs on whichever stream launches it.
  size_t r = 0;
  for (int i = 0; i < rec->S; ++i) {
    hipStream_t cs = streams[1];
    RRF_CHECK_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    int rc = RRF_OK;
    for (const auto& p : work[i].plans) {
      rc = enqueue_plan(cs, p, rec->dev + rec->offsets[r++]);
      if (rc != RRF_OK) break;
    }
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(cs, &g);
    if (rc != RRF_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    RRF_CHECK_HIP(e);
    e = hipGraphInstantiate(&rec->exec[i], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    RRF_CHECK_HIP(e);
  }
  return RRF_OK;
}

// Launch the recorded graphs, slice 0 on the caller's stream and the others on
// their own, ordered after and before the caller's stream.
int replay(hipStream_t st, const hipStream_t* streams, DeviceRes& res, Recording* rec) {
  if (rec->S > 1) RRF_CHECK_HIP(hipEventRecord(res.start, st));
  for (int i = 1; i < rec->S; ++i) {
    RRF_CHECK_HIP(hipStreamWaitEvent(streams[i], res.start, 0));
    RRF_CHECK_HIP(hipGraphLaunch(rec->exec[i], streams[i]));
    RRF_CHECK_HIP(hipEventRecord(res.done[i], streams[i]));
  }
  RRF_CHECK_HIP(hipGraphLaunch(rec->exec[0], st));
  for (int i = 1; i < rec->S; ++i) RRF_CHECK_HIP(hipStreamWaitEvent(st, res.done[i], 0));
  RRF_CHECK_HIP(hipEventRecord(rec->done, st));
  return RRF_OK;
}

bool same_shapes(const Recording* r, const std::vector<Mat>& mats, const std::vector<int64_t>& cut,
                 const BatchedCfg& cfg, int q, int precision) {
  if (r->cfg.b != cfg.b || r->cfg.tile_mask != cfg.tile_mask || r->cfg.leaf != cfg.leaf ||
      r->q != q || r->precision != precision || r->cut != cut || r->m.size() != mats.size())
    return false;
  for (size_t j = 0; j < mats.size(); ++j)
    if (r->m[j] != mats[j].m || r->n[j] != mats[j].n) return false;
  return true;
}

int run_recorded(hipStream_t st, const hipStream_t* streams, int dev, DeviceRes& res,
                 std::vector<Slice>& work,
                 const std::vector<Mat>& mats, const std::vector<int64_t>& cut, const void* ws,
                 const BatchedCfg& cfg, int q, int precision) {
  const uint64_t h = args_hash(mats, ws);
  Recording* rec = nullptr;
  for (auto* r : res.recs)
    if (same_shapes(r, mats, cut, cfg, q, precision)) rec = r;
  if (rec && rec->args != h) {
    RRF_TRY(build_plans(dev, work, cfg, q, precision));
    size_t nr = 0;
    bool same = true;
    for (const auto& w : work)
      for (const auto& p : w.plans) {
        same = same && nr < rec->sizes.size() && rec->sizes[nr] == p.bytes.size();
        ++nr;
      }
    if (same && nr == rec->sizes.size()) {
      // the staging buffer is reused once its last copy has been read, and
      // the device buffer once the last replay (on any stream) has read it
      RRF_CHECK_HIP(hipEventSynchronize(rec->uploaded));
      pack_plans(work, rec->offsets, rec->host);
      RRF_CHECK_HIP(hipStreamWaitEvent(st, rec->done, 0));
      RRF_CHECK_HIP(hipMemcpyAsync(rec->dev, rec->host, rec->bytes, hipMemcpyHostToDevice, st));
      RRF_CHECK_HIP(hipEventRecord(rec->uploaded, st));
      rec->args = h;
    } else {  // not expected (the rounds follow the shapes): record afresh
      res.recs.erase(std::find(res.recs.begin(), res.recs.end(), rec));
      RRF_TRY(free_recording(rec));
      rec = nullptr;
    }
  }
  if (!rec) {
    if (work[0].plans.empty()) RRF_TRY(build_plans(dev, work, cfg, q, precision));
    if ((int)res.recs.size() >= kMaxRecordings) {
      auto lru = std::min_element(res.recs.begin(), res.recs.end(),
                                  [](const Recording* x, const Recording* y) {
                                    return x->used < y->used;
                                  });
      Recording* old = *lru;
      res.recs.erase(lru);
      RRF_TRY(free_recording(old));
    }
    rec = new Recording();
    rec->cfg = cfg;
    rec->q = q;
    rec->precision = precision;
    rec->S = (int)work.size();
    rec->cut = cut;
    for (const auto& x : mats) {
      rec->m.push_back(x.m);
      rec->n.push_back(x.n);
    }
    rec->args = h;
    const int rc = record(st, streams, work, rec);
    if (rc != RRF_OK) {
      const std::string msg = rrf_last_error();
      (void)free_recording(rec);
      return set_error(rc, msg.c_str());
    }
    res.recs.push_back(rec);
  }
  rec->used = ++res.clock;
  return replay(st, streams, res, rec);
}

}  // namespace

int randutv_batched_run(hipStream_t st, int64_t count, const int64_t* m, const int64_t* n,
                        const double* const* A, const int64_t* lda, const BatchedCfg& cfg, int q,
                        const uint64_t* seeds, double* const* U, double* const* T,
                        double* const* V, void* ws, size_t ws_bytes, int precision,
                        bool use_graph) {
  if (count < 1) return RRF_OK;
  const int64_t b = cfg.b;
  std::vector<Mat> mats;
  Shared sh;
  const size_t need =
      layout(count, m, n, b, precision, reinterpret_cast<char*>(ws), &sh, &mats);
  if (need > ws_bytes) return set_error(RRF_E_NOMEM, "batched randutv: workspace too small");
  for (int64_t j = 0; j < count; ++j) {
    mats[j].A = A[j];
    mats[j].lda = lda[j];
    mats[j].U = U ? U[j] : nullptr;
    mats[j].T = T[j];
    mats[j].V = V ? V[j] : nullptr;
    mats[j].seed = seeds[j];
  }
  int dev = 0;
  RRF_CHECK_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_ring_mu);
  DeviceRes& res = g_res[dev];

  // Contiguous slices of about equal work (m n^2 per matrix): the lockstep
  // rounds of one slice leave the chip partly idle in their latency-bound
  // launches (panels, small SVDs), which the other slices' GEMMs fill.
  const int S = (int)std::min<int64_t>(kMaxSlices, std::max<int64_t>(1, count / 256));
  DeviceContext* ctx = nullptr;
  RRF_TRY(device_context(&ctx));
  std::lock_guard<std::mutex> ctx_lk(ctx->mu);
  hipStream_t streams[kMaxSlices] = {};
  RRF_TRY(slice_resources(res, ctx, st, streams));
  double total = 0.0;
  for (auto& x : mats) total += (double)x.m * x.n * x.n;
  std::vector<int64_t> cut(S + 1, count);
  cut[0] = 0;
  {
    double acc = 0.0;
    int c = 1;
    for (int64_t j = 0; j < count && c < S; ++j) {
      acc += (double)mats[j].m * mats[j].n * mats[j].n;
      if (acc >= total * c / S) cut[c++] = j + 1;
    }
  }
  std::vector<Slice> work(S);
  const size_t svd_per_block = sh.nblocks ? sh.svd_bytes / (size_t)sh.nblocks : 0;
  for (int i = 0; i < S; ++i) {
    Slice& w = work[i];
    w.mats.assign(mats.begin() + cut[i], mats.begin() + cut[i + 1]);
    const int64_t off = w.mats.empty() ? 0 : w.mats.front().blk0;
    int64_t nb = 0;
    for (auto& x : w.mats) {
      x.blk0 -= off;
      nb += x.s;
    }
    w.sh = sh;
    w.sh.nblocks = nb;
    w.sh.R = sh.R + off * b * b;
    w.sh.Us = sh.Us + off * b * b;
    w.sh.Vs = sh.Vs + off * b * b;
    w.sh.d = sh.d + off * b;
    w.sh.sizes = sh.sizes + off;
    w.sh.svd = static_cast<char*>(sh.svd) + off * svd_per_block;
    w.sh.svd_bytes = nb * svd_per_block;
  }
  if (use_graph && !trace_on())
    return run_recorded(st, streams, dev, res, work, mats, cut, ws, cfg, q, precision);

  // lockstep rounds streamed through the descriptor rings; the rings' slots
  // are reused only after every round a previous call enqueued (possibly on
  // another stream) has been read
  if (res.ring_used) RRF_CHECK_HIP(hipStreamWaitEvent(st, res.ring_done, 0));
  if (S == 1) {
    const int rc = run_slice(st, res.rings[0], work[0].mats, work[0].sh, cfg, q, precision);
    RRF_CHECK_HIP(hipEventRecord(res.ring_done, st));
    res.ring_used = true;
    return rc;
  }
  RRF_CHECK_HIP(hipEventRecord(res.start, st));
  for (int i = 1; i < S; ++i) RRF_CHECK_HIP(hipStreamWaitEvent(streams[i], res.start, 0));
  std::vector<std::thread> threads;
  for (int i = 0; i < S; ++i) {
    threads.emplace_back([&, i]() {
      Slice& w = work[i];
      hipError_t e = hipSetDevice(dev);  // the current device is per thread
      if (e != hipSuccess) {
        w.rc = set_hip_error(e, "hipSetDevice", __FILE__, __LINE__);
      } else if (!w.mats.empty()) {
        w.rc = run_slice(streams[i], res.rings[i], w.mats, w.sh, cfg, q, precision);
      }
      if (w.rc != RRF_OK) w.msg = rrf_last_error();
    });
  }
  for (auto& t : threads) t.join();
  // the caller's stream waits for every slice, also after a failure
  for (int i = 1; i < S; ++i) {
    RRF_CHECK_HIP(hipEventRecord(res.done[i], streams[i]));
    RRF_CHECK_HIP(hipStreamWaitEvent(st, res.done[i], 0));
  }
  RRF_CHECK_HIP(hipEventRecord(res.ring_done, st));
  res.ring_used = true;
  for (auto& w : work)
    if (w.rc != RRF_OK) return set_error(w.rc, w.msg.c_str());
  return RRF_OK;
}

int randutv_batched_release() {
  std::lock_guard<std::mutex> lk(g_ring_mu);
  int cur = 0;
  RRF_CHECK_HIP(hipGetDevice(&cur));
  for (auto& kvp : g_res) {
    DeviceRes& r = kvp.second;
    RRF_CHECK_HIP(hipSetDevice(kvp.first));
    RRF_CHECK_HIP(hipDeviceSynchronize());
    for (auto& ring : r.rings) {
      for (int s = 0; s < kSlots; ++s)
        if (ring.copied[s]) RRF_CHECK_HIP(hipEventDestroy(ring.copied[s]));
      if (ring.host) RRF_CHECK_HIP(hipHostFree(ring.host));
      if (ring.dev) RRF_CHECK_HIP(hipFree(ring.dev));
    }
    for (auto* rec : r.recs) RRF_TRY(free_recording(rec));
    r.recs.clear();
    for (int i = 0; i < kMaxSlices; ++i) {
      if (r.done[i]) RRF_CHECK_HIP(hipEventDestroy(r.done[i]));
    }
    if (r.start) RRF_CHECK_HIP(hipEventDestroy(r.start));
    if (r.ring_done) RRF_CHECK_HIP(hipEventDestroy(r.ring_done));
  }
  g_res.clear();
  RRF_CHECK_HIP(hipSetDevice(cur));
  return RRF_OK;
}

}  // namespace rrf
