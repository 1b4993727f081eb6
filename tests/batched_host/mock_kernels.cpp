// Test double for the device side of the batched randUTV driver
// (randutv_batched.hip), built with the host compiler: the HIP runtime calls
// the driver makes are stubbed, and each batched kernel is replaced by a
// plain CPU loop over its descriptors with the kernel's contract (problem p,
// tile / column group / block -> one "workgroup"). Every access is checked:
//  * inside an allocation made through the stubbed hipMalloc (workspace,
//    matrices, descriptor slots);
//  * no element written by one workgroup and read or written by another
//    within one launch (the kernels have no ordering between workgroups);
//  * device memory starts as NaN, so a read of anything not written first
//    poisons the results.
// A grouped-GEMM tile reads all its operands before it stores, as the
// kernel's epilogue does, so a product may write over an operand that only
// its own workgroup reads.
// Used only by tests/test_batched_planner.py; nothing here runs on a GPU.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <unordered_map>
#include <vector>
#include <algorithm>
#include <functional>

#include "batched.hpp"
#include "common.hpp"
#include "context.hpp"
#include "kernels.hpp"

#include <mutex>
static std::recursive_mutex g_kmu;  // kernels emulated one at a time
static std::map<uintptr_t, size_t> g_alloc;  // base -> bytes
static long g_errors = 0;
static const char* g_launch = "";

static void fail(const char* what, const void* p) {
  if (g_errors < 20) fprintf(stderr, "MOCK ERROR [%s]: %s at %p\n", g_launch, what, p);
  ++g_errors;
}

static bool inb(const void* p, size_t bytes) {
  uintptr_t a = (uintptr_t)p;
  auto it = g_alloc.upper_bound(a);
  if (it == g_alloc.begin()) return false;
  --it;
  return a >= it->first && a + bytes <= it->first + it->second;
}

// per-launch race tracking at element granularity
static std::unordered_map<const void*, long> g_w, g_r;
static void begin_launch(const char* name) {
  g_launch = name;
  g_w.clear();
  g_r.clear();
}
static double rd(const double* p, long wg) {
  if (!inb(p, 8)) { fail("read out of bounds", p); return NAN; }
  auto it = g_w.find(p);
  if (it != g_w.end() && it->second != wg) fail("read of another workgroup's write", p);
  auto jt = g_r.find(p);
  if (jt == g_r.end()) g_r[p] = wg;
  else if (jt->second != wg) jt->second = -2;
  return *p;
}
static void wr(double* p, double v, long wg) {
  if (!inb(p, 8)) { fail("write out of bounds", p); return; }
  auto it = g_w.find(p);
  if (it != g_w.end() && it->second != wg) fail("write-write race", p);
  g_w[p] = wg;
  auto jt = g_r.find(p);
  if (jt != g_r.end() && jt->second != wg) fail("write of another workgroup's read", p);
  *p = v;
}

extern "C" {
long mock_errors() { return g_errors; }
void* mock_malloc(size_t bytes) {
  std::lock_guard<std::recursive_mutex> lk_(g_kmu);
  void* p = aligned_alloc(256, (bytes + 255) & ~(size_t)255);
  double* d = (double*)p;
  for (size_t i = 0; i < bytes / 8; ++i) d[i] = NAN;
  g_alloc[(uintptr_t)p] = bytes;
  return p;
}
void mock_free(void* p) {
  g_alloc.erase((uintptr_t)p);
  free(p);
}
}

hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned int) { *p = malloc(bytes); return hipSuccess; }
hipError_t hipHostFree(void* p) { free(p); return hipSuccess; }
hipError_t hipMalloc(void** p, size_t bytes) { *p = mock_malloc(bytes); return hipSuccess; }
hipError_t hipFree(void* p) { if (p) mock_free(p); return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { *e = (hipEvent_t)malloc(8); return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventDestroy(hipEvent_t e) { free(e); return hipSuccess; }
// Stream capture: operations enqueued on the capturing stream are kept as
// closures in the graph (descriptors and data are read when the graph is
// launched, as on the device) instead of running at once.
struct MockGraph {
  std::vector<std::function<void()>> ops;
};
static hipStream_t g_capture = nullptr;
static MockGraph* g_captured = nullptr;
static long g_graph_launches = 0;
static bool mock_capturing(hipStream_t st) { return st != nullptr && st == g_capture; }
static void mock_defer(std::function<void()> f) { g_captured->ops.push_back(std::move(f)); }
#define MOCK_DEFER(st, call)                   \
  if (mock_capturing(st)) {                    \
    mock_defer([=]() { (void)(call); });       \
    return RRF_OK;                             \
  }

hipError_t hipStreamBeginCapture(hipStream_t st, hipStreamCaptureMode) {
  if (g_capture) return hipErrorIllegalState;
  g_capture = st;
  g_captured = new MockGraph();
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t st, hipGraph_t* g) {
  if (st != g_capture) return hipErrorIllegalState;
  *g = reinterpret_cast<hipGraph_t>(g_captured);
  g_capture = nullptr;
  g_captured = nullptr;
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
  *e = reinterpret_cast<hipGraphExec_t>(new MockGraph(*reinterpret_cast<MockGraph*>(g)));
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
  delete reinterpret_cast<MockGraph*>(g);
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t e) {
  delete reinterpret_cast<MockGraph*>(e);
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t) {
  ++g_graph_launches;
  for (auto& f : reinterpret_cast<MockGraph*>(e)->ops) f();
  return hipSuccess;
}
extern "C" long mock_graph_launches() { return g_graph_launches; }

hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind k, hipStream_t st) {
  if (mock_capturing(st)) {
    mock_defer([=]() { (void)hipMemcpyAsync(d, s, n, k, nullptr); });
    return hipSuccess;
  }
  if (!inb(d, n) && g_alloc.size() && k != hipMemcpyDeviceToHost) fail("copy to unallocated memory", d);
  memcpy(d, s, n);
  return hipSuccess;
}
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) { memcpy(d, s, n); return hipSuccess; }
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { *s = (hipStream_t)malloc(8); return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t s) { free(s); return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "mock"; }

namespace rrf {

// The error helpers are weak: a build that links the library's own
// (api.hip) takes those.
__attribute__((weak)) int set_hip_error(hipError_t, const char* what, const char* file, int line) {
  fprintf(stderr, "hip error %s %s:%d\n", what, file, line);
  return RRF_E_HIP;
}
__attribute__((weak)) int set_error(int status, const char* msg) {
  fprintf(stderr, "error %d: %s\n", status, msg);
  return status;
}

extern "C" __attribute__((weak)) const char* rrf_last_error(void) { return "mock"; }
bool trace_on() { return false; }
void trace_unmark_stream(hipStream_t) {}
// The driver runs slices 1 and 2 on the context's side streams.
int device_context(DeviceContext** out) {
  static DeviceContext* c = nullptr;
  if (!c) {
    c = new DeviceContext();
    for (auto& st : c->side) (void)hipStreamCreateWithFlags(&st, 0);
  }
  *out = c;
  return RRF_OK;
}
int fill_u32(hipStream_t, unsigned* p, int64_t count, unsigned v) {
  for (int64_t i = 0; i < count; ++i) p[i] = v;
  return RRF_OK;
}

int gemm_grouped(hipStream_t st_, bool ta, bool tb, int tile, bool vec, const GemmDesc* d,
                 const int* prefix, int count, int64_t total_tiles, double) {
  MOCK_DEFER(st_, gemm_grouped(nullptr, ta, tb, tile, vec, d, prefix, count, total_tiles, 0.0));
  std::lock_guard<std::recursive_mutex> lk_(g_kmu);
  if (vec)
    for (int p = 0; p < count; ++p)
      if ((uintptr_t)d[p].A % 16 || (uintptr_t)d[p].B % 16 || d[p].lda % 2 || d[p].ldb % 2)
        fail("vec with unaligned operand", nullptr);
  begin_launch("gemm_grouped");
  if (prefix[0] != 0 || prefix[count] != total_tiles) fail("prefix ends", nullptr);
  const int64_t R = tile_rows(tile), Cc = tile_cols(tile);
  for (int p = 0; p < count; ++p) {
    const GemmDesc g = d[p];
    const int64_t tm = (g.M + R - 1) / R, tiles = tm * ((g.N + Cc - 1) / Cc);
    if (prefix[p + 1] - prefix[p] != tiles) fail("prefix count", nullptr);
    for (int64_t t = 0; t < tiles; ++t) {
      const long wg = prefix[p] + t;
      const int64_t i0 = (t % tm) * R, j0 = (t / tm) * Cc;
      const int64_t i1 = std::min(i0 + R, g.M), j1 = std::min(j0 + Cc, g.N);
      // the kernel reads all of a tile's operands (and C for beta != 0)
      // before its epilogue stores, so C may be the A or B it reads
      std::vector<double> tile((size_t)(i1 - i0) * (j1 - j0));
      for (int64_t i = i0; i < i1; ++i)
        for (int64_t j = j0; j < j1; ++j) {
          double s = 0.0;
          for (int64_t k = 0; k < g.K; ++k) {
            const double a = ta ? rd(g.A + k + i * g.lda, wg) : rd(g.A + i + k * g.lda, wg);
            const double b = tb ? rd(g.B + j + k * g.ldb, wg) : rd(g.B + k + j * g.ldb, wg);
            s += a * b;
          }
          double c = g.alpha * s;
          if (g.beta != 0.0) c += g.beta * rd(g.C + i + j * g.ldc, wg);
          tile[(size_t)(i - i0) + (size_t)(j - j0) * (i1 - i0)] = c;
        }
      for (int64_t i = i0; i < i1; ++i)
        for (int64_t j = j0; j < j1; ++j)
          wr(g.C + i + j * g.ldc, tile[(size_t)(i - i0) + (size_t)(j - j0) * (i1 - i0)], wg);
    }
  }
  return RRF_OK;
}

int elem_batched(hipStream_t st_, const ElemDesc* d, int count, int64_t max_cols) {
  MOCK_DEFER(st_, elem_batched(nullptr, d, count, max_cols));
  std::lock_guard<std::recursive_mutex> lk_(g_kmu);
  begin_launch("elem");
  for (int p = 0; p < count; ++p) {
    const ElemDesc e = d[p];
    if (e.cols > max_cols) fail("cols beyond grid", nullptr);
    for (int64_t c = 0; c < e.cols; ++c) {
      const long wg = (long)p * 1000000 + c / 8;
      for (int64_t r = 0; r < e.rows; ++r) {
        double v;
        switch (e.op) {
          case kElemFill: v = e.v; break;
          case kElemCopy: v = rd(e.S + r + c * e.lds, wg); break;
          case kElemDiag: v = (r == c) ? rd(e.S + c, wg) : 0.0; break;
          default: v = (r == c) ? 1.0 : 0.0;
        }
        wr(e.X + r + c * e.ld, v, wg);
      }
    }
  }
  return RRF_OK;
}

static uint64_t mulhi(uint64_t a, uint64_t b) { return (uint64_t)(((unsigned __int128)a * b) >> 64); }

// The sketch generator from its definition (Philox4x64-10 with the key
// schedule and multipliers of Salmon et al., SC'11; uniforms from the top 53
// bits; Box-Muller), so that the emulated factorization uses the same G as
// the oracle.
static void gauss4(uint64_t seed, uint64_t sid, uint64_t gr, uint64_t c, double v[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  uint64_t x0 = gr, x1 = c, x2 = 0, x3 = 0, k0 = seed, k1 = sid;
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += W0; k1 += W1; }
    const uint64_t hi0 = mulhi(M0, x0), lo0 = M0 * x0, hi1 = mulhi(M1, x2), lo1 = M1 * x2;
    const uint64_t y0 = hi1 ^ x1 ^ k0, y2 = hi0 ^ x3 ^ k1;
    x0 = y0; x1 = lo1; x2 = y2; x3 = lo0;
  }
  const double ua = ((double)(x0 >> 11) + 1.0) * 0x1p-53, va = (double)(x1 >> 11) * 0x1p-53;
  const double ub = ((double)(x2 >> 11) + 1.0) * 0x1p-53, vb = (double)(x3 >> 11) * 0x1p-53;
  const double ra = sqrt(-2.0 * log(ua)), rb = sqrt(-2.0 * log(ub));
  const double tw = 6.283185307179586;
  v[0] = ra * cos(tw * va); v[1] = ra * sin(tw * va);
  v[2] = rb * cos(tw * vb); v[3] = rb * sin(tw * vb);
}

int gauss_batched(hipStream_t st_, const GaussDesc* d, int count, int64_t max_elems) {
  MOCK_DEFER(st_, gauss_batched(nullptr, d, count, max_elems));
  std::lock_guard<std::recursive_mutex> lk_(g_kmu);
  begin_launch("gauss");
  for (int p = 0; p < count; ++p) {
    const GaussDesc g = d[p];
    if (g.rows * g.cols > max_elems) fail("elems beyond grid", nullptr);
    for (int64_t c = 0; c < g.cols; ++c)
      for (int64_t gr = 0; gr < (g.rows + 3) / 4; ++gr) {
        double v[4];
        gauss4(g.seed, g.sid, gr, c, v);
        for (int k = 0; k < 4; ++k)
          if (gr * 4 + k < g.rows) wr(g.out + gr * 4 + k + c * g.ld, v[k], p);
      }
  }
  return RRF_OK;
}

// --- the mixed sketch's batched kernels ------------------------------------

static void chk(const void* p, size_t bytes) {
  if (!inb(p, bytes)) fail("access out of bounds", p);
}
static uint16_t bf16_of_f64(double x) {
  if (x == 0.0) return 0;
  int lead = ilogb(x);
  if (lead < -126) lead = -126;
  const double q = rint(scalbn(x, 7 - lead));
  float r = (float)scalbn(q, lead - 7);
  uint32_t u;
  memcpy(&u, &r, 4);
  return (uint16_t)(u >> 16);
}
static uint16_t bf16_of_f32(float x) {
  uint32_t u;
  memcpy(&u, &x, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
static float f32_of_bf16(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}
static double pow2s(double m) {
  if (!(m > 0.0)) return 1.0;
  int e;
  frexp(m, &e);
  return ldexp(1.0, -e);
}

int maxabs_batched(hipStream_t st_, const MaxDesc* d, int count, int64_t max_rows) {
  MOCK_DEFER(st_, maxabs_batched(nullptr, d, count, max_rows));
  std::lock_guard<std::recursive_mutex> lk_(g_kmu);
  begin_launch("maxabs_batched");
  for (int p = 0; p < count; ++p) {
    if (d[p].rows > max_rows) fail("rows beyond grid", nullptr);
    double m = 0.0;
    for (int64_t c = 0; c < d[p].cols; ++c)
      for (int64_t r = 0; r < d[p].rows; ++r) m = std::max(m, fabs(rd(d[p].X + r + c * d[p].ld, p)));
    chk(d[p].word, 8);
    unsigned long long bits;
    memcpy(&bits, &m, 8);
    if (bits > *d[p].word) *d[p].word = bits;
  }
  return RRF_OK;
}

int to_bf16_batched(hipStream_t st_, const Bf16Desc* d, int count, int64_t max_tiles) {
  MOCK_DEFER(st_, to_bf16_batched(nullptr, d, count, max_tiles));
  std::lock_guard<std::recursive_mutex> lk_(g_kmu);
  begin_launch("to_bf16_batched");
  for (int p = 0; p < count; ++p) {
    const Bf16Desc e = d[p];
    if (bf16_conv_tiles(e.rows, e.cols, e.ldo, e.outT ? e.ldot : 0) > max_tiles)
      fail("tiles beyond grid", nullptr);
    double s = 1.0;
    if (e.word) {
      chk(e.word, 8);
      double m;
      memcpy(&m, e.word, 8);
      s = pow2s(m);
    }
    for (int64_t c = 0; c < e.cols; ++c)
      for (int64_t r = 0; r < std::max(e.rows, e.ldo); ++r) {
        const uint16_t v = r < e.rows ? bf16_of_f64(rd(e.X + r + c * e.ld, p) * s) : 0;
        if (r < e.ldo) { chk(e.out + r + c * e.ldo, 2); e.out[r + c * e.ldo] = v; }
        if (e.outT && r < e.rows) { chk(e.outT + c + r * e.ldot, 2); e.outT[c + r * e.ldot] = v; }
      }
    if (e.outT)
      for (int64_t r = 0; r < e.rows; ++r)
        for (int64_t c = e.cols; c < e.ldot; ++c) { chk(e.outT + c + r * e.ldot, 2); e.outT[c + r * e.ldot] = 0; }
  }
  return RRF_OK;
}

int gemm_bf16_grouped(hipStream_t st_, const Bf16GemmDesc* d, const int* prefix, int count,
                      int64_t total_tiles, double) {
  MOCK_DEFER(st_, gemm_bf16_grouped(nullptr, d, prefix, count, total_tiles, 0.0));
  std::lock_guard<std::recursive_mutex> lk_(g_kmu);
  begin_launch("gemm_bf16_grouped");
  if (prefix[0] != 0 || prefix[count] != total_tiles) fail("prefix ends", nullptr);
  for (int p = 0; p < count; ++p) {
    const Bf16GemmDesc g = d[p];
    if (prefix[p + 1] - prefix[p] != bf16_group_tiles(g.M, g.N)) fail("prefix count", nullptr);
    if (g.lda % 8 || g.ldb % 8 || (uintptr_t)g.A % 16 || (uintptr_t)g.B % 16)
      fail("bf16 operand alignment", nullptr);
    const int64_t kpad = (g.K + 7) / 8 * 8;
    for (int64_t i = 0; i < g.M; ++i)
      for (int64_t j = 0; j < g.N; ++j) {
        float acc = 0.f;
        for (int64_t k = 0; k < kpad; ++k) {  // the kernel reads the zero padding too
          chk(g.A + k + i * g.lda, 2);
          chk(g.B + k + j * g.ldb, 2);
          acc += f32_of_bf16(g.A[k + i * g.lda]) * f32_of_bf16(g.B[k + j * g.ldb]);
        }
        if (g.out64) wr(g.out64 + i + j * g.ld64, (double)acc, p);
        else { chk(g.P + i + j * g.ldp, 4); g.P[i + j * g.ldp] = acc; }
      }
  }
  return RRF_OK;
}

int round_columns_batched(hipStream_t st_, const RoundDesc* d, int count, int64_t max_cols) {
  MOCK_DEFER(st_, round_columns_batched(nullptr, d, count, max_cols));
  std::lock_guard<std::recursive_mutex> lk_(g_kmu);
  begin_launch("round_columns_batched");
  for (int p = 0; p < count; ++p) {
    const RoundDesc e = d[p];
    if (e.N > max_cols) fail("cols beyond grid", nullptr);
    for (int64_t n = 0; n < e.N; ++n) {
      float m = 0.f;
      for (int64_t i = 0; i < e.M; ++i) { chk(e.P + i + n * e.ldp, 4); m = std::max(m, fabsf(e.P[i + n * e.ldp])); }
      const float s = (float)pow2s((double)m);
      for (int64_t i = 0; i < e.ld16; ++i) {
        chk(e.out16 + i + n * e.ld16, 2);
        e.out16[i + n * e.ld16] = i < e.M ? bf16_of_f32(e.P[i + n * e.ldp] * s) : 0;
      }
    }
  }
  return RRF_OK;
}

int64_t panel_wg_max_rows(int k) {
  if (k < 1 || k > 64) return 0;
  int K = 1;
  while (K < k) K <<= 1;
  return 512 * std::max(1, std::min(32 / K, 8));
}

int panel_wg_batched(hipStream_t st_, const PanelDesc* d, int count, int k, int64_t max_rows) {
  MOCK_DEFER(st_, panel_wg_batched(nullptr, d, count, k, max_rows));
  std::lock_guard<std::recursive_mutex> lk_(g_kmu);
  begin_launch("panel");
  if (k < 1 || k > 64 || max_rows > panel_wg_max_rows(k)) return set_error(5, "panel shape");
  for (int p = 0; p < count; ++p) {
    const PanelDesc a = d[p];
    const int64_t M = a.M;
    if (M > max_rows) fail("rows beyond max", nullptr);
    if (M < k) fail("panel with M < k", nullptr);
    std::vector<double> X(M * k), T(k * k, 0.0);
    for (int64_t c = 0; c < k; ++c)
      for (int64_t r = 0; r < M; ++r) X[r + c * M] = rd(a.P + r + c * a.ldp, p);
    if (a.zero)
      for (int64_t c = 0; c < k; ++c)
        for (int64_t r = 0; r < M; ++r) wr(a.zero + r + c * a.ldz, 0.0, p);
    std::vector<double> tau(k), Rm(k * k, 0.0);
    for (int j = 0; j < k; ++j) {
      double alpha = X[j + j * M], xn2 = 0.0;
      for (int64_t r = j + 1; r < M; ++r) xn2 += X[r + j * M] * X[r + j * M];
      double t, beta, scal;
      if (xn2 == 0.0) { t = 0.0; beta = alpha; scal = 0.0; }
      else {
        const double nrm = sqrt(alpha * alpha + xn2);
        beta = -copysign(nrm, alpha);
        t = (beta - alpha) / beta;
        scal = 1.0 / (alpha - beta);
      }
      tau[j] = t;
      X[j + j * M] = 1.0;
      for (int64_t r = j + 1; r < M; ++r) X[r + j * M] *= scal;
      Rm[j + j * k] = beta;
      for (int c = j + 1; c < k; ++c) {  // H_j^T applied to column c
        double s = 0.0;
        for (int64_t r = j; r < M; ++r) s += X[r + j * M] * X[r + c * M];
        for (int64_t r = j; r < M; ++r) X[r + c * M] -= t * s * X[r + j * M];
        Rm[j + c * k] = X[j + c * M];
      }
      // T(0:j, j) = -tau_j T(0:j, 0:j) V(:, 0:j)^T v_j
      std::vector<double> w(j, 0.0);
      for (int i = 0; i < j; ++i) {
        double s = 0.0;
        for (int64_t r = j; r < M; ++r) s += X[r + i * M] * X[r + j * M];
        w[i] = s;
      }
      for (int i = 0; i < j; ++i) {
        double s = 0.0;
        for (int c = i; c < j; ++c) s += T[i + c * k] * w[c];
        T[i + j * k] = -t * s;
      }
      T[j + j * k] = t;
    }
    for (int j = 0; j < k; ++j) wr(a.tau + j, tau[j], p);
    for (int c = 0; c < k; ++c)
      for (int i = 0; i < k; ++i) {
        wr(a.Tf + i + c * a.ldt, i <= c ? T[i + c * k] : 0.0, p);
        if (a.R) wr(a.R + i + c * a.ldr, i <= c ? Rm[i + c * k] : 0.0, p);
      }
    for (int c = 0; c < k; ++c)
      for (int64_t r = 0; r < M; ++r)
        wr(a.W + r + c * a.ldw, r < c ? 0.0 : (r == c ? 1.0 : X[r + c * M]), p);
  }
  return RRF_OK;
}

size_t block_svd_work_bytes(int k) { return (size_t)2 * k * k * 8 + 256; }

int block_svd_sized(hipStream_t st_, int count, int kmax, const int* sizes, const double* B,
                    int64_t ldb, int64_t stride, double* Us, double* d, int64_t dstride,
                    double* Vs, void* work, size_t work_bytes, int* status) {
  MOCK_DEFER(st_, block_svd_sized(nullptr, count, kmax, sizes, B, ldb, stride, Us, d, dstride, Vs,
                                  work, work_bytes, status));
  std::lock_guard<std::recursive_mutex> lk_(g_kmu);
  begin_launch("svd");
  (void)work; (void)work_bytes; (void)status;
  for (int blk = 0; blk < count; ++blk) {
    const int k = sizes[blk];
    if (k < 1 || k > kmax) fail("bad block size", nullptr);
    std::vector<double> A(k * k), V(k * k, 0.0);
    for (int j = 0; j < k; ++j) {
      V[j + j * k] = 1.0;
      for (int i = 0; i < k; ++i) A[i + j * k] = rd(B + blk * stride + i + j * ldb, blk);
    }
    for (int sweep = 0; sweep < 60; ++sweep) {
      bool rot = false;
      for (int p = 0; p < k; ++p)
        for (int q = p + 1; q < k; ++q) {
          double app = 0, aqq = 0, apq = 0;
          for (int r = 0; r < k; ++r) {
            app += A[r + p * k] * A[r + p * k];
            aqq += A[r + q * k] * A[r + q * k];
            apq += A[r + p * k] * A[r + q * k];
          }
          if (apq == 0.0 || fabs(apq) <= 1e-15 * sqrt(app * aqq)) continue;
          rot = true;
          const double zeta = (aqq - app) / (2 * apq);
          const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1 + zeta * zeta));
          const double c = 1 / sqrt(1 + t * t), s = c * t;
          for (int r = 0; r < k; ++r) {
            double x = A[r + p * k], y = A[r + q * k];
            A[r + p * k] = c * x - s * y;
            A[r + q * k] = s * x + c * y;
            x = V[r + p * k]; y = V[r + q * k];
            V[r + p * k] = c * x - s * y;
            V[r + q * k] = s * x + c * y;
          }
        }
      if (!rot) break;
    }
    std::vector<double> nrm(k);
    std::vector<int> perm(k);
    for (int j = 0; j < k; ++j) {
      double s = 0;
      for (int r = 0; r < k; ++r) s += A[r + j * k] * A[r + j * k];
      nrm[j] = sqrt(s);
      perm[j] = j;
    }
    std::stable_sort(perm.begin(), perm.end(), [&](int x, int y) { return nrm[x] > nrm[y]; });
    std::vector<double> U(k * k, 0.0);
    for (int jj = 0; jj < k; ++jj) {
      const int j = perm[jj];
      for (int r = 0; r < k; ++r) U[r + jj * k] = nrm[j] > 0 ? A[r + j * k] / nrm[j] : 0.0;
      if (!(nrm[j] > 1e-300)) {  // completion
        for (int e = 0; e < k; ++e) {
          std::vector<double> u(k, 0.0);
          u[e] = 1.0;
          for (int c = 0; c < jj; ++c) {
            double s = 0;
            for (int r = 0; r < k; ++r) s += U[r + c * k] * u[r];
            for (int r = 0; r < k; ++r) u[r] -= s * U[r + c * k];
          }
          double s = 0;
          for (int r = 0; r < k; ++r) s += u[r] * u[r];
          if (s > 0.5) {
            for (int r = 0; r < k; ++r) U[r + jj * k] = u[r] / sqrt(s);
            break;
          }
        }
      }
      wr(d + blk * dstride + jj, nrm[j], blk);
      for (int r = 0; r < k; ++r) {
        wr(Us + blk * stride + r + jj * k, U[r + jj * k], blk);
        wr(Vs + blk * stride + r + jj * k, V[r + j * k], blk);
      }
    }
  }
  return RRF_OK;
}

}  // namespace rrf
