// Optional per-kernel timing: a pair of HIP events around each launch of a
// kernel class, on the stream the kernel runs on, plus the algorithmic flop
// and byte counts of that launch. Off by default (one branch per launch).
// Launches on streams marked with trace_mark_stream (the streams that form
// U and V after the randUTV loop, where kernels run concurrently) are kept
// as separate classes, named with a ":UV" suffix.
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "common.hpp"
#include "trace.hpp"

namespace rrf {

namespace {

struct Record {
  int cls;
  double flops, bytes;
  hipEvent_t e0, e1;
  bool ended;  // e1 recorded (only ended records are drained)
};

struct Totals {
  int64_t launches = 0;
  double ms = 0.0, flops = 0.0, bytes = 0.0;
};

std::mutex g_mu;
bool g_on = false;
int g_only = -1;  // trace only this class index (-1: all)
std::unordered_map<int, Record> g_pending;  // by token
int g_next = 0;
std::vector<hipEvent_t> g_free;
Totals g_tot[2 * kTraceClasses];
std::vector<hipStream_t> g_marked;

const char* kNames[kTraceClasses] = {
    "dgemm_mfma_128x128_NN", "dgemm_mfma_128x128_TN", "dgemm_mfma_128x128_NT",
    "dgemm_mfma_128x128_TT", "dgemm_mfma_64x64_NN",   "dgemm_mfma_64x64_TN",
    "dgemm_mfma_64x64_NT",   "dgemm_mfma_64x64_TT",   "splitk_reduce",
    "householder_panel",     "jacobi_svd",            "gaussian",
    "elementwise",           "gemm_bf16_mfma_TN",     "dgemm_grouped_64x64",
    "dgemm_grouped_128x64",  "dgemm_grouped_128x32",  "dgemm_grouped_128x16",
    "dgemm_grouped_128x128", "gemm_x3_128x128",       "gemm_x3_64x64",
    "gemm_x6_128x128",       "gemm_x6_64x64",         "householder_panel_tree",
    "cholqr_cholesky_inverse", "cholqr_reconstruct",  "householder_panel_fallback",
};

hipEvent_t get_event() {
  if (!g_free.empty()) {
    hipEvent_t e = g_free.back();
    g_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Fold the ended records into the totals; records whose launch is still
// being enqueued by another thread stay pending.
void drain_locked() {
  for (auto it = g_pending.begin(); it != g_pending.end();) {
    Record& r = it->second;
    if (!r.ended) {
      ++it;
      continue;
    }
    float ms = 0.f;
    if (r.e0 && r.e1 && hipEventSynchronize(r.e1) == hipSuccess &&
        hipEventElapsedTime(&ms, r.e0, r.e1) == hipSuccess) {
      Totals& t = g_tot[r.cls];
      t.launches += 1;
      t.ms += ms;
      t.flops += r.flops;
      t.bytes += r.bytes;
    }
    if (r.e0) g_free.push_back(r.e0);
    if (r.e1) g_free.push_back(r.e1);
    it = g_pending.erase(it);
  }
}

}  // namespace

bool trace_on() { return g_on; }

void trace_mark_stream(hipStream_t st) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (hipStream_t m : g_marked)
    if (m == st) return;
  g_marked.push_back(st);
}

void trace_unmark_stream(hipStream_t st) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (size_t i = 0; i < g_marked.size(); ++i)
    if (g_marked[i] == st) {
      g_marked.erase(g_marked.begin() + (long)i);
      return;
    }
}

int trace_begin(hipStream_t st, int cls, double flops, double bytes) {
  if (!g_on) return -1;
  std::lock_guard<std::mutex> lk(g_mu);
  for (hipStream_t m : g_marked)
    if (m == st) cls += kTraceClasses;
  if (g_only >= 0 && cls != g_only) return -1;
  Record r{cls, flops, bytes, get_event(), get_event(), false};
  if (r.e0) (void)hipEventRecord(r.e0, st);
  const int token = g_next;
  g_next = (g_next + 1) & 0x3fffffff;
  g_pending[token] = r;
  return token;
}

void trace_end(hipStream_t st, int token) {
  if (token < 0) return;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_pending.find(token);
  if (it == g_pending.end()) return;
  if (it->second.e1) (void)hipEventRecord(it->second.e1, st);
  it->second.ended = true;
  if (g_pending.size() > 4096) drain_locked();
}

int gemm_trace_class(int tile, bool ta, bool tb) {
  return (tile == 128 ? 0 : 4) + (ta ? 1 : 0) + (tb ? 2 : 0);
}

}  // namespace rrf

using namespace rrf;

extern "C" {

int rrf_trace_enable(int on) {
  std::lock_guard<std::mutex> lk(g_mu);
  drain_locked();
  for (auto& t : g_tot) t = Totals{};
  g_on = on != 0;
  g_only = -1;
  return RRF_OK;
}

int rrf_trace_enable_class(const char* name) {
  if (name == nullptr) return set_error(-1, "name is NULL"), -1;
  const size_t len = strlen(name);
  const bool uv = len > 3 && strcmp(name + len - 3, ":UV") == 0;
  const std::string base(name, uv ? len - 3 : len);
  int cls = -1;
  for (int c = 0; c < kTraceClasses; ++c)
    if (base == kNames[c]) cls = c + (uv ? kTraceClasses : 0);
  if (cls < 0) return set_error(-1, "unknown kernel class"), -1;
  std::lock_guard<std::mutex> lk(g_mu);
  drain_locked();
  for (auto& t : g_tot) t = Totals{};
  g_on = true;
  g_only = cls;
  return RRF_OK;
}

int rrf_trace_read(rrf_trace_entry* out, int max_entries) {
  std::lock_guard<std::mutex> lk(g_mu);
  drain_locked();
  int n = 0;
  for (int c = 0; c < 2 * kTraceClasses && n < max_entries; ++c) {
    if (g_tot[c].launches == 0) continue;
    rrf_trace_entry& e = out[n++];
    memset(&e, 0, sizeof e);
    strncpy(e.name, kNames[c % kTraceClasses], sizeof e.name - 4);
    if (c >= kTraceClasses) strncat(e.name, ":UV", sizeof e.name - 1 - strlen(e.name));
    e.launches = g_tot[c].launches;
    e.ms = g_tot[c].ms;
    e.flops = g_tot[c].flops;
    e.bytes = g_tot[c].bytes;
  }
  return n;
}

}  // extern "C"
