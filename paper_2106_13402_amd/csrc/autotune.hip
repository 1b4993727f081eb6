// Autotuner of the batched randUTV call: per bucket of matrix sizes it times
// candidate configurations (block size b, the grouped GEMM's tile shapes, the
// panel leaf width) on a synthetic batch of that bucket and keeps the
// fastest. Tables are keyed by (architecture, precision) and kept in memory;
// they are written to and read from a JSON cache. With b = 0 the batched
// call takes each matrix's configuration from the table of the current
// device's architecture and its precision (batched_config); without one it
// uses the built-in rule.
//
// Cache format (one object):
//   {"format": "rrf-batched-tune-1",
//    "tables": [{"arch": "gfx950", "precision": 0, "q": 1, "count": 256,
//                "buckets": [{"nmin": 1, "nmax": 64, "b": 16, "tile_mask": 31,
//                             "leaf": 0, "ms": 1.25, "candidates": 12}, ...]}]}
// q and count record the workload the table was timed on; lookups use the
// architecture, the precision and the bucket only.
#include <dlfcn.h>

#include <algorithm>
#include <cctype>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "batched.hpp"
#include "common.hpp"
#include "driver.hpp"
#include "kernels.hpp"

namespace rrf {

namespace {

struct Bucket {
  int64_t nmin, nmax;
  BatchedCfg cfg;
  double ms;
  int candidates;
};
struct Table {
  std::string arch;
  int precision = 0;
  int q = 1;
  int64_t count = 0;
  std::vector<Bucket> buckets;
};

std::mutex g_mu;
std::vector<Table> g_tables;
bool g_default_tried = false;

// ---- a small JSON reader (objects, arrays, numbers, strings, literals) ----
struct Json {
  enum Kind { kNull, kBool, kNum, kStr, kArr, kObj } kind = kNull;
  double num = 0.0;
  bool boolean = false;
  std::string str;
  std::vector<Json> arr;
  std::map<std::string, Json> obj;
  const Json* get(const char* k) const {
    auto it = obj.find(k);
    return it == obj.end() ? nullptr : &it->second;
  }
};

struct Parser {
  const char* p;
  const char* end;
  bool ok = true;
  void ws() {
    while (p < end && std::isspace((unsigned char)*p)) ++p;
  }
  bool lit(const char* s) {
    const size_t n = strlen(s);
    if ((size_t)(end - p) >= n && memcmp(p, s, n) == 0) {
      p += n;
      return true;
    }
    return false;
  }
  std::string string() {
    std::string out;
    ++p;  // opening quote
    while (p < end && *p != '"') {
      if (*p == '\\' && p + 1 < end) ++p;  // escapes are taken literally
      out.push_back(*p++);
    }
    if (p >= end) ok = false;
    else ++p;
    return out;
  }
  Json value(int depth = 0) {
    Json v;
    ws();
    if (p >= end || depth > 32) {
      ok = false;
      return v;
    }
    if (*p == '{') {
      v.kind = Json::kObj;
      ++p;
      ws();
      if (p < end && *p == '}') {
        ++p;
        return v;
      }
      while (ok) {
        ws();
        if (p >= end || *p != '"') {
          ok = false;
          break;
        }
        std::string k = string();
        ws();
        if (p >= end || *p != ':') {
          ok = false;
          break;
        }
        ++p;
        v.obj[k] = value(depth + 1);
        ws();
        if (p < end && *p == ',') {
          ++p;
          continue;
        }
        if (p < end && *p == '}') {
          ++p;
          break;
        }
        ok = false;
      }
    } else if (*p == '[') {
      v.kind = Json::kArr;
      ++p;
      ws();
      if (p < end && *p == ']') {
        ++p;
        return v;
      }
      while (ok) {
        v.arr.push_back(value(depth + 1));
        ws();
        if (p < end && *p == ',') {
          ++p;
          continue;
        }
        if (p < end && *p == ']') {
          ++p;
          break;
        }
        ok = false;
      }
    } else if (*p == '"') {
      v.kind = Json::kStr;
      v.str = string();
    } else if (lit("true")) {
      v.kind = Json::kBool;
      v.boolean = true;
    } else if (lit("false")) {
      v.kind = Json::kBool;
    } else if (lit("null")) {
      v.kind = Json::kNull;
    } else {
      char* e = nullptr;
      v.kind = Json::kNum;
      v.num = strtod(p, &e);
      if (e == p) ok = false;
      p = e;
    }
    return v;
  }
};

bool num_field(const Json& o, const char* k, double* out) {
  const Json* v = o.get(k);
  if (!v || v->kind != Json::kNum) return false;
  *out = v->num;
  return true;
}

// Integer field `k` of `o`. Absent: *out keeps its value and the result is
// !required. Present: it must be a whole number in [lo, hi] (|lo|, |hi| at
// most 2^53, so both are exact doubles); NaN, infinities, fractions and
// values out of range fail, and the conversion is always defined.
bool int_field(const Json& o, const char* k, int64_t lo, int64_t hi, bool required,
               int64_t* out) {
  const Json* v = o.get(k);
  if (!v) return !required;
  if (v->kind != Json::kNum) return false;
  const double d = v->num;
  if (!std::isfinite(d) || d != std::floor(d) || d < (double)lo || d > (double)hi) return false;
  *out = (int64_t)d;
  return true;
}

constexpr int64_t kIntLo = INT32_MIN, kIntHi = INT32_MAX;
constexpr int64_t kWhole = int64_t(1) << 53;

bool cfg_valid(const BatchedCfg& c) {
  return c.b >= 1 && c.b <= 64 && (c.tile_mask & ~kTileMaskAll) == 0 && c.leaf >= 0 && c.leaf <= 64;
}

// Tables of a cache text; false (and nothing) when it does not parse or a
// bucket is invalid.
bool parse_tables(const std::string& text, std::vector<Table>* out) {
  Parser ps{text.data(), text.data() + text.size()};
  Json root = ps.value();
  ps.ws();
  if (!ps.ok || ps.p != ps.end || root.kind != Json::kObj) return false;
  const Json* fmt = root.get("format");
  if (!fmt || fmt->kind != Json::kStr || fmt->str != "rrf-batched-tune-1") return false;
  const Json* tabs = root.get("tables");
  if (!tabs || tabs->kind != Json::kArr) return false;
  std::vector<Table> res;
  for (const auto& t : tabs->arr) {
    if (t.kind != Json::kObj) return false;
    Table tb;
    const Json* arch = t.get("arch");
    int64_t prec = 0, q = 1, count = 0;
    if (!arch || arch->kind != Json::kStr || !int_field(t, "precision", kIntLo, kIntHi, true, &prec) ||
        !int_field(t, "q", kIntLo, kIntHi, false, &q) ||
        !int_field(t, "count", -kWhole, kWhole, false, &count))
      return false;
    tb.arch = arch->str;
    tb.precision = (int)prec;
    tb.q = (int)q;
    tb.count = count;
    const Json* bs = t.get("buckets");
    if (!bs || bs->kind != Json::kArr) return false;
    for (const auto& bj : bs->arr) {
      int64_t nmin = 0, nmax = 0, b = 0, mask = kTileMaskAll, leaf = 0, cand = 0;
      double ms = 0;
      if (bj.kind != Json::kObj || !int_field(bj, "nmin", -kWhole, kWhole, true, &nmin) ||
          !int_field(bj, "nmax", -kWhole, kWhole, true, &nmax) ||
          !int_field(bj, "b", -kWhole, kWhole, true, &b) ||
          !int_field(bj, "tile_mask", kIntLo, kIntHi, false, &mask) ||
          !int_field(bj, "leaf", kIntLo, kIntHi, false, &leaf) ||
          !int_field(bj, "candidates", kIntLo, kIntHi, false, &cand))
        return false;
      num_field(bj, "ms", &ms);
      Bucket bk{nmin, nmax, BatchedCfg{b, (int)mask, (int)leaf}, ms, (int)cand};
      if (bk.nmin < 1 || bk.nmax < bk.nmin || !cfg_valid(bk.cfg)) return false;
      tb.buckets.push_back(bk);
    }
    res.push_back(std::move(tb));
  }
  *out = std::move(res);
  return true;
}

std::string format_tables(const std::vector<Table>& tabs) {
  std::string s = "{\"format\": \"rrf-batched-tune-1\",\n \"tables\": [";
  char buf[512];
  for (size_t i = 0; i < tabs.size(); ++i) {
    const Table& t = tabs[i];
    snprintf(buf, sizeof buf,
             "%s\n  {\"arch\": \"%s\", \"precision\": %d, \"q\": %d, \"count\": %lld,\n"
             "   \"buckets\": [",
             i ? "," : "", t.arch.c_str(), t.precision, t.q, (long long)t.count);
    s += buf;
    for (size_t k = 0; k < t.buckets.size(); ++k) {
      const Bucket& b = t.buckets[k];
      snprintf(buf, sizeof buf,
               "%s\n    {\"nmin\": %lld, \"nmax\": %lld, \"b\": %lld, \"tile_mask\": %d, "
               "\"leaf\": %d, \"ms\": %.4f, \"candidates\": %d}",
               k ? "," : "", (long long)b.nmin, (long long)b.nmax, (long long)b.cfg.b,
               b.cfg.tile_mask, b.cfg.leaf, b.ms, b.candidates);
      s += buf;
    }
    s += "]}";
  }
  s += "]}\n";
  return s;
}

bool read_file(const char* path, std::string* out) {
  FILE* f = fopen(path, "rb");
  if (!f) return false;
  std::string s;
  char buf[4096];
  size_t n;
  while ((n = fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, n);
  fclose(f);
  *out = std::move(s);
  return true;
}

// Replace the tables of the same (arch, precision) by those in `tabs`.
void merge_tables(const std::vector<Table>& tabs) {
  for (const auto& t : tabs) {
    auto it = std::find_if(g_tables.begin(), g_tables.end(), [&](const Table& x) {
      return x.arch == t.arch && x.precision == t.precision;
    });
    if (it != g_tables.end()) *it = t;
    else g_tables.push_back(t);
  }
}

// The default cache: $RRF_TUNE_CACHE when set (empty: none), else
// tuning/batched.json beside the library.
void load_default_locked() {
  if (g_default_tried) return;
  g_default_tried = true;
  std::string path;
  if (const char* env = getenv("RRF_TUNE_CACHE")) {
    path = env;
  } else {
    Dl_info info;
    if (dladdr(reinterpret_cast<void*>(&load_default_locked), &info) && info.dli_fname) {
      std::string lib = info.dli_fname;
      const size_t slash = lib.rfind('/');
      path = (slash == std::string::npos ? std::string(".") : lib.substr(0, slash)) +
             "/tuning/batched.json";
    }
  }
  std::string text;
  std::vector<Table> tabs;
  if (!path.empty() && read_file(path.c_str(), &text) && parse_tables(text, &tabs))
    merge_tables(tabs);
}

// Architecture name of the current device (gcnArchName up to the first ':'),
// empty without a device. The properties are queried once per device: a
// batched call with b = 0 looks up every matrix's configuration, and a
// property query per matrix would cost the host thousands of queries per call.
std::mutex g_arch_mu;
std::map<int, std::string> g_arch;

std::string current_arch() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return "";
  }
  {
    std::lock_guard<std::mutex> lk(g_arch_mu);
    auto it = g_arch.find(dev);
    if (it != g_arch.end()) return it->second;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    (void)hipGetLastError();
    return "";
  }
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');
  if (c != std::string::npos) a = a.substr(0, c);
  std::lock_guard<std::mutex> lk(g_arch_mu);
  g_arch[dev] = a;
  return a;
}

BatchedCfg builtin_config(int64_t m, int64_t n) {
  return BatchedCfg{randutv_batched_block(m, n), kTileMaskAll, 0};
}

bool lookup_locked(const std::string& arch, int64_t n, int precision, BatchedCfg* out) {
  for (const auto& t : g_tables) {
    if (t.arch != arch || t.precision != precision) continue;
    for (const auto& b : t.buckets)
      if (n >= b.nmin && n <= b.nmax) {
        *out = b.cfg;
        return true;
      }
  }
  return false;
}

// ---- the search -----------------------------------------------------------
struct Rng {  // splitmix64: shapes of the synthetic batches
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
  }
  int64_t uniform(int64_t lo, int64_t hi) { return lo + (int64_t)(next() % (uint64_t)(hi - lo + 1)); }
};

constexpr int64_t kWorkloadMax = 256;

const int64_t kBuckets[][2] = {{1, 64},    {65, 128},  {129, 192}, {193, 256}, {257, 320},
                               {321, 384}, {385, 448}, {449, 512}, {513, 768}, {769, 1024}};

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  int alloc(size_t bytes) {
    RRF_CHECK_HIP(hipMalloc(&p, std::max<size_t>(bytes, 256)));
    return RRF_OK;
  }
};

int read_status(hipStream_t st, const int* status) {
  int h[2] = {0, 0};
  RRF_CHECK_HIP(hipMemcpyAsync(h, status, sizeof h, hipMemcpyDeviceToHost, st));
  RRF_CHECK_HIP(hipStreamSynchronize(st));
  if (h[0]) return set_error(RRF_E_INTERNAL, "autotune: a device-side check failed");
  return RRF_OK;
}

// The configurations tried for a bucket whose largest n is nmax: b in
// {16, 32, 64} (b > nmax only for 16), three tile families, leaf 0 or 16.
std::vector<BatchedCfg> candidates(int64_t nmax) {
  std::vector<BatchedCfg> cands;
  const int masks[3] = {kTileMaskAll, kTileMaskAll & ~(1 << kTile128x128),
                        (1 << kTile128x32) | (1 << kTile128x16) | (1 << kTile64x64)};
  for (int64_t b : {16, 32, 64}) {
    if (b > nmax && b != 16) continue;
    for (int mask : masks)
      for (int leaf : {0, 16}) {
        if (leaf && leaf >= b) continue;
        cands.push_back(BatchedCfg{b, mask, leaf});
      }
  }
  return cands;
}

// Time every candidate on one bucket; fills *best.
int tune_bucket(hipStream_t st, int64_t nmin, int64_t nmax, int precision, int q, int64_t count,
                uint64_t seed, Bucket* best) {
  Rng rng{seed * 0x100000001b3ull + (uint64_t)nmax};
  std::vector<int64_t> m(count), n(count), lda(count);
  for (int64_t j = 0; j < count; ++j) {
    n[j] = rng.uniform(nmin, nmax);
    m[j] = rng.uniform(n[j], 2 * n[j]);
    lda[j] = m[j];
  }
  const std::vector<BatchedCfg> cands = candidates(nmax);
  size_t ws_bytes = 0, a_el = 0, u_el = 0, v_el = 0;
  for (const auto& c : cands)
    ws_bytes = std::max(ws_bytes, randutv_batched_workspace(count, m.data(), n.data(), c.b, precision));
  for (int64_t j = 0; j < count; ++j) {
    a_el += (size_t)m[j] * n[j];
    u_el += (size_t)m[j] * m[j];
    v_el += (size_t)n[j] * n[j];
  }
  if (ws_bytes == 0) return set_error(RRF_E_NOTSUP, "autotune: bucket outside the kernel limits");
  DevBuf ws, a, t, u, v;
  RRF_TRY(ws.alloc(ws_bytes));
  RRF_TRY(a.alloc(a_el * 8));
  RRF_TRY(t.alloc(a_el * 8));
  RRF_TRY(u.alloc(u_el * 8));
  RRF_TRY(v.alloc(v_el * 8));
  std::vector<const double*> A(count);
  std::vector<double*> T(count), U(count), V(count);
  std::vector<uint64_t> seeds(count);
  size_t oa = 0, ou = 0, ov = 0;
  for (int64_t j = 0; j < count; ++j) {
    double* aj = static_cast<double*>(a.p) + oa;
    A[j] = aj;
    T[j] = static_cast<double*>(t.p) + oa;
    U[j] = static_cast<double*>(u.p) + ou;
    V[j] = static_cast<double*>(v.p) + ov;
    oa += (size_t)m[j] * n[j];
    ou += (size_t)m[j] * m[j];
    ov += (size_t)n[j] * n[j];
    seeds[j] = seed + (uint64_t)j;
    RRF_TRY(gaussian(st, seed, (uint64_t)(1u << 20) + (uint64_t)j, m[j], n[j], aj, m[j]));
  }
  hipEvent_t e0, e1;
  RRF_CHECK_HIP(hipEventCreate(&e0));
  RRF_CHECK_HIP(hipEventCreate(&e1));
  int rc = RRF_OK;
  best->ms = -1.0;
  best->candidates = (int)cands.size();
  for (const auto& c : cands) {
    int* status = static_cast<int*>(ws.p);
    rc = fill_u32(st, reinterpret_cast<unsigned*>(status), 2, 0u);
    double t_ms[3] = {0, 0, 0};
    // the first call records the graphs; three replays are timed
    for (int r = -1; r < 3 && rc == RRF_OK; ++r) {
      if (r >= 0 && hipEventRecord(e0, st) != hipSuccess) rc = set_error(RRF_E_HIP, "event");
      if (rc == RRF_OK)
        rc = randutv_batched_run(st, count, m.data(), n.data(), A.data(), lda.data(), c, q,
                                 seeds.data(), U.data(), T.data(), V.data(), ws.p, ws_bytes,
                                 precision, true);
      if (r >= 0 && rc == RRF_OK) {
        float ms = 0.f;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
          rc = set_error(RRF_E_HIP, "autotune: event timing failed");
        t_ms[r] = ms;
      }
    }
    if (rc == RRF_OK) rc = read_status(st, status);
    if (rc != RRF_OK) break;
    std::sort(t_ms, t_ms + 3);
    if (best->ms < 0.0 || t_ms[1] < best->ms) {
      best->ms = t_ms[1];
      best->cfg = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  RRF_CHECK_HIP(hipStreamSynchronize(st));
  best->nmin = nmin;
  best->nmax = nmax;
  return rc;
}

int bucket_of(int64_t n) {
  for (int i = 0; i < (int)(sizeof kBuckets / sizeof kBuckets[0]); ++i)
    if (n >= kBuckets[i][0] && n <= kBuckets[i][1]) return i;
  return -1;
}

// Install `t` as the table of its (arch, precision).
void install(const Table& t) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_default_tried = true;
  merge_tables(std::vector<Table>{t});
}

// Tuning on the caller's workload: every bucket that holds a matrix of the
// batch starts at the built-in configuration; bucket by bucket, each
// candidate is installed and the whole batched call timed (one recording
// call, the median of three replays), and the fastest kept.
int tune_workload(hipStream_t st, int precision, int q, int64_t count, const int64_t* m,
                  const int64_t* n, int64_t nmax, uint64_t seed, Table* tab) {
  std::vector<int> present(sizeof kBuckets / sizeof kBuckets[0], 0);
  size_t a_el = 0, u_el = 0, v_el = 0;
  for (int64_t j = 0; j < count; ++j) {
    const int bk = bucket_of(std::min(m[j], n[j]));
    if (bk >= 0 && kBuckets[bk][0] <= nmax) present[bk] = 1;
    a_el += (size_t)m[j] * n[j];
    u_el += (size_t)m[j] * m[j];
    v_el += (size_t)n[j] * n[j];
  }
  for (size_t i = 0; i < present.size(); ++i)
    if (present[i]) {
      const int64_t hi = std::min(kBuckets[i][1], nmax);
      tab->buckets.push_back(
          Bucket{kBuckets[i][0], hi, builtin_config(2 * hi, hi), 0.0, 0});
    }
  if (tab->buckets.empty()) return set_error(-4, "autotune: no matrix of the batch in a bucket");
  DevBuf a, t, u, v, ws;
  size_t ws_bytes = 0;
  RRF_TRY(a.alloc(a_el * 8));
  RRF_TRY(t.alloc(a_el * 8));
  RRF_TRY(u.alloc(u_el * 8));
  RRF_TRY(v.alloc(v_el * 8));
  std::vector<const double*> A(count);
  std::vector<double*> T(count), U(count), V(count);
  std::vector<int64_t> lda(count);
  size_t oa = 0, ou = 0, ov = 0;
  for (int64_t j = 0; j < count; ++j) {
    double* aj = static_cast<double*>(a.p) + oa;
    A[j] = aj;
    T[j] = static_cast<double*>(t.p) + oa;
    U[j] = static_cast<double*>(u.p) + ou;
    V[j] = static_cast<double*>(v.p) + ov;
    lda[j] = m[j];
    oa += (size_t)m[j] * n[j];
    ou += (size_t)m[j] * m[j];
    ov += (size_t)n[j] * n[j];
    RRF_TRY(gaussian(st, seed, (uint64_t)(1u << 20) + (uint64_t)j, m[j], n[j], aj, m[j]));
  }
  hipEvent_t e0, e1;
  RRF_CHECK_HIP(hipEventCreate(&e0));
  RRF_CHECK_HIP(hipEventCreate(&e1));
  auto timed = [&](const Table& cand, double* ms) -> int {
    install(cand);
    const size_t need = rrf_randutv_batched_workspace_size(count, m, n, 0, precision);
    if (need == 0) return set_error(RRF_E_NOTSUP, "autotune: workspace size");
    if (need > ws_bytes) {
      if (ws.p) RRF_CHECK_HIP(hipFree(ws.p));
      ws.p = nullptr;
      RRF_TRY(ws.alloc(need));
      ws_bytes = need;
    }
    rrf_opts o;
    rrf_opts_init(&o);
    o.precision = precision;
    o.stream = st;
    o.workspace = ws.p;
    o.workspace_bytes = ws_bytes;
    double t_ms[3] = {0, 0, 0};
    for (int r = -1; r < 3; ++r) {
      if (r >= 0) RRF_CHECK_HIP(hipEventRecord(e0, st));
      RRF_TRY(rrf_randutv_batched(count, m, n, A.data(), lda.data(), 0, q, seed, U.data(),
                                  T.data(), V.data(), &o));
      if (r >= 0) {
        float f = 0.f;
        RRF_CHECK_HIP(hipEventRecord(e1, st));
        RRF_CHECK_HIP(hipEventSynchronize(e1));
        RRF_CHECK_HIP(hipEventElapsedTime(&f, e0, e1));
        t_ms[r] = f;
      }
    }
    std::sort(t_ms, t_ms + 3);
    *ms = t_ms[1];
    return RRF_OK;
  };
  int rc = RRF_OK;
  double best_ms = 0.0;
  rc = timed(*tab, &best_ms);
  for (size_t bi = 0; bi < tab->buckets.size() && rc == RRF_OK; ++bi) {
    Bucket& bk = tab->buckets[bi];
    const std::vector<BatchedCfg> cands = candidates(bk.nmax);
    bk.candidates = (int)cands.size();
    for (const auto& c : cands) {
      if (c.b == bk.cfg.b && c.tile_mask == bk.cfg.tile_mask && c.leaf == bk.cfg.leaf) continue;
      Table trial = *tab;
      trial.buckets[bi].cfg = c;
      double ms = 0.0;
      rc = timed(trial, &ms);
      if (rc != RRF_OK) break;
      if (ms < best_ms) {
        best_ms = ms;
        bk.cfg = c;
      }
    }
  }
  for (auto& bk : tab->buckets) bk.ms = best_ms;  // the whole call's time
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

}  // namespace

BatchedCfg batched_config(int64_t m, int64_t n, int precision) {
  const std::string arch = current_arch();
  std::lock_guard<std::mutex> lk(g_mu);
  load_default_locked();
  BatchedCfg c;
  if (!arch.empty() && lookup_locked(arch, n, precision, &c)) return c;
  return builtin_config(m, n);
}

}  // namespace rrf

using namespace rrf;

extern "C" {

int rrf_batched_tune_load(const char* path) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_default_tried = true;  // an explicit load replaces the default cache
  if (path == nullptr) {
    g_tables.clear();
    return RRF_OK;
  }
  std::string text;
  if (!read_file(path, &text)) return set_error(-1, "rrf_batched_tune_load: cannot read the file");
  std::vector<Table> tabs;
  if (!parse_tables(text, &tabs))
    return set_error(-1, "rrf_batched_tune_load: not an rrf-batched-tune-1 cache");
  g_tables.clear();
  merge_tables(tabs);
  return RRF_OK;
}

int rrf_batched_config(int64_t m, int64_t n, int precision, rrf_batched_cfg* out) {
  if (m < 1) return set_error(-1, "m must be >= 1"), -1;
  if (n < 1) return set_error(-2, "n must be >= 1"), -2;
  if (precision != RRF_PREC_FP64 && precision != RRF_PREC_BF16_SKETCH)
    return set_error(-3, "precision must be RRF_PREC_FP64 or RRF_PREC_BF16_SKETCH"), -3;
  if (out == nullptr) return set_error(-4, "out is NULL"), -4;
  const int64_t M = std::max(m, n), N = std::min(m, n);
  const std::string arch = current_arch();
  std::lock_guard<std::mutex> lk(g_mu);
  load_default_locked();
  BatchedCfg c;
  const bool tuned = !arch.empty() && lookup_locked(arch, N, precision, &c);
  if (!tuned) c = builtin_config(M, N);
  out->b = c.b;
  out->tile_mask = c.tile_mask;
  out->leaf = c.leaf;
  out->tuned = tuned ? 1 : 0;
  return RRF_OK;
}

int rrf_batched_autotune(int precision, int32_t q, int64_t count, const int64_t* m,
                         const int64_t* n, int64_t nmax, uint64_t seed, const char* path,
                         const rrf_opts* opts) {
  if (precision != RRF_PREC_FP64 && precision != RRF_PREC_BF16_SKETCH)
    return set_error(-1, "precision must be RRF_PREC_FP64 or RRF_PREC_BF16_SKETCH"), -1;
  if (q < 0) return set_error(-2, "q must be >= 0"), -2;
  if (count < 1) return set_error(-3, "count must be >= 1"), -3;
  if ((m == nullptr) != (n == nullptr))
    return set_error(-4, "m and n must both be given or both be NULL"), -4;
  // Tuning on a caller's batch is limited to kWorkloadMax matrices: one run
  // over 4096 matrices ended in a host-side segmentation fault whose cause
  // is not yet known, so larger workloads are refused rather than run.
  if (m && count > kWorkloadMax)
    return set_error(RRF_E_NOTSUP, "rrf_batched_autotune: at most 256 matrices on a workload");
  if (m)
    for (int64_t j = 0; j < count; ++j) {
      if (m[j] < 1 || m[j] > 4096) return set_error(-4, "m[j] must be in [1, 4096]"), -4;
      if (n[j] < 1 || n[j] > 4096) return set_error(-5, "n[j] must be in [1, 4096]"), -5;
    }
  if (nmax < 1 || nmax > 1024) return set_error(-6, "nmax must be in [1, 1024]"), -6;
  const std::string arch = current_arch();
  if (arch.empty()) return set_error(RRF_E_HIP, "autotune: no HIP device");
  hipStream_t st = opts ? reinterpret_cast<hipStream_t>(opts->stream) : nullptr;
  Table tab;
  tab.arch = arch;
  tab.precision = precision;
  tab.q = q;
  tab.count = count;
  if (m) {
    // a failed trial leaves the tables as they were before the call
    std::vector<Table> saved;
    {
      std::lock_guard<std::mutex> lk(g_mu);
      load_default_locked();
      saved = g_tables;
    }
    const int rc = tune_workload(st, precision, q, count, m, n, nmax, seed, &tab);
    if (rc != RRF_OK) {
      std::lock_guard<std::mutex> lk(g_mu);
      g_tables = saved;
      return rc;
    }
  } else {
    for (const auto& bk : kBuckets) {
      if (bk[0] > nmax) break;
      Bucket best{};
      RRF_TRY(tune_bucket(st, bk[0], std::min(bk[1], nmax), precision, q, count, seed, &best));
      tab.buckets.push_back(best);
    }
  }
  std::lock_guard<std::mutex> lk(g_mu);
  g_default_tried = true;
  merge_tables(std::vector<Table>{tab});
  if (path) {
    FILE* f = fopen(path, "wb");
    if (!f) return set_error(-8, "rrf_batched_autotune: cannot write the cache file");
    const std::string text = format_tables(g_tables);
    const bool ok = fwrite(text.data(), 1, text.size(), f) == text.size();
    fclose(f);
    if (!ok) return set_error(-8, "rrf_batched_autotune: cannot write the cache file");
  }
  return RRF_OK;
}

}  // extern "C"
