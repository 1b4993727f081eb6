// Runs the batched driver against the test double of mock_kernels.cpp:
// reads matrices from argv[1], writes T (and U, V) to argv[2], prints the
// status and the number of access violations.
//
// Mode 0 streams the lockstep rounds through the descriptor rings. Mode 1
// records the call as graphs and replays it three times: the recording call,
// a replay into the same buffers after they were overwritten with NaN (A
// restored for an in-place call), and a replay into newly allocated outputs
// (the descriptors rebuilt and uploaded); the last results are written.
// At the end the driver's resources are released and every allocation the
// harness made is freed, so a leak checker sees only what the driver lost.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>
#include <cstdint>
#include <hip/hip_runtime.h>
#include "driver.hpp"
extern "C" long mock_errors();
extern "C" long mock_graph_launches();
extern "C" void* mock_malloc(size_t);
extern "C" void mock_free(void*);

static void poison(double* p, size_t count) {
  for (size_t i = 0; i < count; ++i) p[i] = NAN;
}

int main(int argc, char** argv) {
  FILE* f = fopen(argv[1], "rb");
  int64_t hdr[11];
  if (fread(hdr, 8, 11, f) != 11) return 2;
  const int64_t count = hdr[0], b = hdr[1], q = hdr[2];
  const uint64_t seed = hdr[3];
  const bool wu = hdr[4], wv = hdr[5], inplace = hdr[6];
  const int precision = (int)hdr[7];
  const bool graph = hdr[8] != 0;
  const int leaf = (int)hdr[9];
  const int tile_mask = (int)hdr[10];
  std::vector<int64_t> m(count), n(count), lda(count);
  std::vector<const double*> A(count);
  std::vector<std::vector<double>> Ahost(count);
  std::vector<double*> U(count), T(count), V(count);
  std::vector<uint64_t> seeds(count);
  std::vector<void*> owned;
  auto alloc = [&](size_t bytes) {
    owned.push_back(mock_malloc(bytes));
    return (double*)owned.back();
  };
  for (int64_t j = 0; j < count; ++j) {
    int64_t s[3];
    if (fread(s, 8, 3, f) != 3) return 2;
    m[j] = s[0]; n[j] = s[1]; lda[j] = s[2];
    double* a = alloc(8 * lda[j] * n[j]);
    if (fread(a, 8, lda[j] * n[j], f) != (size_t)(lda[j] * n[j])) return 2;
    Ahost[j].assign(a, a + lda[j] * n[j]);
    A[j] = a;
    T[j] = inplace ? a : alloc(8 * m[j] * n[j]);
    U[j] = wu ? alloc(8 * m[j] * m[j]) : nullptr;
    V[j] = wv ? alloc(8 * n[j] * n[j]) : nullptr;
    seeds[j] = seed + j;
  }
  fclose(f);
  size_t ws = rrf::randutv_batched_workspace(count, m.data(), n.data(), b, precision);
  void* w = alloc(ws);
  ((int*)w)[0] = 0; ((int*)w)[1] = 0;
  auto call = [&]() {
    const rrf::BatchedCfg cfg{b, tile_mask, leaf};
    return rrf::randutv_batched_run(nullptr, count, m.data(), n.data(), A.data(), lda.data(), cfg,
                                    (int)q, seeds.data(), wu ? U.data() : nullptr, T.data(),
                                    wv ? V.data() : nullptr, w, ws, precision, graph);
  };
  int rc = call();
  if (graph && rc == 0) {
    for (int64_t j = 0; j < count; ++j) {
      if (inplace) memcpy((void*)A[j], Ahost[j].data(), 8 * lda[j] * n[j]);
      else poison(T[j], m[j] * n[j]);
      if (wu) poison(U[j], m[j] * m[j]);
      if (wv) poison(V[j], n[j] * n[j]);
    }
    rc = call();
  }
  if (graph && rc == 0) {
    for (int64_t j = 0; j < count; ++j) {
      if (inplace) {
        double* a = alloc(8 * lda[j] * n[j]);
        memcpy(a, Ahost[j].data(), 8 * lda[j] * n[j]);
        A[j] = a;
        T[j] = a;
      } else {
        T[j] = alloc(8 * m[j] * n[j]);
      }
      if (wu) U[j] = alloc(8 * m[j] * m[j]);
      if (wv) V[j] = alloc(8 * n[j] * n[j]);
    }
    rc = call();
  }
  printf("rc=%d mock_errors=%ld ws=%zu graph_launches=%ld\n", rc, mock_errors(), ws,
         mock_graph_launches());
  FILE* o = fopen(argv[2], "wb");
  for (int64_t j = 0; j < count; ++j) {
    fwrite(T[j], 8, m[j] * n[j], o);
    if (wu) fwrite(U[j], 8, m[j] * m[j], o);
    if (wv) fwrite(V[j], 8, n[j] * n[j], o);
  }
  fclose(o);
  const int rel = rrf::randutv_batched_release();
  for (void* p : owned) mock_free(p);
  if (rel != 0) printf("release rc=%d\n", rel);
  return rc != 0 ? rc : rel;
}
