// Runs the batched driver against the test double of mock_kernels.cpp:
// reads matrices from argv[1], writes T (and U, V) to argv[2], prints the
// status and the number of access violations.
#include <cstdio>
#include <cstdlib>
#include <vector>
#include <cstdint>
#include <hip/hip_runtime.h>
#include "driver.hpp"
extern "C" long mock_errors();
extern "C" void* mock_malloc(size_t);
int main(int argc, char** argv) {
  FILE* f = fopen(argv[1], "rb");
  int64_t hdr[8];
  if (fread(hdr, 8, 8, f) != 8) return 2;
  const int64_t count = hdr[0], b = hdr[1], q = hdr[2];
  const uint64_t seed = hdr[3];
  const bool wu = hdr[4], wv = hdr[5], inplace = hdr[6];
  const int precision = (int)hdr[7];
  std::vector<int64_t> m(count), n(count), lda(count);
  std::vector<const double*> A(count);
  std::vector<double*> U(count), T(count), V(count);
  std::vector<uint64_t> seeds(count);
  for (int64_t j = 0; j < count; ++j) {
    int64_t s[3];
    if (fread(s, 8, 3, f) != 3) return 2;
    m[j] = s[0]; n[j] = s[1]; lda[j] = s[2];
    double* a = (double*)mock_malloc(8 * lda[j] * n[j]);
    if (fread(a, 8, lda[j] * n[j], f) != (size_t)(lda[j] * n[j])) return 2;
    A[j] = a;
    T[j] = inplace ? a : (double*)mock_malloc(8 * m[j] * n[j]);
    U[j] = wu ? (double*)mock_malloc(8 * m[j] * m[j]) : nullptr;
    V[j] = wv ? (double*)mock_malloc(8 * n[j] * n[j]) : nullptr;
    seeds[j] = seed + j;
  }
  fclose(f);
  size_t ws = rrf::randutv_batched_workspace(count, m.data(), n.data(), b, precision);
  void* w = mock_malloc(ws);
  ((int*)w)[0] = 0; ((int*)w)[1] = 0;
  int rc = rrf::randutv_batched_run(nullptr, count, m.data(), n.data(), A.data(), lda.data(), b, (int)q,
                                    seeds.data(), wu ? U.data() : nullptr, T.data(),
                                    wv ? V.data() : nullptr, w, ws, precision);
  printf("rc=%d mock_errors=%ld ws=%zu\n", rc, mock_errors(), ws);
  FILE* o = fopen(argv[2], "wb");
  for (int64_t j = 0; j < count; ++j) {
    fwrite(T[j], 8, m[j] * n[j], o);
    if (wu) fwrite(U[j], 8, m[j] * m[j], o);
    if (wv) fwrite(V[j], 8, n[j] * n[j], o);
  }
  fclose(o);
  return rc;
}
