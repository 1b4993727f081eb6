// Algorithm drivers behind the C-ABI (host code enqueuing kernels).
#pragma once

#include "common.hpp"

namespace rrf {

// Alg. 3. Status words (device ints) live at the start of `ws`: word 0
// collects kernel failure bits, word 1 the input finiteness check.
bool randutv_supported(int64_t m, int64_t n, int64_t b);
size_t randutv_workspace(int64_t m, int64_t n, int64_t b, int precision);
int randutv_run(hipStream_t st, int64_t m, int64_t n, const double* A, int64_t lda, int64_t b,
                int q, uint64_t seed, double* U, double* T, double* V, void* ws, size_t ws_bytes,
                bool check_input, int precision, int* status_out);

// Alg. 1, same status layout.
bool powerurv_supported(int64_t m, int64_t n, int64_t b);
size_t powerurv_workspace(int64_t m, int64_t n, int64_t b, int q);
int powerurv_run(hipStream_t st, int64_t m, int64_t n, const double* A, int64_t lda, int64_t b,
                 int q, uint64_t seed, double* U, double* T, double* V, void* ws, size_t ws_bytes,
                 bool check_input);

}  // namespace rrf
