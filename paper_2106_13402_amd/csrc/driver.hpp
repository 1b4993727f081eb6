// Algorithm drivers behind the C-ABI (host code enqueuing kernels).
#pragma once

#include "common.hpp"

namespace rrf {

// Alg. 3. Status words (device ints) live at the start of `ws`: word 0
// collects kernel failure bits, word 1 the input finiteness check.
// Early stop of randUTV (Sec. 4.1): before each step the loop ends when the
// reduced columns reach kmax or ||T22||_F <= tol ||A||_F (one host
// synchronization per step); k_out receives the columns reduced.
struct EarlyStop {
  double tol;
  int64_t kmax;
  int64_t* k_out;
  int64_t i0;  // first step: > 0 resumes a partial run whose state is in T, U, V
};

// p < 0 runs Alg. 3; p >= 0 runs Alg. 2 (randUTV_boosted) with oversampling p
// (b + p <= 256, FP64 only). stop: early stop (null: the full factorization).
bool randutv_supported(int64_t m, int64_t n, int64_t b);
size_t randutv_workspace(int64_t m, int64_t n, int64_t b, int precision, int64_t p = -1);
int randutv_run(hipStream_t st, int64_t m, int64_t n, const double* A, int64_t lda, int64_t b,
                int q, uint64_t seed, double* U, double* T, double* V, void* ws, size_t ws_bytes,
                bool check_input, int precision, int* status_out, int64_t p = -1,
                const EarlyStop* stop = nullptr, bool thin_u = false);

// Alg. 1, same status layout.
bool powerurv_supported(int64_t m, int64_t n, int64_t b);
size_t powerurv_workspace(int64_t m, int64_t n, int64_t b, int q, int precision);
int powerurv_run(hipStream_t st, int64_t m, int64_t n, const double* A, int64_t lda, int64_t b,
                 int q, uint64_t seed, double* U, double* T, double* V, void* ws, size_t ws_bytes,
                 bool check_input, int precision);

// The randomized SVD (Sec. 3.3): U (m x l, ld ldu) and V (n x l, ld ldv) may
// be null; S receives the l singular values (descending). Status layout as
// for Alg. 3.
bool rsvd_supported(int64_t m, int64_t n, int64_t l);
size_t rsvd_workspace(int64_t m, int64_t n, int64_t l);
int rsvd_run(hipStream_t st, int64_t m, int64_t n, const double* A, int64_t lda, int64_t l, int q,
             uint64_t seed, double* U, int64_t ldu, double* S, double* V, int64_t ldv, void* ws,
             size_t ws_bytes, bool check_input);

// Configuration of one lockstep group of the batched call: the block size,
// the grouped GEMM's allowed tile shapes (bit mask over GemmTile of
// batched.hpp; 64 x 64 is always allowed) and the widest panel one launch
// factors before the column split takes over (0: as wide as one workgroup
// holds).
constexpr int kTileMaskAll = 0x1f;
struct BatchedCfg {
  int64_t b;
  int tile_mask;
  int leaf;
};
// The configuration b = 0 selects for an m x n matrix (m >= n) in `precision`:
// the loaded tuning table of the current device's architecture when it has
// a bucket holding n (autotune.hip), else the built-in rule
// (randutv_batched_block, every tile shape, no forced split).
BatchedCfg batched_config(int64_t m, int64_t n, int precision);

// Batched Alg. 3 (one configuration for the whole call; matrix j keyed by
// seeds[j]); outputs packed column-major (ld m, m, n). The status words of
// `ws` (word 0: device-side failure bits) are not cleared here. use_graph:
// record the call's launches as HIP graphs on first use and replay them when
// called again with the same shapes (ignored while tracing); else stream the
// lockstep rounds through the descriptor rings.
int64_t randutv_batched_block(int64_t m, int64_t n);
size_t randutv_batched_workspace(int64_t count, const int64_t* m, const int64_t* n, int64_t b,
                                 int precision);
int randutv_batched_run(hipStream_t st, int64_t count, const int64_t* m, const int64_t* n,
                        const double* const* A, const int64_t* lda, const BatchedCfg& cfg, int q,
                        const uint64_t* seeds, double* const* U, double* const* T,
                        double* const* V, void* ws, size_t ws_bytes, int precision,
                        bool use_graph);
// Free the descriptor rings and recorded calls of every device.
int randutv_batched_release();

}  // namespace rrf
