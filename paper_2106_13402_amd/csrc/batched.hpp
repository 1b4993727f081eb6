// Descriptors and launchers of the batched building blocks (batched.hip).
#pragma once

#include "common.hpp"

namespace rrf {

// C = alpha op(A) op(B) + beta C; with beta == 0, C is not read.
struct GemmDesc {
  int64_t M, N, K;
  const double* A;
  int64_t lda;
  const double* B;
  int64_t ldb;
  double* C;
  int64_t ldc;
  double alpha, beta;
};

enum { kElemFill = 0, kElemCopy = 1, kElemDiag = 2, kElemIdentity = 3 };

// X (rows x cols, ld ld) = v | S (ld lds) | [diag(S); 0] | I.
struct ElemDesc {
  int op;
  int64_t rows, cols;
  const double* S;
  int64_t lds;
  double* X;
  int64_t ld;
  double v;
};

// The rows x cols sketch Gaussian of key (seed, sid).
struct GaussDesc {
  uint64_t seed, sid;
  int64_t rows, cols;
  double* out;
  int64_t ld;
};

// Householder QR of the M x k panel P (k given per launch); outputs as
// rrf_householder_panel (R may be null); `zero` (ld ldz) is cleared after
// the panel is read when non-null.
struct PanelDesc {
  int64_t M;
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
};

// --- mixed sketch of the batch (sketch_bf16.hip) ---------------------------

// max|X| of each problem into *word (binary64 bits; words zeroed first).
struct MaxDesc {
  int64_t rows, cols;
  const double* X;
  int64_t ld;
  unsigned long long* word;
};
// out = bf16(X s) (ld ldo, rows past `rows` zero), outT its transpose when
// non-null (ld ldot); s = the power of two of *word (1 when word is null).
struct Bf16Desc {
  int64_t rows, cols;
  const double* X;
  int64_t ld;
  const unsigned long long* word;
  uint16_t* out;
  int64_t ldo;
  uint16_t* outT;
  int64_t ldot;
};
// A^T B (A: K x M, B: K x N, bfloat16, ld multiples of 8, rows past K zero)
// with FP32 accumulation, to P (FP32, ld ldp) or, when out64 is non-null,
// widened to out64.
struct Bf16GemmDesc {
  int64_t M, N, K;
  const uint16_t* A;
  int64_t lda;
  const uint16_t* B;
  int64_t ldb;
  float* P;
  int64_t ldp;
  double* out64;
  int64_t ld64;
};
// out16(:, j) = bf16(P(:, j) 2^-e_j), the power of two putting the column's
// max in [0.5, 1); rows [M, ld16) zero.
struct RoundDesc {
  int64_t M, N;
  const float* P;
  int64_t ldp;
  uint16_t* out16;
  int64_t ld16;
};
int maxabs_batched(hipStream_t st, const MaxDesc* d, int count, int64_t max_rows);
int to_bf16_batched(hipStream_t st, const Bf16Desc* d, int count, int64_t max_tiles);
// d_prefix: running counts of 128 x 32 output tiles (count + 1 ints)
int gemm_bf16_grouped(hipStream_t st, const Bf16GemmDesc* d, const int* d_prefix, int count,
                      int64_t total_tiles, double flops);
int round_columns_batched(hipStream_t st, const RoundDesc* d, int count, int64_t max_cols);
inline int64_t bf16_group_tiles(int64_t M, int64_t N) { return ((M + 127) / 128) * ((N + 31) / 32); }
inline int64_t bf16_conv_tiles(int64_t rows, int64_t cols, int64_t ldo, int64_t ldot) {
  const int64_t R = rows > ldo ? rows : ldo, C = cols > ldot ? cols : ldot;
  return ((R + 63) / 64) * ((C + 63) / 64);
}

// Tile shapes of the grouped GEMM: rows x columns of C per workgroup.
enum GemmTile { kTile64x64 = 0, kTile128x64 = 1, kTile128x32 = 2, kTile128x16 = 3,
                kTile128x128 = 4, kGemmTiles = 5 };
inline int64_t tile_rows(int tile) { return tile == kTile64x64 ? 64 : 128; }
inline int64_t tile_cols(int tile) {
  return tile == kTile128x32 ? 32 : (tile == kTile128x16 ? 16 : (tile == kTile128x128 ? 128 : 64));
}
inline int64_t tile_count(int tile, int64_t M, int64_t N) {
  const int64_t r = tile_rows(tile), c = tile_cols(tile);
  return ((M + r - 1) / r) * ((N + c - 1) / c);
}

// Device-resident descriptor arrays; one launch each. The grouped GEMM runs
// total_tiles workgroups: d_prefix (count + 1 ints, d_prefix[0] = 0) holds
// the running tile counts, problem p owning workgroups [d_prefix[p],
// d_prefix[p+1]).
// vec: every A and B starts 16-byte aligned with even leading dimensions
// (16-byte loads).
int gemm_grouped(hipStream_t st, bool ta, bool tb, int tile, bool vec, const GemmDesc* d_descs,
                 const int* d_prefix, int count, int64_t total_tiles, double flops);
int elem_batched(hipStream_t st, const ElemDesc* d_descs, int count, int64_t max_cols);
int gauss_batched(hipStream_t st, const GaussDesc* d_descs, int count, int64_t max_elems);
// All panels must have at most panel_wg_max_rows(k) rows (k <= 64).
int panel_wg_batched(hipStream_t st, const PanelDesc* d_descs, int count, int k,
                     int64_t max_rows);
int64_t panel_wg_max_rows(int k);

}  // namespace rrf
