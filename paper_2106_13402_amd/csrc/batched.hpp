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

// Device-resident descriptor arrays; one launch each.
int gemm_grouped(hipStream_t st, bool ta, bool tb, const GemmDesc* d_descs, int count,
                 int64_t max_tiles, double flops);
int elem_batched(hipStream_t st, const ElemDesc* d_descs, int count, int64_t max_cols);
int gauss_batched(hipStream_t st, const GaussDesc* d_descs, int count, int64_t max_elems);
// All panels must have at most panel_wg_max_rows(k) rows (k <= 64).
int panel_wg_batched(hipStream_t st, const PanelDesc* d_descs, int count, int k,
                     int64_t max_rows);
int64_t panel_wg_max_rows(int k);

// 64 x 64 tiles of the grouped GEMM.
inline int64_t grouped_tiles(int64_t M, int64_t N) {
  return ((M + 63) / 64) * ((N + 63) / 64);
}

}  // namespace rrf
