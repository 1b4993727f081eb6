// Internal launch interfaces of the rrf kernels (not part of the C-ABI).
#pragma once

#include "common.hpp"

namespace rrf {

// ---- gemm_f64.hip --------------------------------------------------------
// C = alpha op(A) op(B) + beta C (FP64 MFMA). `work` (work_elems doubles) is
// split-K scratch; fewer elements only limit the split.
int dgemm(hipStream_t st, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
          const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
          int64_t ldc, double* work, size_t work_elems);
// dgemm with its launch shape chosen by the caller: 64 x 64 tiles when
// `small_tiles`, and K split `want_splits` ways (fewer when the workspace
// does not hold the partials; 0 or 1: the automatic choice).
int dgemm_shaped(hipStream_t st, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
                 const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                 double* C, int64_t ldc, double* work, size_t work_elems, bool small_tiles,
                 int want_splits);
// C = alpha op(A) op(B) where C is also one operand, with no temporary:
// C = A (op(A) = A, lda = ldc) needs M >= 128 and N = 128; C = B (op(B) = B,
// ldb = ldc) needs M = 128 and N >= 128. The product runs on 128 x 128
// tiles, one tile across the dimension in which the aliased operand is
// read, so each workgroup reads only the rows (columns) it writes, and every
// read precedes the epilogue's stores (a split-K product writes C only in
// its reduction, after all partial products). dgemm_in_place_fits tells
// whether a call qualifies; dgemm_in_place returns RRF_E_NOTSUP without
// launching when it does not.
bool dgemm_in_place_fits(bool ta, bool tb, int64_t M, int64_t N, const double* A, int64_t lda,
                         const double* B, int64_t ldb, const double* C, int64_t ldc);
int dgemm_in_place(hipStream_t st, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
                   const double* A, int64_t lda, const double* B, int64_t ldb, double* C,
                   int64_t ldc, double* work, size_t work_elems);
// C = alpha sum_z P_z + beta C for split-K partials P_z = P + z M N (ld M),
// summed in split order.
int splitk_reduce(hipStream_t st, int64_t M, int64_t N, int splits, const double* P, double alpha,
                  double beta, double* C, int64_t ldc);

// The signature shared by dgemm and gemm_x3.
typedef int (*GemmFn)(hipStream_t, bool, bool, int64_t, int64_t, int64_t, double, const double*,
                      int64_t, const double*, int64_t, double, double*, int64_t, double*, size_t);

// ---- gemm_x3.hip -----------------------------------------------------------
// As dgemm, with every operand split into bfloat16 hi + lo (from its binary32
// rounding) and the product hi hi + hi lo + lo hi accumulated in binary32.
int gemm_x3(hipStream_t st, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
            const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
            int64_t ldc, double* work, size_t work_elems);

// ---- gemm_x6.hip -----------------------------------------------------------
// As dgemm, with every operand split into bfloat16 hi + mid + lo (from its
// binary32 rounding) and the six leading products hi hi + hi mid + mid hi +
// hi lo + lo hi + mid mid accumulated in binary32 per K slice of 32, the
// slices summed in binary64.
int gemm_x6(hipStream_t st, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
            const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
            int64_t ldc, double* work, size_t work_elems);

// ---- philox.hip ----------------------------------------------------------
int gaussian(hipStream_t st, uint64_t seed, uint64_t stream_id, int64_t rows, int64_t cols,
             double* out, int64_t ld);
// The uniforms behind the Gaussian above: row 4g + i, column c holds uniform
// i of counter (g, c, 0, 0) (order u_a, v_a, u_b, v_b).
int sketch_uniforms(hipStream_t st, uint64_t seed, uint64_t stream_id, int64_t rows, int64_t cols,
                    double* out, int64_t ld);

// ---- util.hip ------------------------------------------------------------
int set_identity(hipStream_t st, int64_t rows, int64_t cols, double* X, int64_t ld);
// D (cols x rows, ld ldd) = S^T (S rows x cols, ld lds).
int transpose_matrix(hipStream_t st, int64_t rows, int64_t cols, const double* S, int64_t lds,
                     double* D, int64_t ldd);
// Q(:, 0:k) of a Householder QR (W unit lower trapezoidal M x k, Tf k x k):
// (I - W Tf W^T)(:, 0:k) = [I; 0] - W (Tf W(0:k, :)^T); C: k x k scratch.
int thin_q(hipStream_t st, int64_t M, int64_t k, const double* W, int64_t ldw, const double* Tf,
           int64_t ldt, double* Q, int64_t ldq, double* C);
int copy_matrix(hipStream_t st, int64_t rows, int64_t cols, const double* S, int64_t lds,
                double* D, int64_t ldd);
int fill_matrix(hipStream_t st, int64_t rows, int64_t cols, double v, double* X, int64_t ld);
// X(0:rows, 0:cols) = 0 except X(k, k) = d[k], k < min(rows, cols).
int set_diag(hipStream_t st, int64_t rows, int64_t cols, const double* d, double* X, int64_t ld);
int fill_u32(hipStream_t st, unsigned* p, int64_t count, unsigned v);
// status[0] |= 1 when X (rows x cols) holds a NaN or an infinity.
int check_finite(hipStream_t st, int64_t rows, int64_t cols, const double* X, int64_t ld,
                 int* status);

// ---- panel_qr.hip --------------------------------------------------------
struct PanelPlan {
  int G = 0;          // workgroups
  int rows_per = 0;   // rows owned by each workgroup
  size_t lds = 0;     // dynamic LDS bytes
  size_t work = 0;    // global scratch bytes
};
bool panel_plan(int64_t M, int k, PanelPlan* plan);  // one launch
// Workspace of householder_panel for every panel height up to Mmax with k
// columns (0 when unsupported); taller panels than one launch takes are split
// by columns.
size_t panel_work_bytes(int64_t Mmax, int k);
// Householder QR of the M x k panel P; see rrf_householder_panel. When
// `zero` is non-null the M x k region it points to (ld ldz) is set to 0 after
// the panel has been read (used to clear T(I2 u I3, J2) in place).
int householder_panel(hipStream_t st, int64_t M, int k, const double* P, int64_t ldp,
                      double* W, int64_t ldw, double* R, int64_t ldr, double* Tf, int64_t ldt,
                      double* tau, double* zero, int64_t ldz, void* work, size_t work_bytes,
                      int* status);

// The column-exchange kernel alone (one cooperative launch, the panel within
// panel_plan); when `cond` is not null every workgroup returns at once unless
// *cond != 0 (the CholeskyQR path's fallback).
int panel_launch_if(hipStream_t st, int64_t M, int k, const double* P, int64_t ldp, double* W,
                    int64_t ldw, double* R, int64_t ldr, double* Tf, int64_t ldt, double* tau,
                    double* zero, int64_t ldz, void* work, size_t work_bytes, int* status,
                    const int* cond);

// ---- panel_cholqr.hip -----------------------------------------------------
// The same factorization as householder_panel by CholeskyQR2 and
// reconstruction of the reflectors, for 16 <= k <= 128, M >= 1024 and W not
// overlapping P; ill-conditioned or rank-deficient panels fall back to the
// column-exchange kernel on the device. Off when
// RRF_PANEL_COLUMN=1 is in the environment (read at each call).
bool cholqr_enabled();
bool cholqr_panel_ok(int64_t M, int k, const double* P, int64_t ldp, const double* W,
                     int64_t ldw);
size_t cholqr_work_bytes(int64_t M, int k);
int cholqr_panel(hipStream_t st, int64_t M, int k, const double* P, int64_t ldp, double* W,
                 int64_t ldw, double* R, int64_t ldr, double* Tf, int64_t ldt, double* tau,
                 double* zero, int64_t ldz, void* work, size_t work_bytes, int* status);

// ---- panel_tsqr.hip -------------------------------------------------------
// The same factorization as householder_panel for 1 <= k <= 64 and
// k <= M <= 65536, by a tree of QRs over 256-row leaves and reconstruction
// of the reflectors; one cooperative launch of ceil(M / 256) workgroups.
bool tsqr_panel_ok(int64_t M, int k);
size_t tsqr_work_bytes(int64_t M, int k);  // 0 when not tsqr_panel_ok
int tsqr_panel(hipStream_t st, int64_t M, int k, const double* P, int64_t ldp, double* W,
               int64_t ldw, double* R, int64_t ldr, double* Tf, int64_t ldt, double* tau,
               double* zero, int64_t ldz, void* work, size_t work_bytes, int* status);

// ---- sketch_bf16.hip ------------------------------------------------------
// Leading dimension of a bfloat16 copy with `rows` rows (a multiple of 8).
inline int64_t bf16_ld(int64_t rows) { return (rows + 7) & ~(int64_t)7; }
// *word = max|X| as binary64 bits (word zeroed first).
int maxabs(hipStream_t st, int64_t rows, int64_t cols, const double* X, int64_t ld,
           unsigned long long* word);
// out = bf16(X s) (rows x cols, ld ldo, rows [rows, ldo) zero) and, when
// outT is non-null, its transpose (ld ldot, rows [cols, ldot) zero); s is the
// power of two putting max|X| (from *word) in [0.5, 1), or 1 when word is null.
// *out (device) = ||X||_F, summing the squares of X s with s the power of two
// of the max in *word (a bound on |X|); parts: scratch of max_parts doubles,
// at least ceil(rows / 256). Deterministic.
int frob_norm(hipStream_t st, int64_t rows, int64_t cols, const double* X, int64_t ld,
              const unsigned long long* word, double* parts, int max_parts, double* out);
// X *= s (inverse: X /= s), s the power of two putting max|X| from *word in
// [0.5, 1) (1 when the max is 0); exact. guard_exp > 0: s = 1 (nothing done)
// unless s lies outside [2^-guard_exp, 2^guard_exp].
int scale_pow2(hipStream_t st, int64_t rows, int64_t cols, double* X, int64_t ld,
               const unsigned long long* word, bool inverse, int guard_exp = 0);
int to_bf16(hipStream_t st, int64_t rows, int64_t cols, const double* X, int64_t ld,
            const unsigned long long* word, uint16_t* out, int64_t ldo, uint16_t* outT,
            int64_t ldot);
// Workspace of gemm_bf16_tn for any K (16 split-K partials), and for one K.
size_t gemm_bf16_work_bytes(int64_t M, int64_t N);
size_t gemm_bf16_work_bytes_k(int64_t M, int64_t N, int64_t K);
// A^T B (A: K x M, B: K x N, bfloat16, ld multiples of 8, rows past K zero)
// with FP32 accumulation; the M x N result goes either to out16 as bfloat16
// with each column scaled by its own power of two (rows [M, ld16) zero), or to
// out64 widened to FP64.
int gemm_bf16_tn(hipStream_t st, int64_t M, int64_t N, int64_t K, const uint16_t* A,
                 int64_t lda, const uint16_t* B, int64_t ldb, uint16_t* out16, int64_t ld16,
                 double* out64, int64_t ld64, void* work, size_t work_bytes);

// ---- svd_left.hip --------------------------------------------------------
// Left singular vectors U (k x k, ld k; columns in descending order of d) and
// singular values d of the k x k matrix B (ld ldb), k <= 256, by block
// one-sided Jacobi; column signs unspecified. status bit 2: no convergence.
size_t left_svd_work_bytes(int k);
int left_svd(hipStream_t st, int k, const double* B, int64_t ldb, double* U, double* d, void* work,
             size_t work_bytes, int* status);

// ---- jacobi_svd.hip ------------------------------------------------------
size_t block_svd_work_bytes(int k);
// As block_svd_batched with the size of every block in d_sizes (device ints,
// each <= kmax; blocks laid out with stride elements between them).
int block_svd_sized(hipStream_t st, int count, int kmax, const int* d_sizes, const double* B,
                    int64_t ldb, int64_t stride, double* Us, double* d, int64_t dstride,
                    double* Vs, void* work, size_t work_bytes, int* status);
int block_svd(hipStream_t st, int k, const double* B, int64_t ldb, double* Us, double* d,
              double* Vs, void* work, size_t work_bytes, int* status);
// `count` independent SVDs in one launch (one workgroup each): blocks 0..count-2
// are k x k, the last is k_last x k_last (k_last <= k); block i of B / Us / Vs
// starts at i * stride (B with leading dimension ldb, Us and Vs tight), d_i at
// i * dstride. Global scratch when a block does not fit in LDS:
// count * block_svd_work_bytes(k).
int block_svd_batched(hipStream_t st, int count, int k, int k_last, const double* B, int64_t ldb,
                      int64_t stride, double* Us, double* d, int64_t dstride, double* Vs,
                      void* work, size_t work_bytes, int* status);

}  // namespace rrf
