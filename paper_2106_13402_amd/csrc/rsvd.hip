// The randomized SVD (RSVD; Sec. 3.3, where it is related to powerURV).
//
// Y = (A A^T)^q A G (m x l) with G the Gaussian of stream 0 (the first l
// columns of powerURV's G, so the two methods can be compared as the paper's
// Theorem 1 does), Q from the Householder QR of Y, the thin SVD
// Q^T A = W Sigma V^T and U = Q W. The SVD of the l x n matrix Q^T A is taken
// through its transpose B^T = A^T Q (n x l), tall and thin like the samples
// of randUTV_boosted: B^T = Q2 R2 (Householder QR), R2 = Ur Sigma Vr^T
// (one-workgroup Jacobi), so Q^T A = Vr Sigma (Q2 Ur)^T, W = Vr, V = Q2 Ur.
// Every product is an FP64 MFMA GEMM; nothing here needs m >= n.
#include <algorithm>

#include "common.hpp"
#include "driver.hpp"
#include "kernels.hpp"
#include "trace.hpp"

namespace rrf {

namespace {

struct RBufs {
  int* status = nullptr;
  double* G = nullptr;   // n x l
  double* Y = nullptr;   // m x l  sample, then its Householder QR in place
  double* Z = nullptr;   // n x l  power-step product, then Q2(:, 0:l)
  double* Q = nullptr;   // m x l
  double* Bt = nullptr;  // n x l  A^T Q, then its Householder QR in place
  double* R = nullptr;   // l x l
  double* Tf = nullptr;  // l x l
  double* Us = nullptr;  // l x l
  double* Vs = nullptr;  // l x l
  double* d = nullptr;   // l
  double* C = nullptr;   // l x l
  double* tau = nullptr; // l
  double* split = nullptr;
  size_t split_elems = 0;
  void* panel = nullptr;
  size_t panel_bytes = 0;
  void* svd = nullptr;
  size_t svd_bytes = 0;
};

bool rplan(Arena& ar, int64_t m, int64_t n, int64_t l, RBufs* B) {
  const int64_t mx = std::max(m, n);
  B->status = ar.take<int>(64);
  B->G = ar.take<double>((size_t)n * l);
  B->Y = ar.take<double>((size_t)m * l);
  B->Z = ar.take<double>((size_t)n * l);
  B->Q = ar.take<double>((size_t)m * l);
  B->Bt = ar.take<double>((size_t)n * l);
  B->R = ar.take<double>((size_t)l * l);
  B->Tf = ar.take<double>((size_t)l * l);
  B->Us = ar.take<double>((size_t)l * l);
  B->Vs = ar.take<double>((size_t)l * l);
  B->d = ar.take<double>((size_t)l);
  B->C = ar.take<double>((size_t)l * l);
  B->tau = ar.take<double>((size_t)l);
  B->split_elems = (size_t)8 * mx * l;
  B->split = ar.take<double>(B->split_elems);
  B->panel_bytes = panel_work_bytes(mx, (int)l);
  if (B->panel_bytes == 0) return false;
  B->panel = ar.take<char>(B->panel_bytes);
  B->svd_bytes = block_svd_work_bytes((int)l);
  B->svd = ar.take<char>(B->svd_bytes);
  return true;
}

}  // namespace

bool rsvd_supported(int64_t m, int64_t n, int64_t l) {
  return l >= 1 && l <= 256 && l <= std::min(m, n) && panel_work_bytes(std::max(m, n), (int)l) > 0;
}

size_t rsvd_workspace(int64_t m, int64_t n, int64_t l) {
  Arena ar;
  ar.counting = true;
  RBufs B;
  if (!rplan(ar, m, n, l, &B)) return 0;
  return ar.used;
}

int rsvd_run(hipStream_t st, int64_t m, int64_t n, const double* A, int64_t lda, int64_t l, int q,
             uint64_t seed, double* U, int64_t ldu, double* S, double* V, int64_t ldv, void* ws,
             size_t ws_bytes, bool check_input) {
  Arena ar;
  ar.base = reinterpret_cast<char*>(ws);
  ar.cap = ws_bytes;
  RBufs B;
  if (!rplan(ar, m, n, l, &B) || ar.used > ws_bytes)
    return set_error(RRF_E_NOMEM, "rsvd: workspace too small");
  const size_t SE = B.split_elems;
  RRF_TRY(fill_u32(st, reinterpret_cast<unsigned*>(B.status), 64, 0u));
  if (check_input) RRF_TRY(check_finite(st, m, n, A, lda, B.status + 1));
  // Y = (A A^T)^q A G
  RRF_TRY(gaussian(st, seed, 0, n, l, B.G, n));
  RRF_TRY(dgemm(st, false, false, m, l, n, 1.0, A, lda, B.G, n, 0.0, B.Y, m, B.split, SE));
  for (int it = 0; it < q; ++it) {
    RRF_TRY(dgemm(st, true, false, n, l, m, 1.0, A, lda, B.Y, m, 0.0, B.Z, n, B.split, SE));
    RRF_TRY(dgemm(st, false, false, m, l, n, 1.0, A, lda, B.Z, n, 0.0, B.Y, m, B.split, SE));
  }
  // Q = Q_Y(:, 0:l)
  RRF_TRY(householder_panel(st, m, (int)l, B.Y, m, B.Y, m, nullptr, 0, B.Tf, l, B.tau, nullptr,
                            0, B.panel, B.panel_bytes, B.status));
  RRF_TRY(thin_q(st, m, l, B.Y, m, B.Tf, l, B.Q, m, B.C));
  // B^T = A^T Q = Q2 R2, R2 = Ur Sigma Vr^T
  RRF_TRY(dgemm(st, true, false, n, l, m, 1.0, A, lda, B.Q, m, 0.0, B.Bt, n, B.split, SE));
  RRF_TRY(householder_panel(st, n, (int)l, B.Bt, n, B.Bt, n, B.R, l, B.Tf, l, B.tau, nullptr, 0,
                            B.panel, B.panel_bytes, B.status));
  RRF_TRY(block_svd(st, (int)l, B.R, l, B.Us, B.d, B.Vs, B.svd, B.svd_bytes, B.status));
  RRF_TRY(copy_matrix(st, l, 1, B.d, l, S, l));
  if (V) {  // V = Q2(:, 0:l) Ur
    RRF_TRY(thin_q(st, n, l, B.Bt, n, B.Tf, l, B.Z, n, B.C));
    RRF_TRY(dgemm(st, false, false, n, l, l, 1.0, B.Z, n, B.Us, l, 0.0, V, ldv, nullptr, 0));
  }
  if (U)  // U = Q Vr
    RRF_TRY(dgemm(st, false, false, m, l, l, 1.0, B.Q, m, B.Vs, l, 0.0, U, ldu, nullptr, 0));
  return RRF_OK;
}

}  // namespace rrf
