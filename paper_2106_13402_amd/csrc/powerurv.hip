// powerURV (Alg. 1) on one GPU.
//
//   V = Gaussian(seed, stream 0)        (n x n, generated in HBM)
//   q = 0: V = Q of HQR(V)              (RURV, Sec. 3.1 step 2)
//   repeat q times:
//     Y_hat = A V;   V_hat = Q of HQR_thin(Y_hat)   (m x n)
//     Y = A^T V_hat; V = Q of HQR_thin(Y)           (n x n)
//   A_hat = A V;  [U, R] = HQR_full(A_hat);  T = [R; 0]
//
// Mixed mode (RRF_PREC_BF16_SKETCH): the 2q power products Y_hat = A V and
// Y = A^T V_hat are formed from bfloat16 values with FP32 accumulation (A
// scaled by a power of two and copied once, with and without transpose, so
// both products read their operands along K; V and V_hat rounded each
// round), widened to FP64 for the QRs. A positive scale of a product leaves
// its Householder Q unchanged. The QRs, the explicit Q factors and the final
// A_hat = A V stay FP64.
//
// The QRs are blocked Householder factorizations: the panel kernel factors
// nb columns at a time (compact WY, Sec. 2.3) and the trailing columns are
// updated with two GEMMs, A <- A - (W Tf^T)(W^T A). Explicit Q factors are
// formed by applying the stored blocks in reverse to [I; 0], touching only
// the rows and columns each block can change, as LAPACK's dorgqr does.
#include <algorithm>

#include "common.hpp"
#include "context.hpp"
#include "driver.hpp"
#include "kernels.hpp"
#include "trace.hpp"

namespace rrf {

namespace {

struct PBufs {
  int* status = nullptr;
  double* Yh = nullptr;    // m x n
  double* Wall = nullptr;  // m x n explicit reflectors
  double* Tall = nullptr;  // nb x n compact-WY factors, block p at column c0
  double* R = nullptr;     // n x n
  double* Vw = nullptr;    // n x n (only when the caller passes no V)
  double* Z = nullptr;     // nb x max(m, n)
  double* Wt = nullptr;    // m x nb
  double* tau = nullptr;   // n
  double* split = nullptr;
  size_t split_elems = 0;
  void* panel = nullptr;
  size_t panel_bytes = 0;
  // mixed mode: bfloat16 copies (ld a multiple of 8) and the bf16 GEMM scratch
  uint16_t *Ab = nullptr, *Abt = nullptr, *Vb = nullptr, *Vhb = nullptr;
  unsigned long long* word = nullptr;
  void* bwork = nullptr;
  size_t bwork_bytes = 0;
};

bool plan(Arena& ar, int64_t m, int64_t n, int64_t nb, bool need_v, int precision, PBufs* B) {
  const int64_t mx = std::max(m, n);
  B->status = ar.take<int>(64);
  B->Yh = ar.take<double>((size_t)m * n);
  B->Wall = ar.take<double>((size_t)m * n);
  B->Tall = ar.take<double>((size_t)nb * n);
  B->R = ar.take<double>((size_t)n * n);
  if (need_v) B->Vw = ar.take<double>((size_t)n * n);
  B->Z = ar.take<double>((size_t)nb * mx);
  B->Wt = ar.take<double>((size_t)mx * nb);
  B->tau = ar.take<double>((size_t)n);
  B->split_elems = (size_t)8 * mx * nb;
  B->split = ar.take<double>(B->split_elems);
  B->panel_bytes = panel_work_bytes(mx, (int)nb);
  if (B->panel_bytes == 0) return false;
  B->panel = ar.take<char>(B->panel_bytes);
  if (precision == RRF_PREC_BF16_SKETCH) {
    const int64_t lm = bf16_ld(m), ln = bf16_ld(n);
    B->Ab = ar.take<uint16_t>((size_t)lm * n);
    B->Abt = ar.take<uint16_t>((size_t)ln * m);
    B->Vb = ar.take<uint16_t>((size_t)ln * n);
    B->Vhb = ar.take<uint16_t>((size_t)lm * n);
    B->word = ar.take<unsigned long long>(1);
    B->bwork_bytes = std::max(gemm_bf16_work_bytes_k(m, n, n), gemm_bf16_work_bytes_k(n, n, m));
    B->bwork = ar.take<char>(B->bwork_bytes);
  }
  return true;
}

// Householder QR of X (M x N, ld ldx, destroyed): reflectors to W (M x N,
// ld M), block factors to Tall, R (N x N, ld N).
//
// Look-ahead (with a side stream sp and two events): once block p's
// reflectors are applied to the next nb columns, panel p+1 is factored on
// sp while the rest of block p's trailing update runs on st, so the
// latency-bound panels overlap the GEMMs instead of alternating with them.
// Panel p+1 touches only its own columns (rows c0+nb..) and its slices of
// W, Tall, R and tau; the update on st touches the columns after it.
int hqr_blocked(hipStream_t st, int64_t M, int64_t N, int64_t nb, double* X, int64_t ldx,
                PBufs& B, double* Rout, hipStream_t sp, hipEvent_t ev_cols, hipEvent_t ev_panel) {
  RRF_TRY(fill_matrix(st, N, N, 0.0, Rout, N));
  auto panel = [&](hipStream_t s, int64_t c0) -> int {
    const int64_t k = std::min(nb, N - c0);
    return householder_panel(s, M - c0, (int)k, X + c0 + c0 * ldx, ldx, B.Wall + c0 + c0 * M, M,
                             Rout + c0 + c0 * N, N, B.Tall + c0 * nb, nb, B.tau + c0, nullptr, 0,
                             B.panel, B.panel_bytes, B.status);
  };
  // Block p's reflectors applied to columns [j0, j0 + w) of X (rows c0..),
  // and the finished rows c0..c0+k of those columns copied into R.
  auto update = [&](int64_t c0, int64_t k, int64_t j0, int64_t w) -> int {
    const int64_t Mp = M - c0;
    const double* Wp = B.Wall + c0 + c0 * M;
    double* Xr = X + c0 + j0 * ldx;
    RRF_TRY(dgemm(st, true, false, k, w, Mp, 1.0, Wp, M, Xr, ldx, 0.0, B.Z, k, B.split,
                  B.split_elems));
    RRF_TRY(dgemm(st, false, false, Mp, w, k, -1.0, B.Wt, Mp, B.Z, k, 1.0, Xr, ldx, nullptr, 0));
    return copy_matrix(st, k, w, Xr, ldx, Rout + c0 + j0 * N, N);
  };
  RRF_TRY(panel(st, 0));
  for (int64_t c0 = 0; c0 < N; c0 += nb) {
    const int64_t k = std::min(nb, N - c0);
    const int64_t Mp = M - c0;
    const int64_t Nr = N - c0 - k;
    if (Nr <= 0) break;
    // Wt = W Tf^T for block p: A <- (I - W Tf^T W^T) A = Q^T A
    RRF_TRY(dgemm(st, false, true, Mp, k, k, 1.0, B.Wall + c0 + c0 * M, M, B.Tall + c0 * nb, nb,
                  0.0, B.Wt, Mp, nullptr, 0));
    const int64_t kn = std::min(nb, Nr);
    RRF_TRY(update(c0, k, c0 + k, kn));
    if (sp != nullptr && Nr > kn) {
      RRF_CHECK_HIP(hipEventRecord(ev_cols, st));
      RRF_CHECK_HIP(hipStreamWaitEvent(sp, ev_cols, 0));
      RRF_TRY(panel(sp, c0 + k));
      RRF_CHECK_HIP(hipEventRecord(ev_panel, sp));
      RRF_TRY(update(c0, k, c0 + k + kn, Nr - kn));
      RRF_CHECK_HIP(hipStreamWaitEvent(st, ev_panel, 0));
    } else {
      if (Nr > kn) RRF_TRY(update(c0, k, c0 + k + kn, Nr - kn));
      RRF_TRY(panel(st, c0 + k));
    }
  }
  return RRF_OK;
}

// Q(:, 0:ncols) of the factorization held in B.Wall / B.Tall (M x N
// reflectors), written to Q (M x ncols, ld M).
int form_q(hipStream_t st, int64_t M, int64_t N, int64_t nb, int64_t ncols, PBufs& B, double* Q) {
  RRF_TRY(set_identity(st, M, ncols, Q, M));
  const int64_t nblk = ceil_div(N, nb);
  for (int64_t p = nblk - 1; p >= 0; --p) {
    const int64_t c0 = p * nb;
    const int64_t k = std::min(nb, N - c0);
    const int64_t Mp = M - c0;
    const int64_t Nc = ncols - c0;
    const double* Wp = B.Wall + c0 + c0 * M;
    const double* Tp = B.Tall + c0 * nb;
    double* Qp = Q + c0 + c0 * M;
    // Q(c0:, c0:) <- (I - W Tf W^T) Q(c0:, c0:) = Q - (W Tf)(W^T Q)
    RRF_TRY(dgemm(st, false, false, Mp, k, k, 1.0, Wp, M, Tp, nb, 0.0, B.Wt, Mp, nullptr, 0));
    RRF_TRY(dgemm(st, true, false, k, Nc, Mp, 1.0, Wp, M, Qp, M, 0.0, B.Z, k, B.split,
                  B.split_elems));
    RRF_TRY(dgemm(st, false, false, Mp, Nc, k, -1.0, B.Wt, Mp, B.Z, k, 1.0, Qp, M, nullptr, 0));
  }
  return RRF_OK;
}

}  // namespace

bool powerurv_supported(int64_t m, int64_t n, int64_t b) {
  if (b > 256) return false;
  return panel_work_bytes(std::max(m, n), (int)std::min(b, n)) > 0;
}

size_t powerurv_workspace(int64_t m, int64_t n, int64_t b, int q, int precision) {
  Arena ar;
  ar.counting = true;
  PBufs B;
  if (!plan(ar, m, n, std::min(b, n), true, q > 0 ? precision : RRF_PREC_FP64, &B)) return 0;
  return ar.used;
}

int powerurv_run(hipStream_t st, int64_t m, int64_t n, const double* A, int64_t lda, int64_t b,
                 int q, uint64_t seed, double* U, double* T, double* V, void* ws, size_t ws_bytes,
                 bool check_input, int precision) {
  const int64_t nb = std::min(b, n);
  if (q == 0) precision = RRF_PREC_FP64;  // no power products to round
  Arena ar;
  ar.base = reinterpret_cast<char*>(ws);
  ar.cap = ws_bytes;
  PBufs B;
  if (!plan(ar, m, n, nb, V == nullptr, precision, &B) || ar.used > ws_bytes)
    return set_error(RRF_E_NOMEM, "powerurv: workspace too small");
  const bool mixed = precision == RRF_PREC_BF16_SKETCH;
  const int64_t lm = bf16_ld(m), ln = bf16_ld(n);
  RRF_TRY(fill_u32(st, reinterpret_cast<unsigned*>(B.status), 64, 0u));
  if (check_input) RRF_TRY(check_finite(st, m, n, A, lda, B.status + 1));
  double* Vm = V ? V : B.Vw;
  DeviceContext* ctx = nullptr;
  RRF_TRY(device_context(&ctx));
  std::lock_guard<std::mutex> lk(ctx->mu);
  hipStream_t sp = ctx->side[0];
  trace_unmark_stream(sp);
  hipEvent_t ev_cols = ctx->ev[0], ev_panel = ctx->ev[1];

  RRF_TRY(gaussian(st, seed, 0, n, n, Vm, n));
  if (q == 0) {
    RRF_TRY(hqr_blocked(st, n, n, nb, Vm, n, B, B.R, sp, ev_cols, ev_panel));
    RRF_TRY(form_q(st, n, n, nb, n, B, Vm));
  }
  if (mixed) {
    RRF_TRY(maxabs(st, m, n, A, lda, B.word));
    RRF_TRY(to_bf16(st, m, n, A, lda, B.word, B.Ab, lm, B.Abt, ln));
  }
  for (int it = 0; it < q; ++it) {
    if (mixed) {
      // Y_hat = A V = (A^T)^T V
      RRF_TRY(to_bf16(st, n, n, Vm, n, nullptr, B.Vb, ln, nullptr, 0));
      RRF_TRY(gemm_bf16_tn(st, m, n, n, B.Abt, ln, B.Vb, ln, nullptr, 0, B.Yh, m, B.bwork,
                           B.bwork_bytes));
    } else {
      RRF_TRY(dgemm(st, false, false, m, n, n, 1.0, A, lda, Vm, n, 0.0, B.Yh, m, B.split,
                    B.split_elems));
    }
    RRF_TRY(hqr_blocked(st, m, n, nb, B.Yh, m, B, B.R, sp, ev_cols, ev_panel));
    RRF_TRY(form_q(st, m, n, nb, n, B, B.Yh));  // V_hat in Yh
    if (mixed) {
      RRF_TRY(to_bf16(st, m, n, B.Yh, m, nullptr, B.Vhb, lm, nullptr, 0));
      RRF_TRY(gemm_bf16_tn(st, n, n, m, B.Ab, lm, B.Vhb, lm, nullptr, 0, Vm, n, B.bwork,
                           B.bwork_bytes));
    } else {
      RRF_TRY(dgemm(st, true, false, n, n, m, 1.0, A, lda, B.Yh, m, 0.0, Vm, n, B.split,
                    B.split_elems));
    }
    RRF_TRY(hqr_blocked(st, n, n, nb, Vm, n, B, B.R, sp, ev_cols, ev_panel));
    RRF_TRY(form_q(st, n, n, nb, n, B, Vm));
  }
  RRF_TRY(dgemm(st, false, false, m, n, n, 1.0, A, lda, Vm, n, 0.0, B.Yh, m, B.split,
                B.split_elems));
  RRF_TRY(hqr_blocked(st, m, n, nb, B.Yh, m, B, B.R, sp, ev_cols, ev_panel));
  if (U) RRF_TRY(form_q(st, m, n, nb, m, B, U));
  RRF_TRY(fill_matrix(st, m, n, 0.0, T, m));
  RRF_TRY(copy_matrix(st, n, n, B.R, n, T, m));
  return RRF_OK;
}

}  // namespace rrf
