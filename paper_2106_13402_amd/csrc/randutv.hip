// randUTV_basic (Alg. 3) on one GPU.
//
// Per step i (0-based here, c0 = i b, J2 = [c0, c2), I2 = [c0, r2)):
//   1. G_i = Gaussian(seed, stream i+1), (m-c0) x b, generated in HBM;
//   2. Y = T22^T G_i, then q times Z = T22 Y, Y = T22^T Z  (MFMA GEMMs);
//   3. [W_v, Tf_v] = Householder QR of Y (panel kernel; W_v overwrites Y);
//   4. X = T(:, J2uJ3) W_v and T(:, J2) -= X (W_v Tf_v^T)(J2, :)^T: only the
//      columns J2 of T V_i are formed here, for the next panel;
//   5. [W_u, Tf_u, R] = Householder QR of T(I2uI3, J2); that panel of T is
//      cleared in the same kernel (T(I3,J2) = 0 of Alg. 3, and T(I2,J2)
//      receives D below);
//   6. the rest of T <- U_i^T T V_i in one pass over T(:, J3):
//        Z^T = T(I2uI3, J3)^T W_u - (W_v Tf_v^T)(J3, :) (X(I2uI3, :)^T W_u)
//      is W_u^T of the right-updated block, formed from the block before the
//      update, and then
//        T(:, J3) -= [X, W_u Tf_u^T] [(W_v Tf_v^T)(J3, :), Z^T]^T,
//      a single GEMM with inner dimension 2b (W_u Tf_u^T is zero on rows I1);
//      V(:, J2uJ3) V_i and U(:, I2uI3) U_i as two GEMMs each;
//   7. [Us, D, Vs] = SVD(R) (one-workgroup Jacobi), then U(:,I2) Us,
//      V(:,J2) Vs, T(I2,J2) = D, T(I2,J3) = Us^T T(I2,J3), T(I1,J2) Vs.
// The last step (J3 empty) takes the SVD of the trailing block, through a
// Householder QR first when the block is tall (Sec. 4.2, tall-thin SVD).
//
// Every compact-WY application uses W Tf W^T = W (W Tf^T)^T: the small
// triangular factor is folded into one operand once per step.
//
// Schedule. The data dependences of a step, not the order in which Alg. 3
// lists its statements, decide what may overlap:
//  * the caller's stream carries the critical path -- generator, sketch,
//    both panels and both updates of T;
//  * a side stream accumulates V and U: V(:, J2uJ3) V_i needs only W_v and
//    U(:, I2uI3) U_i only W_u, and nothing on the critical path reads U or V;
//  * no later step depends on a block's SVD. After step i no step touches
//    columns J2 of T, U or V, and rows I2 of T are only multiplied from the
//    right, which commutes with the left rotation by Us^T. So every R is kept
//    and all the small SVDs run as one batched launch (one workgroup per
//    block) after the loop, followed by T(I2,J2) = D, T(I1,J2) Vs, U(:,I2) Us,
//    V(:,J2) Vs and T(I2,J3) <- Us^T T(I2,J3) for every block.
// W_v, W_u, [X, W_u Tf_u^T] and [W_v Tf_v^T, Z^T] live in two-deep rings, so
// the critical path reuses a slot only after the side stream finished with
// it two steps earlier.
#include <algorithm>

#include "common.hpp"
#include "context.hpp"
#include "driver.hpp"
#include "kernels.hpp"

namespace rrf {

namespace {

struct Bufs {
  int* status = nullptr;
  double* G = nullptr;      // m x b
  double* Z = nullptr;      // m x b
  double* Y[2] = {};        // n x b  sketch, then W_v
  double* Wu[2] = {};       // m x b
  double* XW[2] = {};       // m x 2b [X, W_u Tf_u^T] (ld m; zero rows I1 on the right)
  double* WZ[2] = {};       // n x 2b [W_v Tf_v^T, Z^T] (ld n; Z^T on rows J3)
  double* S = nullptr;      // b x b  X(I2uI3, :)^T W_u
  double* X0 = nullptr;     // max(m,n) x b   (critical stream, after the loop)
  double* X1 = nullptr;     // max(m,n) x b   (side stream)
  double* Zl = nullptr;     // b x n          (critical stream, after the loop)
  double* Tv = nullptr;     // b x b
  double* Tu = nullptr;     // b x b
  double* tau = nullptr;    // b
  double* R = nullptr;      // s x (b x b)
  double* Us = nullptr;     // s x (b x b)
  double* Vs = nullptr;     // s x (b x b)
  double* d = nullptr;      // s x b
  double* split[2] = {};
  size_t split_elems = 0;
  void* panel = nullptr;
  size_t panel_bytes = 0;
  void* svd = nullptr;
  size_t svd_bytes = 0;
  // mixed sketch (bfloat16 copies, ld a multiple of 8)
  uint16_t* Tb = nullptr;   // m x n   T22, scaled
  uint16_t* Tbt = nullptr;  // n x m   its transpose
  uint16_t* Gb = nullptr;   // m x b
  uint16_t* Yb = nullptr;   // n x b
  uint16_t* Zb = nullptr;   // m x b
  unsigned long long* word = nullptr;  // max|T22|
  void* bwork = nullptr;
  size_t bwork_bytes = 0;
};

bool plan(Arena& ar, int64_t m, int64_t n, int64_t b, int precision, Bufs* B) {
  const int64_t mx = std::max(m, n);
  const int64_t kb = std::min(b, n);
  const int64_t s = ceil_div(n, b);
  B->status = ar.take<int>(64);
  B->G = ar.take<double>((size_t)m * kb);
  B->Z = ar.take<double>((size_t)m * kb);
  for (int r = 0; r < 2; ++r) {
    B->Y[r] = ar.take<double>((size_t)n * kb);
    B->Wu[r] = ar.take<double>((size_t)m * kb);
    B->XW[r] = ar.take<double>((size_t)m * 2 * kb);
    B->WZ[r] = ar.take<double>((size_t)n * 2 * kb);
  }
  B->S = ar.take<double>((size_t)kb * kb);
  B->X0 = ar.take<double>((size_t)mx * kb);
  B->X1 = ar.take<double>((size_t)mx * kb);
  B->Zl = ar.take<double>((size_t)kb * n);
  B->Tv = ar.take<double>((size_t)kb * kb);
  B->Tu = ar.take<double>((size_t)kb * kb);
  B->tau = ar.take<double>((size_t)kb);
  B->R = ar.take<double>((size_t)s * kb * kb);
  B->Us = ar.take<double>((size_t)s * kb * kb);
  B->Vs = ar.take<double>((size_t)s * kb * kb);
  B->d = ar.take<double>((size_t)s * kb);
  B->split_elems = (size_t)8 * mx * kb;
  for (int k = 0; k < 2; ++k) B->split[k] = ar.take<double>(B->split_elems);
  B->panel_bytes = panel_work_bytes(mx, (int)kb);
  if (B->panel_bytes == 0) return false;
  B->panel = ar.take<char>(B->panel_bytes);
  B->svd_bytes = (size_t)s * block_svd_work_bytes((int)kb);
  B->svd = ar.take<char>(B->svd_bytes);
  if (precision == RRF_PREC_BF16_SKETCH) {
    B->Tb = ar.take<uint16_t>((size_t)bf16_ld(m) * n);
    B->Tbt = ar.take<uint16_t>((size_t)bf16_ld(n) * m);
    B->Gb = ar.take<uint16_t>((size_t)bf16_ld(m) * kb);
    B->Yb = ar.take<uint16_t>((size_t)bf16_ld(n) * kb);
    B->Zb = ar.take<uint16_t>((size_t)bf16_ld(m) * kb);
    B->word = ar.take<unsigned long long>(32);
    B->bwork_bytes = gemm_bf16_work_bytes(mx, kb);
    B->bwork = ar.take<char>(B->bwork_bytes);
  }
  return true;
}

// X(:, 0:k) <- X(:, 0:k) S  (rows x k times k x k) through `tmp`.
int right_mult(hipStream_t st, int64_t rows, int64_t k, double* X, int64_t ldx, const double* S,
               double* tmp, double* split, size_t split_elems) {
  if (rows <= 0 || k <= 0) return RRF_OK;
  RRF_TRY(dgemm(st, false, false, rows, k, k, 1.0, X, ldx, S, k, 0.0, tmp, rows, split,
                split_elems));
  return copy_matrix(st, rows, k, tmp, rows, X, ldx);
}

// The sketch of the mixed mode into Y (Ni x kb, FP64): bfloat16 copies of
// the scaled T22 and of G, products with FP32 accumulation, each
// intermediate column renormalised by a power of two; the last product is
// widened to FP64. Needs G (Mi x kb) in B.G.
int sketch_mixed(hipStream_t st, int64_t Mi, int64_t Ni, int64_t kb, int q, const double* T22,
                 int64_t ldt, const Bufs& B, double* Y) {
  const int64_t lm = bf16_ld(Mi), ln = bf16_ld(Ni);
  RRF_TRY(to_bf16(st, Mi, kb, B.G, Mi, nullptr, B.Gb, lm, nullptr, 0));
  RRF_TRY(maxabs(st, Mi, Ni, T22, ldt, B.word));
  RRF_TRY(to_bf16(st, Mi, Ni, T22, ldt, B.word, B.Tb, lm, B.Tbt, ln));
  // Y = T22^T G
  RRF_TRY(gemm_bf16_tn(st, Ni, kb, Mi, B.Tb, lm, B.Gb, lm, q > 0 ? B.Yb : nullptr, ln,
                       q > 0 ? nullptr : Y, Ni, B.bwork, B.bwork_bytes));
  for (int it = 0; it < q; ++it) {
    const bool last = it == q - 1;
    // Z = T22 Y = Tbt^T Y, then Y = T22^T Z
    RRF_TRY(gemm_bf16_tn(st, Mi, kb, Ni, B.Tbt, ln, B.Yb, ln, B.Zb, lm, nullptr, 0, B.bwork,
                         B.bwork_bytes));
    RRF_TRY(gemm_bf16_tn(st, Ni, kb, Mi, B.Tb, lm, B.Zb, lm, last ? nullptr : B.Yb, ln,
                         last ? Y : nullptr, Ni, B.bwork, B.bwork_bytes));
  }
  return RRF_OK;
}

// Event slots of the device context.
enum { kEvStart = 0, kEvV = 1, kEvU = 3, kEvVdone = 5, kEvUdone = 7, kEvS1 = 9, kEvSvd = 10 };

}  // namespace

bool randutv_supported(int64_t m, int64_t n, int64_t b) {
  if (b > 256) return false;
  return panel_work_bytes(std::max(m, n), (int)std::min(b, n)) > 0;
}

size_t randutv_workspace(int64_t m, int64_t n, int64_t b, int precision) {
  Arena ar;
  ar.counting = true;
  Bufs B;
  if (!plan(ar, m, n, b, precision, &B)) return 0;
  return ar.used;
}

int randutv_run(hipStream_t st, int64_t m, int64_t n, const double* A, int64_t lda, int64_t b,
                int q, uint64_t seed, double* U, double* T, double* V, void* ws,
                size_t ws_bytes, bool check_input, int precision, int* status_out) {
  Arena ar;
  ar.base = reinterpret_cast<char*>(ws);
  ar.cap = ws_bytes;
  Bufs B;
  if (!plan(ar, m, n, b, precision, &B) || ar.used > ws_bytes)
    return set_error(RRF_E_NOMEM, "randutv: workspace too small");
  *status_out = 0;
  DeviceContext* ctx = nullptr;
  RRF_TRY(device_context(&ctx));
  std::lock_guard<std::mutex> lk(ctx->mu);
  hipStream_t s1 = ctx->side[0];
  hipEvent_t* ev = ctx->ev;
  const size_t SE = B.split_elems;

  RRF_TRY(fill_u32(st, reinterpret_cast<unsigned*>(B.status), 64, 0u));
  if (check_input) RRF_TRY(check_finite(st, m, n, A, lda, B.status + 1));
  const int64_t ldt = m, ldu = m, ldv = n;
  if (T != A) RRF_TRY(copy_matrix(st, m, n, A, lda, T, ldt));
  RRF_CHECK_HIP(hipEventRecord(ev[kEvStart], st));
  RRF_CHECK_HIP(hipStreamWaitEvent(s1, ev[kEvStart], 0));
  if (U) RRF_TRY(set_identity(s1, m, m, U, ldu));
  if (V) RRF_TRY(set_identity(s1, n, n, V, ldv));

  const int64_t s = ceil_div(n, b);
  const int64_t bb = std::min(b, n);  // block slot size of R, Us, Vs, d
  for (int64_t i = 0; i < s; ++i) {
    const int64_t c0 = i * b;
    const int64_t c2 = std::min(c0 + b, n);
    const int64_t r2 = std::min(c0 + b, m);
    const int64_t Mi = m - c0, Ni = n - c0;
    const int r = (int)(i & 1);
    double* T22 = T + c0 + c0 * ldt;
    double* Tc = T + c0 * ldt;  // T(:, J2uJ3)
    double* Ri = B.R + i * bb * bb;  // ld bb
    if (r2 < m && c2 < n) {
      const int64_t kb = b;
      const int64_t N3 = n - c2;
      // ---- critical stream: sketch and V_i
      if (i >= 2) RRF_CHECK_HIP(hipStreamWaitEvent(st, ev[kEvVdone + r], 0));
      RRF_TRY(gaussian(st, seed, (uint64_t)(i + 1), Mi, kb, B.G, Mi));
      if (precision == RRF_PREC_BF16_SKETCH) {
        RRF_TRY(sketch_mixed(st, Mi, Ni, kb, q, T22, ldt, B, B.Y[r]));
      } else {
        RRF_TRY(dgemm(st, true, false, Ni, kb, Mi, 1.0, T22, ldt, B.G, Mi, 0.0, B.Y[r], Ni,
                      B.split[0], SE));
        for (int it = 0; it < q; ++it) {
          RRF_TRY(dgemm(st, false, false, Mi, kb, Ni, 1.0, T22, ldt, B.Y[r], Ni, 0.0, B.Z, Mi,
                        B.split[0], SE));
          RRF_TRY(dgemm(st, true, false, Ni, kb, Mi, 1.0, T22, ldt, B.Z, Mi, 0.0, B.Y[r], Ni,
                        B.split[0], SE));
        }
      }
      RRF_TRY(householder_panel(st, Ni, (int)kb, B.Y[r], Ni, B.Y[r], Ni, nullptr, 0, B.Tv, kb,
                                B.tau, nullptr, 0, B.panel, B.panel_bytes, B.status));
      double* Wr = B.WZ[r];          // W_v Tf_v^T, Ni x b, ld n
      double* Zt = B.WZ[r] + n * kb;  // Z^T on rows [b, Ni), ld n
      double* X = B.XW[r];            // m x b, ld m
      double* Wl = B.XW[r] + m * kb;  // W_u Tf_u^T on rows I2uI3, ld m
      RRF_TRY(dgemm(st, false, true, Ni, kb, kb, 1.0, B.Y[r], Ni, B.Tv, kb, 0.0, Wr, n, nullptr,
                    0));
      RRF_CHECK_HIP(hipEventRecord(ev[kEvV + r], st));
      // X = T(:, J2uJ3) W_v; columns J2 of T V_i
      if (i >= 2) RRF_CHECK_HIP(hipStreamWaitEvent(st, ev[kEvUdone + r], 0));
      RRF_TRY(dgemm(st, false, false, m, kb, Ni, 1.0, Tc, ldt, B.Y[r], Ni, 0.0, X, m,
                    B.split[0], SE));
      RRF_TRY(dgemm(st, false, true, m, kb, kb, -1.0, X, m, Wr, n, 1.0, Tc, ldt, nullptr, 0));
      // ---- critical stream: U_i and R from the panel T(I2uI3, J2)
      RRF_TRY(householder_panel(st, Mi, (int)kb, T22, ldt, B.Wu[r], Mi, Ri, bb, B.Tu, kb, B.tau,
                                T22, ldt, B.panel, B.panel_bytes, B.status));
      // W_u Tf_u^T on rows I2uI3, zero on rows I1 (the rows this slot held
      // two steps earlier are cleared)
      const int64_t z0 = std::max<int64_t>(0, c0 - 2 * b);
      RRF_TRY(fill_matrix(st, c0 - z0, kb, 0.0, Wl + z0, m));
      RRF_TRY(dgemm(st, false, true, Mi, kb, kb, 1.0, B.Wu[r], Mi, B.Tu, kb, 0.0, Wl + c0, m,
                    nullptr, 0));
      RRF_CHECK_HIP(hipEventRecord(ev[kEvU + r], st));
      // Z^T = T(I2uI3, J3)^T W_u - Wr(J3, :) (X(I2uI3, :)^T W_u)
      double* T23 = T + c0 + c2 * ldt;
      RRF_TRY(dgemm(st, true, false, N3, kb, Mi, 1.0, T23, ldt, B.Wu[r], Mi, 0.0, Zt + kb, n,
                    B.split[0], SE));
      RRF_TRY(dgemm(st, true, false, kb, kb, Mi, 1.0, X + c0, m, B.Wu[r], Mi, 0.0, B.S, kb,
                    B.split[0], SE));
      RRF_TRY(dgemm(st, false, false, N3, kb, kb, -1.0, Wr + kb, n, B.S, kb, 1.0, Zt + kb, n,
                    nullptr, 0));
      // T(:, J3) -= [X, W_u Tf_u^T] [Wr(J3, :), Z^T]^T
      RRF_TRY(dgemm(st, false, true, m, N3, 2 * kb, -1.0, X, m, B.WZ[r] + kb, n, 1.0,
                    T + c2 * ldt, ldt, nullptr, 0));

      // ---- side stream: V V_i and U U_i
      RRF_CHECK_HIP(hipStreamWaitEvent(s1, ev[kEvV + r], 0));
      if (V) {
        double* Vc = V + c0 * ldv;
        RRF_TRY(dgemm(s1, false, false, n, kb, Ni, 1.0, Vc, ldv, B.Y[r], Ni, 0.0, B.X1, n,
                      B.split[1], SE));
        RRF_TRY(dgemm(s1, false, true, n, Ni, kb, -1.0, B.X1, n, Wr, n, 1.0, Vc, ldv, nullptr,
                      0));
      }
      RRF_CHECK_HIP(hipEventRecord(ev[kEvVdone + r], s1));
      RRF_CHECK_HIP(hipStreamWaitEvent(s1, ev[kEvU + r], 0));
      if (U) {
        double* Uc = U + c0 * ldu;
        RRF_TRY(dgemm(s1, false, false, m, kb, Mi, 1.0, Uc, ldu, B.Wu[r], Mi, 0.0, B.X1, m,
                      B.split[1], SE));
        RRF_TRY(dgemm(s1, false, true, m, Mi, kb, -1.0, B.X1, m, Wl + c0, m, 1.0, Uc, ldu,
                      nullptr, 0));
      }
      RRF_CHECK_HIP(hipEventRecord(ev[kEvUdone + r], s1));

    } else {
      // Last block: its SVD is of T(I2uI3, J2uJ3), Mi x Ni with Mi >= Ni;
      // a tall block is first reduced by a Householder QR.
      const int64_t kb = Ni;
      if (i >= 2) RRF_CHECK_HIP(hipStreamWaitEvent(st, ev[kEvUdone + r], 0));
      double* Wl = B.XW[r] + m * bb;  // W_u Tf_u^T, Mi x kb, ld m
      if (Mi > Ni) {
        RRF_TRY(householder_panel(st, Mi, (int)kb, T22, ldt, B.Wu[r], Mi, Ri, bb, B.Tu, kb,
                                  B.tau, nullptr, 0, B.panel, B.panel_bytes, B.status));
        RRF_TRY(dgemm(st, false, true, Mi, kb, kb, 1.0, B.Wu[r], Mi, B.Tu, kb, 0.0, Wl, m,
                      nullptr, 0));
      } else {
        RRF_TRY(copy_matrix(st, kb, kb, T22, ldt, Ri, bb));
      }
      RRF_CHECK_HIP(hipEventRecord(ev[kEvU + r], st));
      RRF_CHECK_HIP(hipStreamWaitEvent(s1, ev[kEvU + r], 0));
      if (U && Mi > Ni) {
        double* Uc = U + c0 * ldu;
        RRF_TRY(dgemm(s1, false, false, m, kb, Mi, 1.0, Uc, ldu, B.Wu[r], Mi, 0.0, B.X1, m,
                      B.split[1], SE));
        RRF_TRY(dgemm(s1, false, true, m, Mi, kb, -1.0, B.X1, m, Wl, m, 1.0, Uc, ldu, nullptr,
                      0));
      }
      RRF_CHECK_HIP(hipEventRecord(ev[kEvUdone + r], s1));
    }
  }
  // ---- after the loop: all block SVDs in one launch, then the updates
  // of the processed columns they feed.
  RRF_CHECK_HIP(hipEventRecord(ev[kEvS1], s1));
  RRF_CHECK_HIP(hipStreamWaitEvent(st, ev[kEvS1], 0));
  const int64_t k_last = n - (s - 1) * b;
  RRF_TRY(block_svd_batched(st, (int)s, (int)bb, (int)k_last, B.R, bb, bb * bb, B.Us, B.d, bb,
                            B.Vs, B.svd, B.svd_bytes, B.status));
  RRF_CHECK_HIP(hipEventRecord(ev[kEvSvd], st));
  RRF_CHECK_HIP(hipStreamWaitEvent(s1, ev[kEvSvd], 0));
  for (int64_t i = 0; i < s; ++i) {
    const int64_t c0 = i * b;
    const int64_t kb = std::min(b, n - c0);
    const int64_t c2 = c0 + kb;
    const bool last = (i == s - 1);
    const double* Usi = B.Us + i * bb * bb;  // kb x kb, ld kb
    const double* Vsi = B.Vs + i * bb * bb;
    double* T22 = T + c0 + c0 * ldt;
    // T(I2uI3, J2) = [D; 0] (the panel already cleared it; the last block is
    // written whole)
    RRF_TRY(set_diag(st, last ? m - c0 : kb, kb, B.d + i * bb, T22, ldt));
    RRF_TRY(right_mult(st, c0, kb, T + c0 * ldt, ldt, Vsi, B.X0, B.split[0], SE));  // T(I1, J2)
    if (!last) {
      const int64_t N3 = n - c2;
      double* T2r = T + c0 + c2 * ldt;  // T(I2, J3) <- Us^T T(I2, J3)
      RRF_TRY(dgemm(st, true, false, kb, N3, kb, 1.0, Usi, kb, T2r, ldt, 0.0, B.Zl, kb, nullptr,
                    0));
      RRF_TRY(copy_matrix(st, kb, N3, B.Zl, kb, T2r, ldt));
    }
    if (U) RRF_TRY(right_mult(s1, m, kb, U + c0 * ldu, ldu, Usi, B.X1, B.split[1], SE));
    if (V) RRF_TRY(right_mult(s1, n, kb, V + c0 * ldv, ldv, Vsi, B.X1, B.split[1], SE));
  }
  RRF_CHECK_HIP(hipEventRecord(ev[kEvS1], s1));
  RRF_CHECK_HIP(hipStreamWaitEvent(st, ev[kEvS1], 0));
  *status_out = 0;
  return RRF_OK;
}

}  // namespace rrf
