// randUTV_basic (Alg. 3) and randUTV_boosted (Alg. 2) on one GPU.
//
// Alg. 2 changes only how V_i is built (boosted_sample below): b + p samples,
// V_i from the leading b left singular vectors of the sample matrix, and the
// p extra vectors of one step recycled into the next; the rest of each step
// is the Alg. 3 step described here.
//
// Per step i (0-based here, c0 = i b, J2 = [c0, c2), I2 = [c0, r2)):
//   1. G_i = Gaussian(seed, stream i+1), (m-c0) x b, generated in HBM;
//   2. Y = T22^T G_i, then q times Z = T22 Y, Y = T22^T Z  (MFMA GEMMs, or the
//      bfloat16 sketch of sketch_bf16.hip in the mixed mode);
//   3. [W_v, Tf_v] = Householder QR of Y (panel kernel);
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
//   7. [Us, D, Vs] = SVD(R) (one-workgroup Jacobi), then U(:,I2) Us,
//      V(:,J2) Vs, T(I2,J2) = D, T(I2,J3) = Us^T T(I2,J3), T(I1,J2) Vs.
// The last step (J3 empty) takes the SVD of the trailing block, through a
// Householder QR first when the block is tall (Sec. 4.2, tall-thin SVD).
//
// U and V. Alg. 3 multiplies U by U_i and V by V_i at every step. Nothing in
// the loop reads U or V, so every step's reflectors (W_u, Tf_u, W_v, Tf_v)
// are kept and the products U = U_1 ... U_s and V = V_1 ... V_s are formed
// after the loop, backward from the identity as LAPACK's dorgqr forms Q:
// applied last-first, U_i only touches the trailing (m - c0) x (m - c0)
// block, which costs (4/3) m^3 instead of the 2 m^2 n of the forward
// products. Consecutive steps are merged into one compact-WY factor
// (groups of kGroup steps: T = [T1, -T1 W1^T W2 T2; 0, T2] recursively), so
// each update is a GEMM with inner dimension kGroup b. U and V are formed on
// two streams while the small SVDs run, then rotated by Us and Vs.
//
// Schedule. The data dependences of a step, not the order in which Alg. 3
// lists its statements, decide what may overlap:
//  * the caller's stream carries the loop: generator, sketch, both panels
//    and the updates of T, with the whole GPU to itself;
//  * no later step depends on a block's SVD. After step i no step touches
//    columns J2 of T, U or V, and rows I2 of T are only multiplied from the
//    right, which commutes with the left rotation by Us^T. So every R is kept
//    and all the small SVDs run as one batched launch (one workgroup per
//    block) after the loop, followed by T(I2,J2) = D, T(I1,J2) Vs and
//    T(I2,J3) <- Us^T T(I2,J3) for every block.
#include <algorithm>
#include <vector>

#include "common.hpp"
#include "context.hpp"
#include "driver.hpp"
#include "kernels.hpp"
#include "trace.hpp"

namespace rrf {

// Binary exponent range of max|A| that the binary64 modes factor unscaled at
// q = 0 (divided by 2q + 1 for q power iterations).
constexpr int kGuardExp = 450;

namespace {

constexpr int kGroup = 4;  // steps merged into one compact-WY factor for U and V

// Scratch of one backward accumulation (one per stream).
struct Back {
  double* TG = nullptr;  // gk x gk merged triangular factor
  double* Sx = nullptr;  // gk x k
  double* Sy = nullptr;  // gk x k
  double* Z = nullptr;   // gk x max(m, n)
  double* Z2 = nullptr;  // gk x max(m, n)
  double* tmp = nullptr; // max(m, n) x k  (rotation by Us / Vs)
  double* split = nullptr;
};

// Alg. 2's sampling (b + p columns; kY = b + p).
struct Boost {
  double* G = nullptr;    // m x kY   Gaussian (b + p columns at the first step, b later)
  double* Z = nullptr;    // m x kY   power-iteration products
  double* Y = nullptr;    // n x kY   the sample matrix; its Householder QR in place
  double* X = nullptr;    // m x b    left sample X, then its Householder QR in place
  double* S = nullptr;    // m x kY   [Q_X(:, 1:b), W_l]
  double* Zw = nullptr;   // m x p    T22 W_next, then its Householder QR in place
  double* Qy = nullptr;   // n x kY   Q_Y(:, 1:kY)
  double* WY = nullptr;   // n x kY   W_Y(:, 1:kY) = Q_Y(:, 1:kY) U_R
  double* Wn = nullptr;   // n x p    W_next (rows: the next step's trailing columns)
  double* Ry = nullptr;   // kY x kY  R factor of Y
  double* Tf = nullptr;   // kY x kY  compact-WY factors of the three sample QRs
  double* Us = nullptr;   // kY x kY  left singular vectors of R_Y
  double* Vs = nullptr;   // kY x kY
  double* d = nullptr;    // kY
  double* C = nullptr;    // kY x kY  small products
  double* C2 = nullptr;   // kY x kY
  double* tau = nullptr;  // kY
  void* svd = nullptr;
  size_t svd_bytes = 0;
};

struct Bufs {
  int* status = nullptr;
  double* G = nullptr;      // m x b
  double* Z = nullptr;      // m x b
  double* Y = nullptr;      // n x b  sketch
  double* XW = nullptr;     // m x 2b [X, W_u Tf_u^T] (ld m; zero rows I1 on the right)
  double* WZ = nullptr;     // n x 2b [W_v Tf_v^T, Z^T] (ld n; Z^T on rows J3)
  double* S = nullptr;      // b x b  X(I2uI3, :)^T W_u
  double* X0 = nullptr;     // max(m,n) x b   (after the loop)
  double* Zl = nullptr;     // b x n          (after the loop)
  double* WU = nullptr;     // m x n  every step's W_u (block i at rows/cols c0), zero elsewhere
  double* WV = nullptr;     // n x n  every step's W_v
  double* TU = nullptr;     // s x (b x b)  Tf_u per step (ld b)
  double* TV = nullptr;     // s x (b x b)  Tf_v per step
  double* tau = nullptr;    // b
  double* R = nullptr;      // s x (b x b)
  double* Us = nullptr;     // s x (b x b)
  double* Vs = nullptr;     // s x (b x b)
  double* d = nullptr;      // s x b
  double* split = nullptr;
  size_t split_elems = 0;
  Back back[2];
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
  Boost boost;  // Alg. 2 only
  // early stop: ||T22||_F of each step
  unsigned long long* nword = nullptr;  // max|A|
  double* nparts = nullptr;             // kNormParts partial sums
  double* nout = nullptr;
};

constexpr int kNormParts = 1024;

// p < 0: Alg. 3; p >= 0: Alg. 2 with oversampling p.
bool plan(Arena& ar, int64_t m, int64_t n, int64_t b, int precision, Bufs* B, int64_t p = -1) {
  const int64_t mx = std::max(m, n);
  const int64_t kb = std::min(b, n);
  const int64_t s = ceil_div(n, b);
  const int64_t gk = kGroup * kb;
  B->status = ar.take<int>(64);
  B->nword = ar.take<unsigned long long>(4);
  B->nparts = ar.take<double>(kNormParts);
  B->nout = ar.take<double>(4);
  B->G = ar.take<double>((size_t)m * kb);
  B->Z = ar.take<double>((size_t)m * kb);
  B->Y = ar.take<double>((size_t)n * kb);
  B->XW = ar.take<double>((size_t)m * 2 * kb);
  B->WZ = ar.take<double>((size_t)n * 2 * kb);
  B->S = ar.take<double>((size_t)kb * kb);
  B->X0 = ar.take<double>((size_t)mx * kb);
  B->Zl = ar.take<double>((size_t)kb * n);
  B->WU = ar.take<double>((size_t)m * n);
  B->WV = ar.take<double>((size_t)n * n);
  B->TU = ar.take<double>((size_t)s * kb * kb);
  B->TV = ar.take<double>((size_t)s * kb * kb);
  B->tau = ar.take<double>((size_t)kb);
  B->R = ar.take<double>((size_t)s * kb * kb);
  B->Us = ar.take<double>((size_t)s * kb * kb);
  B->Vs = ar.take<double>((size_t)s * kb * kb);
  B->d = ar.take<double>((size_t)s * kb);
  B->split_elems = (size_t)8 * mx * kb;
  B->split = ar.take<double>(B->split_elems);
  for (int t = 0; t < 2; ++t) {
    Back& k = B->back[t];
    k.TG = ar.take<double>((size_t)gk * gk);
    k.Sx = ar.take<double>((size_t)gk * kb);
    k.Sy = ar.take<double>((size_t)gk * kb);
    k.Z = ar.take<double>((size_t)gk * mx);
    k.Z2 = ar.take<double>((size_t)gk * mx);
    k.tmp = ar.take<double>((size_t)mx * kb);
    k.split = ar.take<double>(B->split_elems);
  }
  const int64_t pw = p > 0 ? std::min(p, std::max<int64_t>(n - kb, 0)) : 0;  // widest p_i
  const int64_t ky = kb + pw;
  B->panel_bytes = panel_work_bytes(mx, (int)kb);
  if (B->panel_bytes == 0) return false;
  if (p >= 0) {
    // the sample QRs have widths b, p_i <= pw and b + p_i <= ky
    for (int64_t w : {pw, ky}) {
      if (w < 1) continue;
      const size_t pb = panel_work_bytes(mx, (int)w);
      if (pb == 0) return false;
      B->panel_bytes = std::max(B->panel_bytes, pb);
    }
  }
  B->panel = ar.take<char>(B->panel_bytes);
  B->svd_bytes = (size_t)s * block_svd_work_bytes((int)kb);
  B->svd = ar.take<char>(B->svd_bytes);
  if (precision == RRF_PREC_BF16_SKETCH || precision == RRF_PREC_BF16_X3 ||
      precision == RRF_PREC_BF16_X6) {
    B->Tb = ar.take<uint16_t>((size_t)bf16_ld(m) * n);
    B->Tbt = ar.take<uint16_t>((size_t)bf16_ld(n) * m);
    B->Gb = ar.take<uint16_t>((size_t)bf16_ld(m) * kb);
    B->Yb = ar.take<uint16_t>((size_t)bf16_ld(n) * kb);
    B->Zb = ar.take<uint16_t>((size_t)bf16_ld(m) * kb);
    B->word = ar.take<unsigned long long>(32);
    B->bwork_bytes = gemm_bf16_work_bytes(mx, kb);
    B->bwork = ar.take<char>(B->bwork_bytes);
  }
  if (p >= 0) {
    Boost& X = B->boost;
    X.G = ar.take<double>((size_t)m * ky);
    X.Z = ar.take<double>((size_t)m * ky);
    X.Y = ar.take<double>((size_t)n * ky);
    X.X = ar.take<double>((size_t)m * kb);
    X.S = ar.take<double>((size_t)m * ky);
    X.Zw = ar.take<double>((size_t)m * std::max<int64_t>(pw, 1));
    X.Qy = ar.take<double>((size_t)n * ky);
    X.WY = ar.take<double>((size_t)n * ky);
    X.Wn = ar.take<double>((size_t)n * std::max<int64_t>(pw, 1));
    X.Ry = ar.take<double>((size_t)ky * ky);
    X.Tf = ar.take<double>((size_t)ky * ky);
    X.Us = ar.take<double>((size_t)ky * ky);
    X.Vs = ar.take<double>((size_t)ky * ky);
    X.d = ar.take<double>((size_t)ky);
    X.C = ar.take<double>((size_t)ky * ky);
    X.C2 = ar.take<double>((size_t)ky * ky);
    X.tau = ar.take<double>((size_t)ky);
    X.svd_bytes = left_svd_work_bytes((int)ky);
    X.svd = ar.take<char>(X.svd_bytes);
  }
  return true;
}

// The sample and V_i of step i (0-based) of Alg. 2, for the trailing block
// T22 (Mi x Ni) with b + pi samples: Y (Sec. 4.3: at the first step b + pi
// fresh samples through q power steps; later b fresh ones through q - 1
// power steps and one more product, projected off W_l = orth(T22 W_next),
// orthonormalised and sampled together with W_l), then W_Y(:, 0:k) from the
// tall-thin SVD of Y (Householder QR, SVD of R_Y, Q_Y U_R), the Householder
// QR of W_Y(:, 0:b) into (Wv, Tv), and W_next = (V_i^T W_Y(:, b:k))(b:, :)
// for the next step (its rows are the next trailing block's columns).
int boosted_sample(hipStream_t st, int64_t i, int64_t Mi, int64_t Ni, int64_t b, int64_t pi,
                   int q, uint64_t seed, const double* T22, int64_t ldt, const Bufs& B,
                   double* Wv, int64_t ldwv, double* Tv, int64_t ldtv, size_t SE) {
  const Boost& X = B.boost;
  const int64_t k = b + pi;
  double* Y = X.Y;  // Ni x k, ld Ni
  if (i == 0) {
    RRF_TRY(gaussian(st, seed, 1, Mi, k, X.G, Mi));
    RRF_TRY(dgemm(st, true, false, Ni, k, Mi, 1.0, T22, ldt, X.G, Mi, 0.0, Y, Ni, B.split, SE));
    for (int it = 0; it < q; ++it) {
      RRF_TRY(dgemm(st, false, false, Mi, k, Ni, 1.0, T22, ldt, Y, Ni, 0.0, X.Z, Mi, B.split, SE));
      RRF_TRY(dgemm(st, true, false, Ni, k, Mi, 1.0, T22, ldt, X.Z, Mi, 0.0, Y, Ni, B.split, SE));
    }
  } else {
    RRF_TRY(gaussian(st, seed, (uint64_t)(i + 1), Mi, b, X.G, Mi));
    if (q >= 1) {
      RRF_TRY(dgemm(st, true, false, Ni, b, Mi, 1.0, T22, ldt, X.G, Mi, 0.0, Y, Ni, B.split, SE));
      for (int it = 0; it + 1 < q; ++it) {
        RRF_TRY(dgemm(st, false, false, Mi, b, Ni, 1.0, T22, ldt, Y, Ni, 0.0, X.Z, Mi, B.split,
                      SE));
        RRF_TRY(dgemm(st, true, false, Ni, b, Mi, 1.0, T22, ldt, X.Z, Mi, 0.0, Y, Ni, B.split,
                      SE));
      }
      RRF_TRY(dgemm(st, false, false, Mi, b, Ni, 1.0, T22, ldt, Y, Ni, 0.0, X.X, Mi, B.split, SE));
    } else {
      RRF_TRY(copy_matrix(st, Mi, b, X.G, Mi, X.X, Mi));
    }
    double* Wl = X.S + b * Mi;  // S = [Q_X(:, 0:b), W_l], ld Mi
    if (pi > 0) {
      // W_l = orth(T22 W_next); X -= W_l (W_l^T X)
      RRF_TRY(dgemm(st, false, false, Mi, pi, Ni, 1.0, T22, ldt, X.Wn, Ni, 0.0, X.Zw, Mi, B.split,
                    SE));
      RRF_TRY(householder_panel(st, Mi, (int)pi, X.Zw, Mi, X.Zw, Mi, nullptr, 0, X.Tf, pi, X.tau,
                                nullptr, 0, B.panel, B.panel_bytes, B.status));
      RRF_TRY(thin_q(st, Mi, pi, X.Zw, Mi, X.Tf, pi, Wl, Mi, X.C));
      RRF_TRY(dgemm(st, true, false, pi, b, Mi, 1.0, Wl, Mi, X.X, Mi, 0.0, X.C, pi, B.split, SE));
      RRF_TRY(dgemm(st, false, false, Mi, b, pi, -1.0, Wl, Mi, X.C, pi, 1.0, X.X, Mi, nullptr, 0));
    }
    RRF_TRY(householder_panel(st, Mi, (int)b, X.X, Mi, X.X, Mi, nullptr, 0, X.Tf, b, X.tau,
                              nullptr, 0, B.panel, B.panel_bytes, B.status));
    RRF_TRY(thin_q(st, Mi, b, X.X, Mi, X.Tf, b, X.S, Mi, X.C));
    RRF_TRY(dgemm(st, true, false, Ni, k, Mi, 1.0, T22, ldt, X.S, Mi, 0.0, Y, Ni, B.split, SE));
  }
  // W_Y(:, 0:k) = Q_Y(:, 0:k) U_R with Y = Q_Y R_Y and R_Y = U_R D V_R^T
  RRF_TRY(householder_panel(st, Ni, (int)k, Y, Ni, Y, Ni, X.Ry, k, X.Tf, k, X.tau, nullptr, 0,
                            B.panel, B.panel_bytes, B.status));
  RRF_TRY(left_svd(st, (int)k, X.Ry, k, X.Us, X.d, X.svd, X.svd_bytes, B.status));
  RRF_TRY(thin_q(st, Ni, k, Y, Ni, X.Tf, k, X.Qy, Ni, X.C));
  RRF_TRY(dgemm(st, false, false, Ni, k, k, 1.0, X.Qy, Ni, X.Us, k, 0.0, X.WY, Ni, nullptr, 0));
  // [V_i, ~] = HQR_full(W_Y(:, 0:b))
  RRF_TRY(householder_panel(st, Ni, (int)b, X.WY, Ni, Wv, ldwv, nullptr, 0, Tv, ldtv, X.tau,
                            nullptr, 0, B.panel, B.panel_bytes, B.status));
  if (pi > 0) {
    // W_next = (W_Y2 - Wv Tv^T (Wv^T W_Y2))(b:, :), W_Y2 = W_Y(:, b:k)
    double* WY2 = X.WY + b * Ni;
    RRF_TRY(dgemm(st, true, false, b, pi, Ni, 1.0, Wv, ldwv, WY2, Ni, 0.0, X.C, b, B.split, SE));
    RRF_TRY(dgemm(st, true, false, b, pi, b, 1.0, Tv, ldtv, X.C, b, 0.0, X.C2, b, nullptr, 0));
    RRF_TRY(dgemm(st, false, false, Ni, pi, b, -1.0, Wv, ldwv, X.C2, b, 1.0, WY2, Ni, nullptr, 0));
    RRF_TRY(copy_matrix(st, Ni - b, pi, WY2 + b, Ni, X.Wn, Ni - b));
  }
  return RRF_OK;
}

// X(:, 0:k) <- X(:, 0:k) S  (rows x k times k x k): in place when one
// 128-wide tile spans X's k columns, else through `tmp`.
int right_mult(hipStream_t st, int64_t rows, int64_t k, double* X, int64_t ldx, const double* S,
               double* tmp, double* split, size_t split_elems) {
  if (rows <= 0 || k <= 0) return RRF_OK;
  if (dgemm_in_place_fits(false, false, rows, k, X, ldx, S, k, X, ldx))
    return dgemm_in_place(st, false, false, rows, k, k, 1.0, X, ldx, S, k, X, ldx, split,
                          split_elems);
  RRF_TRY(dgemm(st, false, false, rows, k, k, 1.0, X, ldx, S, k, 0.0, tmp, rows, split,
                split_elems));
  return copy_matrix(st, rows, k, tmp, rows, X, ldx);
}

// Q(:, 0:ncols) (N x ncols, ld ldq) <- (H_0 H_1 ... H_{s-1})(:, 0:ncols), formed
// backward from the identity's first ncols columns (ncols = N: all of Q; the
// thin U of a tall A needs only its first n columns). Step i's reflectors are the kbs[i] columns of Wall (N x *, ld
// ldw) starting at row and column i*b (zero above), with triangular factor
// Tall + i*bb*bb (ld bb); kbs[i] = 0 means none. Groups of up to kGroup
// consecutive steps are merged into one compact-WY factor
// T_G = [T_1, -T_1 (W_1^T W_2) T_2; 0, T_2] (recursively) and applied to the
// trailing block Q(ca:, ca:) as three GEMMs.
int accumulate_backward(hipStream_t st, int64_t N, double* Q, int64_t ldq, const double* Wall,
                        int64_t ldw, const double* Tall, int64_t bb, int64_t b,
                        const std::vector<int64_t>& kbs, const Back& k, size_t split_elems,
                        GemmFn upd, int64_t ncols) {
  RRF_TRY(set_identity(st, N, ncols, Q, ldq));
  int64_t i1 = (int64_t)kbs.size();
  while (i1 > 0) {
    while (i1 > 0 && kbs[i1 - 1] == 0) --i1;
    if (i1 == 0) break;
    int64_t i0 = std::max<int64_t>(0, i1 - kGroup);
    for (int64_t i = i1 - 1; i >= i0; --i)
      if (kbs[i] == 0) { i0 = i + 1; break; }
    const int64_t ca = i0 * b;
    int64_t width = 0;
    for (int64_t i = i0; i < i1; ++i) width += kbs[i];
    const int64_t Nq = N - ca;
    const double* WG = Wall + ca + ca * ldw;
    RRF_TRY(fill_matrix(st, width, width, 0.0, k.TG, width));
    int64_t p = 0;
    for (int64_t i = i0; i < i1; ++i) {
      const int64_t kbi = kbs[i];
      const double* Ti = Tall + i * bb * bb;
      const double* Wi = WG + p * ldw;  // rows ca.., zero above row ca + p
      if (p > 0) {
        // T_G(0:p, p:p+kbi) = -T_G(0:p, 0:p) (W_G(:, 0:p)^T W_i) T_i
        RRF_TRY(dgemm(st, true, false, p, kbi, Nq, 1.0, WG, ldw, Wi, ldw, 0.0, k.Sx, p, k.split,
                      split_elems));
        RRF_TRY(dgemm(st, false, false, p, kbi, p, 1.0, k.TG, width, k.Sx, p, 0.0, k.Sy, p,
                      nullptr, 0));
        RRF_TRY(dgemm(st, false, false, p, kbi, kbi, -1.0, k.Sy, p, Ti, bb, 0.0,
                      k.TG + p * width, width, nullptr, 0));
      }
      RRF_TRY(copy_matrix(st, kbi, kbi, Ti, bb, k.TG + p + p * width, width));
      p += kbi;
    }
    // Q(ca:, ca:nc) <- (I - W_G T_G W_G^T) Q(ca:, ca:nc)
    double* Qb = Q + ca + ca * ldq;
    const int64_t Nc = ncols - ca;
    RRF_TRY(upd(st, true, false, width, Nc, Nq, 1.0, WG, ldw, Qb, ldq, 0.0, k.Z, width, k.split,
                split_elems));
    RRF_TRY(dgemm(st, false, false, width, Nc, width, 1.0, k.TG, width, k.Z, width, 0.0, k.Z2,
                  width, nullptr, 0));
    RRF_TRY(upd(st, false, false, Nq, Nc, width, -1.0, WG, ldw, k.Z2, width, 1.0, Qb, ldq,
                nullptr, 0));
    i1 = i0;
  }
  return RRF_OK;
}

// Q(:, c0:) <- Q(:, c0:) (I - W_i Tf_i W_i^T) for the steps i >= i0 in order:
// continues U or V of an earlier (partial) run whose steps before i0 are
// already in Q. Scratch: k.Z and k.Z2 (N x kb each).
int accumulate_forward(hipStream_t st, int64_t N, double* Q, int64_t ldq, const double* Wall,
                       int64_t ldw, const double* Tall, int64_t bb, int64_t b,
                       const std::vector<int64_t>& kbs, int64_t i0, const Back& k,
                       size_t split_elems, GemmFn upd) {
  for (int64_t i = i0; i < (int64_t)kbs.size(); ++i) {
    const int64_t kb = kbs[i];
    if (kb == 0) continue;
    const int64_t c0 = i * b;
    const double* W = Wall + c0 + c0 * ldw;  // (N - c0) x kb
    double* Qc = Q + c0 * ldq;
    RRF_TRY(upd(st, false, false, N, kb, N - c0, 1.0, Qc, ldq, W, ldw, 0.0, k.Z, N, k.split,
                split_elems));
    RRF_TRY(dgemm(st, false, false, N, kb, kb, 1.0, k.Z, N, Tall + i * bb * bb, bb, 0.0, k.Z2, N,
                  nullptr, 0));
    RRF_TRY(upd(st, false, true, N, N - c0, kb, -1.0, k.Z2, N, W, ldw, 1.0, Qc, ldq, nullptr, 0));
  }
  return RRF_OK;
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
enum { kEvLoop = 0, kEvSvd = 1, kEvU = 2, kEvV = 3 };

}  // namespace

bool randutv_supported(int64_t m, int64_t n, int64_t b) {
  if (b > 256) return false;
  return panel_work_bytes(std::max(m, n), (int)std::min(b, n)) > 0;
}

size_t randutv_workspace(int64_t m, int64_t n, int64_t b, int precision, int64_t p) {
  Arena ar;
  ar.counting = true;
  Bufs B;
  if (!plan(ar, m, n, b, precision, &B, p)) return 0;
  return ar.used;
}

int randutv_run(hipStream_t st, int64_t m, int64_t n, const double* A, int64_t lda, int64_t b,
                int q, uint64_t seed, double* U, double* T, double* V, void* ws,
                size_t ws_bytes, bool check_input, int precision, int* status_out, int64_t p,
                const EarlyStop* stop, bool thin_u) {
  if (stop && ceil_div(m, 256) > kNormParts)
    return set_error(RRF_E_NOTSUP, "randutv: early stop needs m <= 262144");
  Arena ar;
  ar.base = reinterpret_cast<char*>(ws);
  ar.cap = ws_bytes;
  Bufs B;
  if (!plan(ar, m, n, b, precision, &B, p) || ar.used > ws_bytes)
    return set_error(RRF_E_NOMEM, "randutv: workspace too small");
  const bool boosted = p >= 0;
  *status_out = 0;
  DeviceContext* ctx = nullptr;
  RRF_TRY(device_context(&ctx));
  std::lock_guard<std::mutex> lk(ctx->mu);
  hipEvent_t* ev = ctx->ev;
  const size_t SE = B.split_elems;
  const bool x6 = precision == RRF_PREC_BF16_X6;
  const bool x3 = precision == RRF_PREC_BF16_X3 || x6;  // split-bfloat16 updates
  const bool mixed_sketch = precision == RRF_PREC_BF16_SKETCH || x3;
  // the products that update T, U and V
  const GemmFn upd = x6 ? gemm_x6 : (x3 ? gemm_x3 : dgemm);
  unsigned long long* scale_word = B.nword + 2;  // max|A|, for the scaling of T

  RRF_TRY(fill_u32(st, reinterpret_cast<unsigned*>(B.status), 64, 0u));
  if (check_input) RRF_TRY(check_finite(st, m, n, A, lda, B.status + 1));
  const int64_t ldt = m, ldu = m, ldv = n;
  if (T != A) RRF_TRY(copy_matrix(st, m, n, A, lda, T, ldt));
  // T = 2^-e A with max|T| in [0.5, 1) (exact, undone at the end). The split
  // modes always scale: every entry of T, and of the products formed from
  // it, stays inside the binary32 range of the split. The binary64 modes
  // scale only a max|A| beyond 2^+-g: the sketch grows like |A|^(2q+1) and
  // the Householder norms of the sketch and of T sum its squares, so
  // g = kGuardExp / (2q+1) keeps those squares inside the binary64 range.
  const int guard = x3 ? 0 : std::max(1, kGuardExp / (2 * q + 1));
  RRF_TRY(maxabs(st, m, n, T, ldt, scale_word));
  RRF_TRY(scale_pow2(st, m, n, T, ldt, scale_word, false, guard));
  // reflector stores: zero outside each step's block
  if (U) RRF_TRY(fill_matrix(st, m, n, 0.0, B.WU, m));
  if (V) RRF_TRY(fill_matrix(st, n, n, 0.0, B.WV, n));

  const int64_t s = ceil_div(n, b);
  const int64_t bb = std::min(b, n);  // block slot size of R, Us, Vs, d, TU, TV
  std::vector<int64_t> ku(s, 0), kv(s, 0);  // reflector columns per step
  const int64_t i0 = stop ? stop->i0 : 0;    // first step (> 0: resuming)
  int64_t s_done = i0;                       // steps carried out
  double e0 = 0.0;
  if (stop) RRF_TRY(maxabs(st, m, n, T, ldt, B.nword));
  if (i0 > 0) {
    // ||A||_F = ||T||_F (orthogonal invariance): the reference of the tolerance
    RRF_TRY(frob_norm(st, m, n, T, ldt, B.nword, B.nparts, kNormParts, B.nout));
    RRF_CHECK_HIP(hipMemcpyAsync(&e0, B.nout, sizeof e0, hipMemcpyDeviceToHost, st));
    RRF_CHECK_HIP(hipStreamSynchronize(st));
  }
  for (int64_t i = i0; i < s; ++i) {
    const int64_t c0 = i * b;
    const int64_t c2 = std::min(c0 + b, n);
    const int64_t r2 = std::min(c0 + b, m);
    const int64_t Mi = m - c0, Ni = n - c0;
    double* T22 = T + c0 + c0 * ldt;
    if (stop) {
      // Sec. 4.1: ||A - A_k||_F = ||T22||_F after c0 = k columns; stop once it
      // is within the tolerance, or at the rank cap
      if (c0 >= stop->kmax) break;
      RRF_TRY(frob_norm(st, Mi, Ni, T22, ldt, B.nword, B.nparts, kNormParts, B.nout));
      double e = 0.0;
      RRF_CHECK_HIP(hipMemcpyAsync(&e, B.nout, sizeof e, hipMemcpyDeviceToHost, st));
      RRF_CHECK_HIP(hipStreamSynchronize(st));
      if (i == 0) e0 = e;
      if (e <= stop->tol * e0) break;
    }
    s_done = i + 1;
    double* Tc = T + c0 * ldt;  // T(:, J2uJ3)
    double* Ri = B.R + i * bb * bb;  // ld bb
    double* Tu = B.TU + i * bb * bb;  // ld bb
    double* Wu = B.WU + c0 + c0 * m;  // ld m
    if (r2 < m && c2 < n) {
      const int64_t kb = b;
      const int64_t N3 = n - c2;
      double* Tv = B.TV + i * bb * bb;
      double* Wv = B.WV + c0 + c0 * n;  // ld n
      double* Wr = B.WZ;                // W_v Tf_v^T, Ni x b, ld n
      double* Zt = B.WZ + n * kb;       // Z^T on rows [b, Ni), ld n
      double* X = B.XW;                 // m x b, ld m
      double* Wl = B.XW + m * kb;       // W_u Tf_u^T on rows I2uI3, ld m
      ku[i] = kb;
      kv[i] = kb;
      // ---- sketch and V_i
      if (boosted) {
        const int64_t pi = std::min<int64_t>(p, Ni - kb);
        RRF_TRY(boosted_sample(st, i, Mi, Ni, kb, pi, q, seed, T22, ldt, B, Wv, n, Tv, bb, SE));
      } else {
      RRF_TRY(gaussian(st, seed, (uint64_t)(i + 1), Mi, kb, B.G, Mi));
      if (mixed_sketch) {
        RRF_TRY(sketch_mixed(st, Mi, Ni, kb, q, T22, ldt, B, B.Y));
      } else {
        RRF_TRY(dgemm(st, true, false, Ni, kb, Mi, 1.0, T22, ldt, B.G, Mi, 0.0, B.Y, Ni,
                      B.split, SE));
        for (int it = 0; it < q; ++it) {
          RRF_TRY(dgemm(st, false, false, Mi, kb, Ni, 1.0, T22, ldt, B.Y, Ni, 0.0, B.Z, Mi,
                        B.split, SE));
          RRF_TRY(dgemm(st, true, false, Ni, kb, Mi, 1.0, T22, ldt, B.Z, Mi, 0.0, B.Y, Ni,
                        B.split, SE));
        }
      }
      RRF_TRY(householder_panel(st, Ni, (int)kb, B.Y, Ni, Wv, n, nullptr, 0, Tv, bb, B.tau,
                                nullptr, 0, B.panel, B.panel_bytes, B.status));
      }
      RRF_TRY(dgemm(st, false, true, Ni, kb, kb, 1.0, Wv, n, Tv, bb, 0.0, Wr, n, nullptr, 0));
      // X = T(:, J2uJ3) W_v; columns J2 of T V_i
      RRF_TRY(upd(st, false, false, m, kb, Ni, 1.0, Tc, ldt, Wv, n, 0.0, X, m, B.split, SE));
      RRF_TRY(upd(st, false, true, m, kb, kb, -1.0, X, m, Wr, n, 1.0, Tc, ldt, nullptr, 0));
      // ---- U_i and R from the panel T(I2uI3, J2)
      RRF_TRY(householder_panel(st, Mi, (int)kb, T22, ldt, Wu, m, Ri, bb, Tu, bb, B.tau, T22, ldt,
                                B.panel, B.panel_bytes, B.status));
      // W_u Tf_u^T on rows I2uI3, zero on rows I1 (clear the rows the
      // previous step held)
      const int64_t z0 = std::max<int64_t>(0, c0 - b);
      RRF_TRY(fill_matrix(st, c0 - z0, kb, 0.0, Wl + z0, m));
      RRF_TRY(dgemm(st, false, true, Mi, kb, kb, 1.0, Wu, m, Tu, bb, 0.0, Wl + c0, m, nullptr, 0));
      // Z^T = T(I2uI3, J3)^T W_u - Wr(J3, :) (X(I2uI3, :)^T W_u)
      double* T23 = T + c0 + c2 * ldt;
      RRF_TRY(upd(st, true, false, N3, kb, Mi, 1.0, T23, ldt, Wu, m, 0.0, Zt + kb, n, B.split,
                  SE));
      RRF_TRY(dgemm(st, true, false, kb, kb, Mi, 1.0, X + c0, m, Wu, m, 0.0, B.S, kb, B.split,
                    SE));
      RRF_TRY(upd(st, false, false, N3, kb, kb, -1.0, Wr + kb, n, B.S, kb, 1.0, Zt + kb, n,
                  nullptr, 0));
      // T(:, J3) -= [X, W_u Tf_u^T] [Wr(J3, :), Z^T]^T
      RRF_TRY(upd(st, false, true, m, N3, 2 * kb, -1.0, X, m, B.WZ + kb, n, 1.0, T + c2 * ldt,
                  ldt, nullptr, 0));
    } else {
      // Last block: its SVD is of T(I2uI3, J2uJ3), Mi x Ni with Mi >= Ni;
      // a tall block is first reduced by a Householder QR.
      const int64_t kb = Ni;
      if (Mi > Ni) {
        RRF_TRY(householder_panel(st, Mi, (int)kb, T22, ldt, Wu, m, Ri, bb, Tu, bb, B.tau,
                                  nullptr, 0, B.panel, B.panel_bytes, B.status));
        ku[i] = kb;
      } else {
        RRF_TRY(copy_matrix(st, kb, kb, T22, ldt, Ri, bb));
      }
    }
  }
  RRF_CHECK_HIP(hipEventRecord(ev[kEvLoop], st));
  // ---- U and V from the kept reflectors, on the side streams, while the
  // small SVDs run
  const int64_t k_last = s_done == s ? n - (s - 1) * b : bb;
  hipStream_t su = ctx->side[0], sv = ctx->side[1];
  trace_mark_stream(su);
  trace_mark_stream(sv);
  if (U) {
    RRF_CHECK_HIP(hipStreamWaitEvent(su, ev[kEvLoop], 0));
    if (i0 > 0)
      RRF_TRY(accumulate_forward(su, m, U, ldu, B.WU, m, B.TU, bb, b, ku, i0, B.back[0], SE, upd));
    else
      RRF_TRY(accumulate_backward(su, m, U, ldu, B.WU, m, B.TU, bb, b, ku, B.back[0], SE, upd,
                                  thin_u ? n : m));
  }
  if (V) {
    RRF_CHECK_HIP(hipStreamWaitEvent(sv, ev[kEvLoop], 0));
    if (i0 > 0)
      RRF_TRY(accumulate_forward(sv, n, V, ldv, B.WV, n, B.TV, bb, b, kv, i0, B.back[1], SE, upd));
    else
      RRF_TRY(accumulate_backward(sv, n, V, ldv, B.WV, n, B.TV, bb, b, kv, B.back[1], SE, upd, n));
  }
  if (s_done > i0)
    RRF_TRY(block_svd_batched(st, (int)(s_done - i0), (int)bb, (int)k_last, B.R + i0 * bb * bb, bb,
                              bb * bb, B.Us + i0 * bb * bb, B.d + i0 * bb, bb,
                              B.Vs + i0 * bb * bb, B.svd, B.svd_bytes, B.status));
  RRF_CHECK_HIP(hipEventRecord(ev[kEvSvd], st));
  if (U) RRF_CHECK_HIP(hipStreamWaitEvent(su, ev[kEvSvd], 0));
  if (V) RRF_CHECK_HIP(hipStreamWaitEvent(sv, ev[kEvSvd], 0));
  for (int64_t i = i0; i < s_done; ++i) {
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
    RRF_TRY(right_mult(st, c0, kb, T + c0 * ldt, ldt, Vsi, B.X0, B.split, SE));  // T(I1, J2)
    if (!last) {
      const int64_t N3 = n - c2;
      double* T2r = T + c0 + c2 * ldt;  // T(I2, J3) <- Us^T T(I2, J3)
      if (dgemm_in_place_fits(true, false, kb, N3, Usi, kb, T2r, ldt, T2r, ldt)) {
        RRF_TRY(dgemm_in_place(st, true, false, kb, N3, kb, 1.0, Usi, kb, T2r, ldt, T2r, ldt,
                               nullptr, 0));
      } else {
        RRF_TRY(dgemm(st, true, false, kb, N3, kb, 1.0, Usi, kb, T2r, ldt, 0.0, B.Zl, kb,
                      nullptr, 0));
        RRF_TRY(copy_matrix(st, kb, N3, B.Zl, kb, T2r, ldt));
      }
    }
    if (U)
      RRF_TRY(right_mult(su, m, kb, U + c0 * ldu, ldu, Usi, B.back[0].tmp, B.back[0].split, SE));
    if (V)
      RRF_TRY(right_mult(sv, n, kb, V + c0 * ldv, ldv, Vsi, B.back[1].tmp, B.back[1].split, SE));
  }
  if (U) {
    RRF_CHECK_HIP(hipEventRecord(ev[kEvU], su));
    RRF_CHECK_HIP(hipStreamWaitEvent(st, ev[kEvU], 0));
  }
  if (V) {
    RRF_CHECK_HIP(hipEventRecord(ev[kEvV], sv));
    RRF_CHECK_HIP(hipStreamWaitEvent(st, ev[kEvV], 0));
  }
  RRF_TRY(scale_pow2(st, m, n, T, ldt, scale_word, true, guard));
  if (stop && stop->k_out) *stop->k_out = std::min(s_done * b, n);
  *status_out = 0;
  return RRF_OK;
}

}  // namespace rrf
