// FP64 MFMA tiles: the operand staging shared by the single GEMM
// (gemm_f64.hip) and the grouped GEMM of the batched path (batched.hip), and
// the tile loop of the grouped GEMM (the single GEMM keeps its own copy of
// the loop, which compiles to fewer instructions for its fixed 2 x 2 grid).
//
// A workgroup of 256 threads (four wave64s in a GM x GN grid) computes a
// BM x BN tile of op(A) op(B) over a K range; each wave owns (BM/GM) x
// (BN/GN) as 16 x 16 v_mfma_f64_16x16x4f64 sub-tiles. K is walked in kBK =
// 16 slices through two LDS buffers: the global loads of slice t+1 are
// issued before the matrix cores start on slice t and are written to the
// other buffer afterwards, one barrier per slice. LDS layout follows the
// operand's contiguous dimension in HBM: "mn-major" operands (A for op = N,
// B for op = T) are stored [k][mn] with a row stride of MN + 16 doubles,
// "k-major" ones [mn][k] with an odd row stride of kBK + 1; both the copy
// and the MFMA operand fetch then spread over distinct banks. With VEC,
// global loads move 16 bytes per lane along the contiguous dimension. The
// MFMA computes the transposed tile (operands swapped), so lane l, register
// r of a sub-tile holds C(row l % 16, column 4 r + l / 16) and the stores of
// a quarter-wave coalesce.
#pragma once

#include "common.hpp"

namespace rrf {
namespace tile {

constexpr int kBK = 16;
constexpr int kThreads = 256;

// One operand tile (MN x kBK of op(X)) in LDS, with its copy from HBM.
// KMAJOR: the operand is contiguous along k in HBM (A for op=T, B for op=N).
template <int MN, bool KMAJOR, bool VEC>
struct Operand {
  static constexpr int LD = KMAJOR ? (kBK + 1) : (MN + 16);  // LDS row stride
  static constexpr int SIZE = KMAJOR ? MN * LD : kBK * LD;    // doubles per buffer
  static constexpr int ELEMS = MN * kBK;
  static constexpr int PER_T = ELEMS / kThreads;              // doubles per thread
  static constexpr int VW = (VEC && PER_T >= 2) ? 2 : 1;      // doubles per load
  static constexpr int LOADS = PER_T / VW;
  static_assert(PER_T >= 1 && PER_T * kThreads == ELEMS, "operand tile shape");

  // Element (mn, k) of the tile for load slot (tid, r): consecutive threads
  // walk the operand's contiguous dimension in HBM.
  __device__ static inline void coord(int tid, int r, int& mn, int& k) {
    const int e = (tid + kThreads * r) * VW;
    if (KMAJOR) {
      k = e % kBK;
      mn = e / kBK;
    } else {
      mn = e % MN;
      k = e / MN;
    }
  }
  // Load the slice [k0, k0 + kBK) into registers. X is op(X)'s storage with
  // leading dimension ld; the tile starts at row/column mn0.
  __device__ static inline void load(double (&reg)[PER_T], const double* X, int64_t ld,
                                     int64_t mn0, int64_t mn_end, int64_t k0, int64_t k_end,
                                     int tid) {
#pragma unroll
    for (int r = 0; r < LOADS; ++r) {
      int mn, k;
      coord(tid, r, mn, k);
      const int64_t gm = mn0 + mn, gk = k0 + k;
      const double* p = KMAJOR ? X + gk + gm * ld : X + gm + gk * ld;
      if (VW == 2) {
        // the pair runs along the contiguous dimension
        const bool in0 = gm < mn_end && gk < k_end;
        const bool in1 = KMAJOR ? (gm < mn_end && gk + 1 < k_end) : (gm + 1 < mn_end && gk < k_end);
        if (in0 && in1) {
          const double2 v = *reinterpret_cast<const double2*>(p);
          reg[2 * r] = v.x;
          reg[2 * r + 1] = v.y;
        } else {
          reg[2 * r] = in0 ? p[0] : 0.0;
          reg[2 * r + 1] = in1 ? p[1] : 0.0;
        }
      } else {
        reg[r] = (gm < mn_end && gk < k_end) ? *p : 0.0;
      }
    }
  }
  __device__ static inline void store(double* lds, const double (&reg)[PER_T], int tid) {
#pragma unroll
    for (int r = 0; r < LOADS; ++r) {
      int mn, k;
      coord(tid, r, mn, k);
#pragma unroll
      for (int v = 0; v < VW; ++v) {
        const int mm = KMAJOR ? mn : mn + v;
        const int kk = KMAJOR ? k + v : k;
        lds[KMAJOR ? mm * LD + kk : kk * LD + mm] = reg[VW * r + v];
      }
    }
  }
  // MFMA operand: element (mn, k) of the tile.
  __device__ static inline double frag(const double* lds, int mn, int k) {
    return lds[KMAJOR ? mn * LD + k : k * LD + mn];
  }
};

template <int BM, int BN, bool TA, bool TB, bool VEC, int GM = 2, int GN = 2>
struct Tile {
  // op(A) is k-major in HBM when A is transposed; op(B) when B is not.
  using OA = Operand<BM, TA, VEC>;
  using OB = Operand<BN, !TB, VEC>;
  static constexpr int WM = BM / GM, WN = BN / GN;  // wave tile
  static constexpr int MI = WM / 16, NI = WN / 16;  // 16 x 16 sub-tiles per wave
  static constexpr int LDS = 2 * (OA::SIZE + OB::SIZE);
  static_assert(GM * GN == 4 && MI >= 1 && NI >= 1, "tile shape");

  // acc += op(A)(i0 : i0+BM, kbeg : kend) op(B)(kbeg : kend, j0 : j0+BN),
  // rows of op(A) beyond M and columns of op(B) beyond N read as zero.
  __device__ static inline void run(f64x4 (&acc)[MI][NI], double* lds, const double* A,
                                    int64_t lda, const double* B, int64_t ldb, int64_t M,
                                    int64_t N, int64_t i0, int64_t j0, int64_t kbeg,
                                    int64_t kend) {
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave / GN, wn = wave % GN;
    const int lr = lane & 15;  // row (mn) of the operand fragment
    const int lk = lane >> 4;  // k of the operand fragment
    if (kbeg >= kend) return;
    double ra[OA::PER_T];
    double rb[OB::PER_T];
    OA::load(ra, A, lda, i0, M, kbeg, kend, tid);
    OB::load(rb, B, ldb, j0, N, kbeg, kend, tid);
    OA::store(lds, ra, tid);
    OB::store(lds + OA::SIZE, rb, tid);
    __syncthreads();
    int buf = 0;
    for (int64_t k0 = kbeg; k0 < kend; k0 += kBK) {
      const bool more = k0 + kBK < kend;
      if (more) {
        OA::load(ra, A, lda, i0, M, k0 + kBK, kend, tid);
        OB::load(rb, B, ldb, j0, N, k0 + kBK, kend, tid);
      }
      const double* la = lds + buf * (OA::SIZE + OB::SIZE);
      const double* lb = la + OA::SIZE;
#pragma unroll
      for (int kk = 0; kk < kBK; kk += 4) {
        double af[MI], bf[NI];
#pragma unroll
        for (int mi = 0; mi < MI; ++mi) af[mi] = OA::frag(la, wm * WM + mi * 16 + lr, kk + lk);
#pragma unroll
        for (int ni = 0; ni < NI; ++ni) bf[ni] = OB::frag(lb, wn * WN + ni * 16 + lr, kk + lk);
#pragma unroll
        for (int mi = 0; mi < MI; ++mi)
#pragma unroll
          for (int ni = 0; ni < NI; ++ni)
            acc[mi][ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[ni], af[mi], acc[mi][ni], 0, 0, 0);
      }
      if (more) {
        double* na = lds + (buf ^ 1) * (OA::SIZE + OB::SIZE);
        OA::store(na, ra, tid);
        OB::store(na + OA::SIZE, rb, tid);
      }
      __syncthreads();
      buf ^= 1;
    }
  }

  // Global row / column of sub-tile (mi, ni), register r, for this lane.
  __device__ static inline int64_t row(int64_t i0, int mi) {
    const int wave = threadIdx.x >> 6;
    return i0 + (wave / GN) * WM + mi * 16 + (threadIdx.x & 15);
  }
  __device__ static inline int64_t col(int64_t j0, int ni, int r) {
    const int wave = threadIdx.x >> 6;
    return j0 + (wave % GN) * WN + ni * 16 + 4 * r + ((threadIdx.x & 63) >> 4);
  }
};

}  // namespace tile
}  // namespace rrf
