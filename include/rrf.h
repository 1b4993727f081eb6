/*
 * rrf.h -- randomized rank-revealing UTV factorizations on AMD MI355X (gfx950).
 *
 * Heavner, Chen, Gopal, Martinsson, "Efficient algorithms for computing
 * rank-revealing factorizations on a GPU" (arXiv 2106.13402).
 *
 * Given A (m x n, m >= n), every factorization here returns
 *     A = U * T * V^T,
 * U (m x m) and V (n x n) orthogonal, T (m x n) upper trapezoidal
 * (Sec. 1, the UTV problem statement). rrf_randutv, rrf_randutv_boosted and
 * rrf_powerurv also take m < n, through the transpose (T lower trapezoidal).
 *
 * Conventions shared by every entry point:
 *  - All matrices are column-major IEEE binary64 in DEVICE memory of the
 *    current HIP device, allocated and owned by the caller. The library keeps
 *    no pointer to them after the call returns and frees nothing it did not
 *    allocate.
 *  - Leading dimensions: A has lda >= m; U, T and V are tight: ldu = m,
 *    ldt = m, ldv = n. T may alias A only when lda == m (factor in place).
 *  - U or V may be NULL: that factor is then not accumulated (Sec. 4.1
 *    forms U and V only "when the U and V matrices are desired").
 *  - Return value: RRF_OK (0) on success; -k when argument k (1-based) is
 *    invalid (LAPACK info convention), checked before any device work; a
 *    positive RRF_E_* code otherwise. rrf_last_error() describes the last
 *    failure of the calling thread.
 *  - The sketch matrices are drawn from a counter-based generator:
 *    Philox4x64-10 keyed by (seed, stream) with counter (row/4, col, 0, 0),
 *    turned into N(0,1) numbers by Box-Muller; entry (r, c) of a stream is a
 *    function of (seed, stream, r, c) only. randUTV step i (1-based) uses
 *    stream i; powerURV uses stream 0.
 *  - Unless rrf_opts.async is set, a call returns after the device work is
 *    complete and its status covers device-side failures.
 */
#ifndef RRF_H_
#define RRF_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define RRF_OK          0
#define RRF_E_HIP       1  /* a HIP runtime call or a kernel failed            */
#define RRF_E_NOMEM     2  /* workspace too small or device allocation failed  */
#define RRF_E_NOTSUP    3  /* valid request outside what is implemented        */
#define RRF_E_NUMERIC   4  /* non-finite input (only with check_finite)         */
#define RRF_E_INTERNAL  5  /* a device-side consistency check failed           */
/* Fault injection for tests of callers' error paths, read at every call:
 * RRF_TEST_FAIL=hip in the environment fails every entry point's device
 * check (RRF_E_HIP); RRF_TEST_FAIL=alloc fails the device allocation of the
 * library-managed workspace (RRF_E_NOMEM), leaving no workspace cached. */

/* ---- precision modes -------------------------------------------------- */
#define RRF_PREC_FP64   0  /* every step in binary64                           */
/* The products that only have to capture a dominant singular subspace are
 * formed from bfloat16 values (round to nearest even) with binary32
 * accumulation; everything else stays binary64 (the paper itself is binary64
 * throughout).
 *  randUTV (Alg. 3): the sketch Y = (T22^T T22)^q T22^T G of each step, from
 *    bfloat16 copies of T22 (scaled by a power of two) and G, each
 *    intermediate column rescaled by a power of two before rounding; the QR
 *    of Y and every update of T, U and V in binary64.
 *  powerURV (Alg. 1): the 2q power products A V and A^T V_hat, from a
 *    bfloat16 copy of A (scaled by a power of two) and V, V_hat rounded as
 *    they are; the QRs, the Q factors and the final A V in binary64 (q = 0
 *    has no power products and is binary64). These products are rounded
 *    relative to ||A||, so directions below about 1e-3 of the largest
 *    singular value are not separated (e_k there exceeds the binary64
 *    value). */
#define RRF_PREC_BF16_SKETCH 1
/* randUTV only: the bfloat16 sketch of RRF_PREC_BF16_SKETCH, and every
 * update of T, U and V by a product of Householder transforms (the right
 * update of Alg. 3 with V_i, the left update with U_i, the accumulation of U
 * and V) formed by the split-bfloat16 three-pass product of rrf_gemm_x3
 * (error per term at most about 2^-15 |a| |b|). T keeps binary64 storage and is
 * scaled by the power of two of max|A| for the run (exact, undone at the
 * end). The panels, the b x b SVDs and the small products among the
 * compact-WY factors stay binary64. ||A - U T V^T|| / ||A|| and the
 * orthogonality of U and V are then about 1e-5, not binary64 level; e_k is
 * resolved down to about 1e-5 of each step's trailing norm. */
#define RRF_PREC_BF16_X3 2
/* randUTV only: as RRF_PREC_BF16_X3 with the updates formed by the six-term
 * product of rrf_gemm_x6 (each operand split into three bfloat16 parts of
 * its binary32 rounding; per K slice of 32 the terms are summed in binary32,
 * the slices in binary64), about 1e-8 relative per product. The
 * accumulation of U and V from Householder transforms amplifies that: at
 * n = 16384 ||A - U T V^T|| / ||A|| comes to about 1.4e-6 and the
 * orthogonality of U and V to about 3e-5 (20x and 1.5x closer than the x3
 * mode); e_k is resolved down to about 1e-6 of each step's trailing norm. */
#define RRF_PREC_BF16_X6 3

/* ---- algorithms (for rrf_workspace_size) -------------------------------- */
#define RRF_ALG_RANDUTV  0
#define RRF_ALG_POWERURV 1

typedef struct rrf_opts {
  int precision;          /* RRF_PREC_*                                        */
  void* stream;           /* hipStream_t to order the work on; NULL = null stream */
  void* workspace;        /* device scratch; NULL = library-managed cache      */
  size_t workspace_bytes; /* size of `workspace` (>= rrf_workspace_size(...))  */
  int async;              /* 0: return after completion; 1: only enqueue       */
  int check_finite;       /* 1: reject A with NaN/Inf (RRF_E_NUMERIC) before any
                             work is enqueued; synchronizes the stream        */
  int thin_u;             /* randUTV: 1 forms only U(:, 1:n) (m x n, ld m), all
                             that A = U T V^T needs since T(n:m, :) = 0      */
  int no_replay;          /* rrf_randutv_batched: 1 issues the lockstep rounds
                             directly; 0 (default) records the call's launches
                             as HIP graphs and replays them on later calls
                             with the same shapes                            */
} rrf_opts;

/* Fill `opts` with the defaults (FP64, null stream, library workspace,
 * synchronous, no finiteness check, full m x m U, batched calls replayed). */
void rrf_opts_init(rrf_opts* opts);

/*
 * randUTV_basic -- Alg. 3 (Appendix B), the blocked randomized UTV of Sec. 4.1.
 *
 * Loop over s = ceil(n/b) steps; step i sketches the trailing block T22 with
 * Y = (T22^T T22)^q T22^T G_i, takes V_i from an unpivoted Householder QR of
 * Y, updates T <- T V_i, takes U_i and R from the Householder QR of the new
 * panel T(I2 u I3, J2), updates T <- U_i^T T, and diagonalizes the b x b block
 * R by an SVD. The last step takes the SVD of the remaining block (as a
 * Householder QR followed by an SVD of its square R factor when it is tall).
 *
 *  m, n   : rows and columns of A, 1 <= n <= m            (args 1, 2)
 *  A      : input, read only unless T == A                 (arg 3)
 *  lda    : leading dimension of A, lda >= m               (arg 4)
 *  b      : block size, b >= 1                             (arg 5)
 *  q      : number of power iterations, q >= 0             (arg 6)
 *  seed   : generator key                                  (arg 7)
 *  U      : m x m output (m x n with opts->thin_u) or NULL  (arg 8)
 *  T      : m x n output, upper trapezoidal; every b x b diagonal block is
 *           diagonal with non-negative entries in descending order (arg 9)
 *  V      : n x n output or NULL                           (arg 10)
 * m < n (Sec. 3.2): A^T is factored instead, A^T = U' T' V'^T, and the
 * result is returned as U = V' (m x m), T = T'^T (m x n, lower trapezoidal,
 * diagonal b x b blocks) and V = U' (n x n); opts->thin_u does not apply.
 * rrf_workspace_size then covers the transpose's factorization plus A^T and
 * T^T (2 m n doubles).
 */
int rrf_randutv(int64_t m, int64_t n, const double* A, int64_t lda, int64_t b,
                int32_t q, uint64_t seed, double* U, double* T, double* V);
int rrf_randutv_ex(int64_t m, int64_t n, const double* A, int64_t lda, int64_t b,
                   int32_t q, uint64_t seed, double* U, double* T, double* V,
                   const rrf_opts* opts);

/*
 * rrf_randutv_noalloc -- rrf_randutv_ex for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, and
 * harnesses that forbid hipMalloc. Same arguments, results and error codes
 * as rrf_randutv_ex (bitwise the same results), except:
 *  - opts->workspace must be NULL and opts->workspace_bytes 0 (else -11):
 *    the workspace is a static device array of RRF_NOALLOC_SCRATCH_BYTES
 *    (64 MiB) inside the library, one per device, held until the process
 *    ends. A request whose rrf_workspace_size() exceeds it returns
 *    RRF_E_NOMEM before any device work (square FP64 inputs at q = 1 fit up
 *    to n = 1807 at b = 16, 1611 at b = 32, 1280 at b = 64, 812 at b = 128).
 *  - The call itself performs no hipMalloc/hipFree and calls no allocating
 *    library routine. The first call on a device looks up the array's
 *    device address and creates the library's side streams there.
 *  - Every call on one device shares that device's array, which keeps the
 *    previous call's contents (the kernels clear what must start at zero):
 *    calls that overlap on one device (other host threads, or opts->async
 *    with work still in flight on another stream) race and must be ordered
 *    by the caller.
 */
#define RRF_NOALLOC_SCRATCH_BYTES (64ull << 20)
int rrf_randutv_noalloc(int64_t m, int64_t n, const double* A, int64_t lda, int64_t b,
                        int32_t q, uint64_t seed, double* U, double* T, double* V,
                        const rrf_opts* opts);

/*
 * The randomized SVD (RSVD) -- Sec. 3.3 (its relation to powerURV).
 *
 * Y = (A A^T)^q A G with G the n x l Gaussian of stream 0 (the first l columns
 * of powerURV's G for the same seed), Q from a Householder QR of Y, the thin
 * SVD Q^T A = W diag(S) V^T, U = Q W: A ~ U diag(S) V^T with the error of the
 * rank-l projection Q Q^T A. Any m, n (no transposition needed). FP64.
 *
 *  m, n   : rows and columns of A                           (args 1, 2)
 *  A, lda : input, lda >= m                                 (args 3, 4)
 *  l      : rank, 1 <= l <= min(m, n), l <= 256             (arg 5)
 *  q      : power steps, q >= 0                             (arg 6)
 *  seed   : generator key                                   (arg 7)
 *  U      : m x l output (ld m) or NULL                     (arg 8)
 *  S      : l singular values, descending, non-negative     (arg 9)
 *  V      : n x l output (ld n) or NULL                     (arg 10)
 *  opts   : stream, workspace (rrf_rsvd_workspace_size bytes), async,
 *           check_finite; precision must be RRF_PREC_FP64
 * All pointers are device memory; l > 256 returns RRF_E_NOTSUP.
 */
int rrf_rsvd(int64_t m, int64_t n, const double* A, int64_t lda, int64_t l, int32_t q,
             uint64_t seed, double* U, double* S, double* V, const rrf_opts* opts);
size_t rrf_rsvd_workspace_size(int64_t m, int64_t n, int64_t l, int32_t q);

/*
 * randUTV halted early -- Sec. 4.1 (error of the rank-k approximation).
 *
 * Runs the steps of rrf_randutv_ex and, before each step (c0 = i b columns
 * reduced), stops when c0 >= kmax or when e = ||T(c0:m, c0:n)||_F, which is
 * ||A - A_k||_F of the rank-c0 approximation, is <= tol ||A||_F. e is formed
 * directly from the trailing block (one pass over it; the paper's update
 * e_i^2 = e_{i-1}^2 - ||T(I2, J2 u J3)||_F^2 loses its relative accuracy
 * once e_i falls below sqrt(eps) ||A||_F). On return *k_out = k, the
 * columns reduced; A = U T V^T holds with T = [T11 T12; 0 T22], T11 (k x k)
 * upper triangular with diagonal, non-negative, descending b x b blocks,
 * and T22 = T(k:m, k:n) the unreduced remainder (U, V the product of the
 * steps taken). tol = 0 and kmax >= n give rrf_randutv_ex's result.
 * m < n goes through the transpose as for rrf_randutv: k counts the
 * transpose's reduced columns (k <= m), T = [T11 0; T21 T22] with T11
 * lower triangular, and the workspace is rrf_workspace_size's for m < n.
 *
 *  m, n, A, lda, b, q, seed : as for rrf_randutv            (args 1-7)
 *  tol    : relative Frobenius tolerance, tol >= 0         (arg 8)
 *  kmax   : cap on the columns reduced, kmax >= 0          (arg 9)
 *  U, T, V: as for rrf_randutv                             (args 10-12)
 *  k_out  : host int64 receiving k                         (arg 13)
 *  opts   : as for rrf_randutv_ex (any precision mode); the call always
 *           synchronizes (the stopping test reads each step's norm)
 */
int rrf_randutv_partial(int64_t m, int64_t n, const double* A, int64_t lda, int64_t b,
                        int32_t q, uint64_t seed, double tol, int64_t kmax, double* U, double* T,
                        double* V, int64_t* k_out, const rrf_opts* opts);

/*
 * Resume an early-stopped randUTV: continue the steps of
 * rrf_randutv_partial from its state (T with T(k_in:, k_in:) unreduced, and
 * the U, V it returned) with a new tol / kmax. The steps use the same
 * generator streams, so the result is that of one rrf_randutv_partial call
 * with the new criteria (to rounding: U and V are continued by applying the
 * new steps' Householder transforms to them). ||A||_F is taken as ||T||_F.
 *
 *  m, n   : as for rrf_randutv                             (args 1, 2)
 *  b, q, seed : the values of the interrupted call         (args 3-5)
 *  tol, kmax  : the new stopping criteria                  (args 6, 7)
 *  k_in   : columns already reduced (the k it returned), a multiple of b
 *           in [0, min(m, n)] or min(m, n) itself           (arg 8)
 *  U, T, V: in/out, U m x m (or NULL), T m x n, V n x n (or NULL), the
 *           arrays the interrupted call filled             (args 9-11)
 *  k_out  : host int64 receiving the new k                 (arg 12)
 *  opts   : as for rrf_randutv_partial; thin_u is rejected (RRF_E_NOTSUP)
 * m < n: the state is that of a wide rrf_randutv_partial (T lower
 * trapezoidal); T is transposed into the workspace, the transpose's steps
 * continue (V carrying its U, U its V) and the result is transposed back.
 */
int rrf_randutv_resume(int64_t m, int64_t n, int64_t b, int32_t q, uint64_t seed, double tol,
                       int64_t kmax, int64_t k_in, double* U, double* T, double* V,
                       int64_t* k_out, const rrf_opts* opts);

/*
 * randUTV_boosted -- Alg. 2 (Sec. 4.2-4.3): randUTV with oversampling.
 *
 * Each step samples the trailing block with b + p_i columns,
 * p_i = min(p, N_i - b) (N_i = n - i b), and takes V_i from an unpivoted
 * Householder QR of the leading b left singular vectors W_Y(:, 1:b) of the
 * sample matrix Y (QR of Y, SVD of its R factor). The first step draws all
 * b + p_1 Gaussian columns (stream 1) through q power steps; each later step
 * draws b (stream i), applies q - 1 power steps and one more product to
 * them (q = 0: the Gaussian itself), projects them off W_l, orthonormalises
 * them and samples Y = T22^T [Q, W_l], where W_l is the orthonormalised
 * image T22 W_next of the previous step's extra vectors
 * W_next = V_i(:, b+1:N_i)^T W_Y(:, b+1:b+p_i) (the paper's listing applies
 * W_next on the left of T22, which only types for square blocks; this
 * library maps it through T22 first). The rest of each step, the last step
 * and the output form are those of rrf_randutv. FP64 only.
 *
 *  m, n, A, lda, b, q : as for rrf_randutv                 (args 1-6)
 *  p      : oversampling, p >= 0, with b + p <= 256        (arg 7)
 *  seed, U, T, V      : as for rrf_randutv                 (args 8-11)
 * opts: precision must be RRF_PREC_FP64; the workspace must hold
 * rrf_randutv_boosted_workspace_size(m, n, b, q, p) bytes. b + p > 256
 * returns RRF_E_NOTSUP. m < n goes through the transpose as for rrf_randutv
 * (p is then clipped against m - b, and the workspace size covers A^T and
 * T^T).
 */
int rrf_randutv_boosted(int64_t m, int64_t n, const double* A, int64_t lda, int64_t b,
                        int32_t q, int64_t p, uint64_t seed, double* U, double* T, double* V);
int rrf_randutv_boosted_ex(int64_t m, int64_t n, const double* A, int64_t lda, int64_t b,
                           int32_t q, int64_t p, uint64_t seed, double* U, double* T,
                           double* V, const rrf_opts* opts);
size_t rrf_randutv_boosted_workspace_size(int64_t m, int64_t n, int64_t b, int32_t q,
                                          int64_t p);

/*
 * powerURV -- Alg. 1 (Sec. 3.2).
 *
 * V starts as an n x n Gaussian; q rounds of  Y_hat = A V,
 * V_hat = HQR_thin(Y_hat), Y = A^T V_hat, V = HQR_thin(Y); then
 * A_hat = A V and [U, R] = HQR_full(A_hat), T = R. With q = 0 the method is
 * RURV (Sec. 3.1) and V is the orthogonal factor of the Householder QR of the
 * Gaussian. T(k,k) carries the sign of the Householder R diagonal.
 *
 * Arguments as for rrf_randutv, except that b is the panel width of the
 * blocked Householder QR (it changes rounding only; b > min(m, n) acts as
 * min(m, n)).
 * m < n goes through the transpose as for rrf_randutv: A^T = U' T' V'^T is
 * factored and U = V' (m x m), T = T'^T (lower trapezoidal), V = U'
 * (n x n); rrf_workspace_size covers A^T and T^T as well.
 */
int rrf_powerurv(int64_t m, int64_t n, const double* A, int64_t lda, int64_t b,
                 int32_t q, uint64_t seed, double* U, double* T, double* V);
int rrf_powerurv_ex(int64_t m, int64_t n, const double* A, int64_t lda, int64_t b,
                    int32_t q, uint64_t seed, double* U, double* T, double* V,
                    const rrf_opts* opts);

/* Bytes of device workspace an _ex call with these arguments needs
 * (alg = RRF_ALG_*); 0 for invalid arguments. */
size_t rrf_workspace_size(int alg, int64_t m, int64_t n, int64_t b, int32_t q,
                          int precision);

/*
 * Batched randUTV -- Alg. 3 on `count` independent matrices in one call, for
 * workloads of many small matrices (one kernel launch serves the same stage of
 * every matrix). Matrix j is factored as rrf_randutv_ex would factor it with
 * the sketch key seed + j (same arithmetic, same generator streams; results
 * agree to rounding, as the products are summed in another order).
 *
 *  count  : number of matrices, >= 0 (0: nothing to do)              (arg 1)
 *  m, n   : host arrays of count sizes, 1 <= m[j], n[j] <= 4096      (args 2, 3)
 *  A      : host array of count device pointers, read only unless T[j] == A[j]
 *                                                                     (arg 4)
 *  lda    : host array, lda[j] >= m[j]                                (arg 5)
 *  b      : block size for every matrix, 1 <= b <= 64; 0 = the configuration
 *           rrf_batched_config(m[j], n[j], precision) gives (tuned table
 *           or built-in rule)                                         (arg 6)
 *  q      : power iterations, >= 0                                    (arg 7)
 *  seed   : generator key of matrix 0                                 (arg 8)
 *  U      : host array of count device pointers to m[j] x m[j] outputs
 *           (ld m[j]), or NULL for no U                               (arg 9)
 *  T      : host array of device pointers to m[j] x n[j] outputs (ld m[j]);
 *           T[j] may be A[j] when lda[j] == m[j]                      (arg 10)
 *  V      : as U with n[j] x n[j] outputs (ld n[j]), or NULL          (arg 11)
 *  opts   : as for rrf_randutv_ex (RRF_PREC_FP64, or RRF_PREC_BF16_SKETCH for
 *           the bfloat16 sketch of every step); the workspace must hold
 *           rrf_randutv_batched_workspace_size(count, m, n, b, precision) bytes
 * The output of every matrix has the form rrf_randutv documents, a wide one
 * (m[j] < n[j]) included: it is factored through its transpose, in a
 * lockstep group of its own, from a copy of A[j]^T held in the workspace
 * (T lower trapezoidal). The host arrays are read during the call only.
 *
 * Execution. The first call with a given set of shapes (count, m[], n[], b,
 * q, precision) builds the descriptors of every stage of every step for every
 * matrix into one device buffer, records the launches as HIP graphs (one per
 * slice of about equal work, up to four, replayed on the library's own
 * streams ordered after and before `stream`) and replays them. A later call
 * with the same shapes only replays the graphs; if pointers, leading
 * dimensions, the seed or the workspace differ, the descriptors are rebuilt
 * on the host and uploaded into the same buffer first. Up to eight recordings
 * are kept per device (least recently used evicted; freed by
 * rrf_release_workspace). With opts->no_replay, or while tracing, the stages
 * are issued directly from host-built descriptors streamed through a pinned
 * ring per slice. Either way the call may wait on the host for earlier work
 * of its own enqueueing while it runs, and consecutive calls on different
 * streams are ordered by the library where they share its buffers.
 */
int rrf_randutv_batched(int64_t count, const int64_t* m, const int64_t* n,
                        const double* const* A, const int64_t* lda, int64_t b,
                        int32_t q, uint64_t seed, double* const* U, double* const* T,
                        double* const* V, const rrf_opts* opts);
/* The block size of the built-in rule for an m x n matrix (16 for
 * min(m, n) <= 256, else 32), which b = 0 follows where no tuning table
 * applies (rrf_batched_config gives the configuration actually used); 0 for
 * invalid sizes. */
int64_t rrf_randutv_batched_block(int64_t m, int64_t n);
/* Bytes of device workspace for rrf_randutv_batched (the largest group's,
 * plus 8 m[j] n[j] bytes for each wide matrix's transposed copy); 0 for
 * invalid sizes or precision. */
size_t rrf_randutv_batched_workspace_size(int64_t count, const int64_t* m,
                                          const int64_t* n, int64_t b, int precision);

/*
 * Autotuner of the batched call (tuned per bucket of sizes; the paper has no
 * batched form -- the buckets follow the many-small-matrices workload).
 *
 * A configuration is the block size b, the tile shapes the grouped GEMM may
 * use (bit mask of RRF_TILE_*; 64 x 64 is always allowed) and the panel leaf
 * width (a panel wider than `leaf` columns is factored by the column split of
 * the compact-WY merge; 0: as wide as one workgroup holds).
 */
#define RRF_TILE_64x64   (1 << 0)
#define RRF_TILE_128x64  (1 << 1)
#define RRF_TILE_128x32  (1 << 2)
#define RRF_TILE_128x16  (1 << 3)
#define RRF_TILE_128x128 (1 << 4)
typedef struct rrf_batched_cfg {
  int64_t b;
  int tile_mask;
  int leaf;
  int tuned;  /* 1: taken from a tuning table; 0: the built-in rule */
} rrf_batched_cfg;

/* Choose a configuration per bucket of n (1-64, 65-128, ..., 449-512 in
 * steps of 64, 513-768, 769-1024; buckets above nmax are not tuned) among the
 * candidates b in {16, 32, 64} x {every tile shape, no 128 x 128, only the
 * narrow 128 x 32 / 128 x 16 / 64 x 64} x leaf {0, 16}, by timing replayed
 * calls with HIP events (q power iterations, U and V formed, Gaussian
 * matrices from `seed`):
 *  - m and n given (host arrays of `count` <= 256 sizes, each in [1, 4096];
 *    more matrices return RRF_E_NOTSUP): on that workload. Every bucket holding some min(m[j], n[j]) starts at the
 *    built-in rule; bucket by bucket each candidate is installed and the whole
 *    batched call timed (median of three replays after the recording call);
 *    the fastest is kept. Meanwhile the trial tables are the process's
 *    tables (batched calls of other threads follow them).
 *  - m and n NULL: on a synthetic batch per bucket, `count` matrices with n
 *    uniform in the bucket and m in [n, 2n].
 * The result forms the table of (the current device's architecture,
 * precision), which replaces any loaded one and is written with all loaded
 * tables to `path` (NULL: not written). Allocates its own device buffers;
 * runs on opts->stream.
 *  precision : RRF_PREC_FP64 or RRF_PREC_BF16_SKETCH             (arg 1)
 *  q >= 0 (arg 2), count >= 1 (arg 3), m, n (args 4, 5),
 *  1 <= nmax <= 1024 (arg 6), seed (arg 7)
 * Returns -8 when `path` cannot be written. */
int rrf_batched_autotune(int precision, int32_t q, int64_t count, const int64_t* m,
                         const int64_t* n, int64_t nmax, uint64_t seed, const char* path,
                         const rrf_opts* opts);
/* Replace the loaded tuning tables by those of the cache file `path` (NULL:
 * unload them, so b = 0 follows the built-in rule). -1 when the file cannot
 * be read or is not a valid cache (the format the autotuner writes; every
 * integer field a whole number in range, every bucket 1 <= nmin <= nmax with
 * 1 <= b <= 64, tile_mask within the tile set and 0 <= leaf <= 64): a
 * rejected file leaves the loaded tables as they were. Without any call the library loads
 * $RRF_TUNE_CACHE (empty: none), else tuning/batched.json beside librrf.so,
 * on its first lookup. */
int rrf_batched_tune_load(const char* path);
/* The configuration rrf_randutv_batched uses with b = 0 for an m x n matrix
 * (the transpose's when m < n) in `precision`: from the loaded table of the
 * current device's architecture when one has a bucket holding min(m, n),
 * else the built-in rule (b = rrf_randutv_batched_block(m, n), every tile,
 * leaf 0). Lookups are deterministic: the same table gives the same choice. */
int rrf_batched_config(int64_t m, int64_t n, int precision, rrf_batched_cfg* out);

/* Release the library-managed workspace cache of the current device and the
 * batched call's staging rings and recordings on every device. */
int rrf_release_workspace(void);

/* ---- building blocks, exported for component tests ------------------------
 * Each runs on `stream` (hipStream_t, NULL = null stream) and returns after
 * the work is enqueued; device memory and ownership as above. */

/* As rrf_dgemm, with each element x of A and B split as x32 = x rounded to
 * binary32, hi = x32 rounded to bfloat16, lo = (x32 - hi) rounded to
 * bfloat16 (all to nearest even), and op(A) op(B) formed as the three-pass
 * sum hi_a hi_b + hi_a lo_b + lo_a hi_b on the bfloat16 matrix cores with
 * binary32 accumulation, widened to binary64 for alpha, beta and C. This is
 * the product of the RRF_PREC_BF16_X3 updates (a mixed-precision extension;
 * the paper computes in binary64). Errors and arguments as rrf_dgemm. */
int rrf_gemm_x3(int transa, int transb, int64_t M, int64_t N, int64_t K, double alpha,
                const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                double* C, int64_t ldc, void* work, size_t work_bytes, void* stream);

/* As rrf_gemm_x3 with the six-term product of the RRF_PREC_BF16_X6 updates:
 * x32 = x rounded to binary32, hi = x32 rounded to bfloat16, mid = (x32 - hi)
 * and lo = (x32 - hi - mid) rounded to bfloat16 (nearest even; the
 * subtractions are exact), op(A) op(B) formed as hi hi + hi mid + mid hi +
 * hi lo + lo hi + mid mid on the bfloat16 matrix cores, binary32 sums per K
 * slice of 32 added in binary64. Errors and arguments as rrf_dgemm. */
int rrf_gemm_x6(int transa, int transb, int64_t M, int64_t N, int64_t K, double alpha,
                const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                double* C, int64_t ldc, void* work, size_t work_bytes, void* stream);

/* The sketch generator: out(r, c) = N(0,1) entry (r, c) of (seed, stream),
 * 0 <= r < rows, 0 <= c < cols, column-major with leading dimension ld. */
int rrf_gaussian(uint64_t seed, uint64_t stream_id, int64_t rows, int64_t cols,
                 double* out, int64_t ld, void* stream);

/* The uniforms the generator above turns into Gaussians, for checking it bit
 * for bit: out(4g + i, c) = uniform i of counter (g, c, 0, 0) under key
 * (seed, stream_id), i = 0..3 in the order u_a, v_a, u_b, v_b
 * (u = ((w >> 11) + 1) 2^-53 from words 0 and 2, v = (w >> 11) 2^-53 from
 * words 1 and 3), 0 <= 4g + i < rows. Device buffer, column-major, ld >= rows.
 * Errors as rrf_gaussian. */
int rrf_sketch_uniforms(uint64_t seed, uint64_t stream_id, int64_t rows, int64_t cols,
                        double* out, int64_t ld, void* stream);

/* C = alpha * op(A) * op(B) + beta * C in binary64 (op = transpose when the
 * trans flag is 1). op(A) is M x K, op(B) is K x N. With beta == 0, C is not
 * read. `work`/`work_bytes` provide scratch for split-K partial sums (may be
 * NULL/0: no split). */
int rrf_dgemm(int transa, int transb, int64_t M, int64_t N, int64_t K, double alpha,
              const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
              double* C, int64_t ldc, void* work, size_t work_bytes, void* stream);

/* Householder QR of the M x k panel P (M >= k, 1 <= k <= 256), Sec. 2.3:
 * reflectors H_i = I - tau_i v_i v_i^T with the LAPACK dlarfg sign rule,
 * Q = H_1 ... H_k = I - W Tf W^T (compact WY). Outputs: W (M x k, explicit
 * unit lower trapezoidal, ld ldw; may alias P when ldw == ldp), R (k x k upper
 * triangular, ld ldr; may be NULL), Tf (k x k upper triangular, ld ldt), tau
 * (k). `work` must hold rrf_panel_workspace_size(M, k) bytes (enough for
 * either kernel below).
 * Kernels: panels of 16 <= k <= 128 and M >= 1024 with W not overlapping P
 * take CholeskyQR2 (two passes of Gram matrix, Cholesky factor and its
 * inverse) and recover the reflectors from Q by an LU of Q(0:k, :) - S,
 * each sign chosen at its pivot; if a Cholesky pivot fails (the panel is
 * ill conditioned or rank deficient, or not finite) the column-exchange
 * kernel factors the panel instead, on the device. Other panels, and all
 * panels with RRF_PANEL_COLUMN=1 in the environment, use the
 * column-exchange kernel (one grid-wide exchange per column); with
 * RRF_PANEL_TREE=1, panels of k <= 64 and M <= 65536 (wider ones split into
 * such halves) go through a tree of QRs over 256-row blocks with the
 * reflectors recovered from its Q. All give the dlarfg reflectors to
 * rounding on full-rank panels, except that the recovered reflectors are
 * tau = 2, v = e_j (and row j of R negated) where dlarfg gives H = I for an
 * exactly zero sub-column, and after an exact rank drop the tree's later
 * reflectors are another exact choice. Environment variables are read at
 * each call. */
size_t rrf_panel_workspace_size(int64_t M, int64_t k);
int rrf_householder_panel(int64_t M, int64_t k, double* P, int64_t ldp, double* W,
                          int64_t ldw, double* R, int64_t ldr, double* Tf, int64_t ldt,
                          double* tau, void* work, size_t work_bytes, void* stream);

/* SVD of a k x k matrix B (1 <= k <= 256): B = Us diag(d) Vs^T with d in
 * descending order and each pair (u_j, v_j) signed so that the entry of v_j
 * of largest magnitude is positive (lowest index on ties). Us, Vs k x k with
 * ld k. `work` must hold rrf_block_svd_workspace_size(k) bytes. */
size_t rrf_block_svd_workspace_size(int64_t k);
int rrf_block_svd(int64_t k, const double* B, int64_t ldb, double* Us, double* d,
                  double* Vs, void* work, size_t work_bytes, void* stream);

/* Building blocks of the RRF_PREC_BF16_SKETCH sketch.
 *
 * rrf_to_bf16: out (rows x cols, ld ldo, ldo a multiple of 8 >= rows) =
 * bfloat16 bit patterns of X s rounded to nearest even directly from binary64;
 * s = 1 when `scaled` is 0, else the power of two putting max|X| in
 * [0.5, 1). Rows [rows, ldo) of out are written as 0. When outT is not NULL
 * it receives the transpose (cols x rows, ld ldot, a multiple of 8 >= cols,
 * rows [cols, ldot) zero). `work` must hold 256 bytes. Device pointers. */
int rrf_to_bf16(int64_t rows, int64_t cols, const double* X, int64_t ldx, int scaled,
                uint16_t* out, int64_t ldo, uint16_t* outT, int64_t ldot, void* work,
                size_t work_bytes, void* stream);

/* rrf_gemm_bf16_tn: the M x N product A^T B of bfloat16 matrices A (K x M,
 * ld lda) and B (K x N, ld ldb), both leading dimensions multiples of 8 and
 * both base addresses 16-byte aligned, with rows [K, ld) of A and B zero, on
 * the bfloat16 matrix cores with binary32 accumulation. The result goes
 * either to out16 (bfloat16, ld ld16 >= M a multiple of 8, rows [M, ld16)
 * zero), each column scaled by the power of two that puts its max|.| in
 * [0.5, 1) before rounding to nearest even, or, when out16 is NULL, to out64
 * (binary64, ld ld64 >= M), widened exactly. `work` must hold
 * rrf_gemm_bf16_workspace_size(M, N) bytes. */
size_t rrf_gemm_bf16_workspace_size(int64_t M, int64_t N);
int rrf_gemm_bf16_tn(int64_t M, int64_t N, int64_t K, const uint16_t* A, int64_t lda,
                     const uint16_t* B, int64_t ldb, uint16_t* out16, int64_t ld16,
                     double* out64, int64_t ld64, void* work, size_t work_bytes, void* stream);

/* ---- diagnostics ------------------------------------------------------- */
const char* rrf_status_string(int status);
const char* rrf_last_error(void);

/* Per-kernel timing. When enabled, the library records a pair of HIP events
 * around every kernel launch, on the launch's own stream, and the launch's
 * algorithmic flop and byte counts (GEMM: 2 M N K flops; panel: the panel
 * read and the reflectors written; generator: the matrix written).
 * rrf_trace_enable(on) clears the totals and switches recording on or off.
 * rrf_trace_read() waits for the recorded events and fills up to
 * max_entries totals, one per kernel class that ran; returns how many.
 * Kernels that form U and V after the randUTV loop run concurrently on two
 * streams of their own; they are reported as separate classes whose names
 * end in ":UV". */
typedef struct rrf_trace_entry {
  char name[48];     /* kernel class, e.g. "dgemm_mfma_128x128_NT"          */
  int64_t launches;  /* launches recorded                                  */
  double ms;         /* summed event-measured duration, milliseconds       */
  double flops;      /* summed algorithmic floating-point operations       */
  double bytes;      /* summed algorithmic HBM bytes (read + written)      */
} rrf_trace_entry;
int rrf_trace_enable(int on);
/* Like rrf_trace_enable(1), but records events around the launches of one
 * kernel class only (a name rrf_trace_read reports, ":UV" suffix included),
 * so that timing one class leaves the other launches uninstrumented.
 * Returns -1 for NULL or an unknown name. rrf_trace_enable ends the filter. */
int rrf_trace_enable_class(const char* name);
int rrf_trace_read(rrf_trace_entry* out, int max_entries);

#ifdef __cplusplus
}
#endif

#endif /* RRF_H_ */
