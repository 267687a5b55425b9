/*
 * srp.h -- C ABI of the sketch-preconditioned Riemannian CCA / FDA library
 * for one AMD MI355X (gfx950).
 *
 * Method: Shustin & Avron, "Faster Randomized Methods for Orthogonality
 * Constrained Problems".  A sketch S (CountSketch, Section 3; or SRHT,
 * Appendix A) of the tall data gives the preconditioner
 * M = Z^T S^T S Z + lambda I (Section 3), used as the Riemannian metric of
 * the generalized Stiefel manifold (Table 1); Riemannian CG then solves the
 * Brockett-cost forms of regularised CCA (Section 4, Algorithm CCAopt) and
 * FDA (Section 5, Algorithm LDAopt).
 *
 * Conventions for every entry point:
 *  - Matrices are row-major and contiguous; data matrices hold samples in
 *    rows (n x d).
 *  - All array arguments are DEVICE pointers owned by the caller, unless a
 *    comment says "host".  The library never frees or retains caller
 *    memory; it allocates its own workspace from the device's stream-
 *    ordered pool and releases it before returning.
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  Work is
 *    enqueued on it; every entry point returns after that work completed
 *    (it synchronises the stream), so outputs are ready on return.
 *  - Return value: SRP_OK or an SRP_E* status.  No exception crosses the
 *    ABI.  srp_last_error() gives a thread-local message for the last
 *    failure in the calling thread.
 *  - dtype codes name the element type of a data matrix: SRP_F64 (double),
 *    SRP_F32 (float), SRP_BF16 (bfloat16, stored as uint16) and, as a
 *    sketch input only, SRP_FP8E4M3 (uint8 codes with per-column scales).
 */
#ifndef SRP_H
#define SRP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define SRP_OK 0
#define SRP_EINVAL 1      /* invalid argument (sizes, pointers, dtype)      */
#define SRP_ENOTSPD 2     /* Cholesky breakdown: matrix not positive definite */
#define SRP_ENOCONV 3     /* max_iter reached; outputs hold the last iterate */
#define SRP_ENOMEM 4      /* device allocation failed                        */
#define SRP_EDEVICE 5     /* HIP runtime error                                */
#define SRP_EBUSY 6       /* serving engine: no capacity right now            */
#define SRP_EREJECTED 7   /* serving engine: request can never fit            */
#define SRP_PENDING 8     /* serving engine: request not finished yet         */

/* ---- element types ---------------------------------------------------- */
#define SRP_F64 0
#define SRP_F32 1
#define SRP_BF16 2
#define SRP_FP8E4M3 3     /* sketch input only: OCP E4M3 codes (see srp_stage_fp8) */

/* ---- Riemannian optimisation methods ---------------------------------- */
#define SRP_RCG 0         /* Riemannian conjugate gradient (the default)      */
#define SRP_RTR 1         /* Riemannian trust region with truncated CG        */

/* ---- sketch kinds ----------------------------------------------------- */
#define SRP_COUNTSKETCH 0 /* Section 3                                       */
#define SRP_SRHT 1        /* Appendix A, Definition SRHT                      */

/* Solver options.  Fill with srp_default_options() and override fields. */
typedef struct srp_options {
  int sketch;             /* SRP_COUNTSKETCH or SRP_SRHT                      */
  uint64_t seed;          /* seed of the sketch randomness (SplitMix64)       */
  int max_iter;           /* Riemannian CG iteration cap (default 1000)       */
  int warm_start_iters;   /* > 0: start from the exact solution of the
                             sketched problem (exact-cca(SX, SY) /
                             exact-fda(SX), Algorithms CCAopt / LDAopt).
                             CCA: this many block subspace iterations on
                             C^T C (block of min(64, dx, dy) columns,
                             rounded up to a multiple of 4: each product
                             applies (C^T C)^4), then a Rayleigh-Ritz step;
                             one when the block spans min(dx, dy) columns.
                             FDA: one c x c eigensolve, exact.  Default 48.
                             0 = start from qf of a seeded Gaussian point    */
  int refresh_every;      /* recompute the data products B*U from the data
                             every this many iterations (default 25)         */
  int check_every;        /* host reads the convergence flag every this many
                             iterations, one batch behind the queued work
                             (default 2; the result does not depend on it)   */
  int pass_compute;       /* arithmetic of the data passes: SRP_F64 or
                             SRP_F32 (default: F64 for F64 data, F32 else)   */
  int final_f64;          /* > 0 with F32 / BF16 passes: after the iteration
                             converges, run up to this many closing
                             iterations whose data products use FP64
                             arithmetic (two GEMM reads of the data where the
                             fused pass has no FP64 instance); the finishing
                             pass is FP64 too.  < 0: only the finishing pass
                             (the Gram of the final retraction and the
                             Rayleigh-Ritz products) in FP64.  Needs F32 or
                             F64 data.  0 = none (default)                   */
  const double* mu;       /* HOST pointer to k weights mu_1 >= ... >= mu_k > 0
                             (N = diag(mu)); NULL = k, k-1, ..., 1.  Equal
                             weights (N = I) optimise the unweighted trace;
                             the closing Rayleigh-Ritz step still returns
                             ordered vectors                                 */
  int time_passes;        /* 1: time every fused data pass over the full data
                             with HIP events on `stream` (srp_info.pass_ms)   */
  /* Low-precision form: BF16 copies of the data (srp_stage_bf16) read by
     BF16 matrix-core passes with FP32 accumulation until lowp_tol (or
     lowp_max_iter iterations); the iteration then continues on the main
     data to tol (refinement).  NULL = off.  CCA only; needs k <= 16.        */
  const void* lowp_x;     /* device, n x dx BF16 copy of X                    */
  const void* lowp_y;     /* device, n x dy BF16 copy of Y                    */
  double lowp_tol;        /* gradient tolerance of the BF16 phase (1e-3)      */
  int lowp_max_iter;      /* iteration cap of the BF16 phase (200)            */
  /* Staged sketch input: the sketch reads these copies instead of the data
     (CCA X / Y; FDA: ignored).  NULL = sketch the data.                      */
  const void* sketch_x;
  const void* sketch_y;
  int sketch_dtype;       /* SRP_F32, SRP_BF16 or SRP_FP8E4M3                  */
  const double* sketch_scale_x;   /* FP8: device column scales (srp_stage_fp8) */
  const double* sketch_scale_y;
  /* SRP_RCG, or SRP_RTR: the Riemannian trust-region method (Section 2.2
     names it among the Riemannian algorithms the Table 1 components serve)
     with a truncated CG inner solver; its Hessian-vector products are
     Table 1's formula (Eq. HessCCA, Eq. LDAhess), one fused data pass each.
     max_iter then caps the outer iterations.  Needs k <= 16; no BF16 phase. */
  int method;
  int rtr_max_inner;      /* inner (truncated CG) iterations per outer one (50) */
} srp_options;

/* Per-solve report. */
typedef struct srp_info {
  int status;             /* same as the return value                        */
  int iterations;         /* Riemannian CG iterations on the full data       */
  int warm_iterations;    /* subspace iterations of the warm start (FDA: 1);
                             0 when it fell back to the Gaussian start        */
  int passes;             /* data passes over the full n rows                */
  double f;               /* final weighted cost f(Z) = -sum mu_i sigma_i    */
  double objective;       /* sum of the returned sigma (or rho)              */
  double grad_norm;       /* ||grad f||_M at the last iterate                 */
  double ms_sketch;       /* wall ms per phase                               */
  double ms_factor;
  double ms_warm;
  double ms_iterate;
  double ms_total;
  double pass_ms;         /* summed duration of the timed fused passes       */
  int pass_launches;      /* timed passes that did the work: a pass launched
                             in the iterations that follow convergence (the
                             host polls every check_every) returns at once;
                             its few microseconds stay in pass_ms, so
                             pass_ms / pass_launches slightly overstates the
                             duration of a working pass                      */
  int lowp_iterations;    /* iterations of the BF16 phase                    */
  double ms_lowp;         /* wall ms of the BF16 phase (inside ms_iterate)   */
  double lowp_pass_ms;    /* summed duration of its timed BF16 passes         */
  int lowp_pass_launches; /* BF16 passes that did the work (as above)       */
  int lowp_status;        /* how the BF16 phase ended: SRP_OK, SRP_ENOCONV
                             (its cap) or SRP_ENOTSPD (a retraction Gram from
                             BF16 products was not positive definite; the
                             iteration then continued on the main data from
                             the phase's start point)                        */
  int inner_iterations;   /* SRP_RTR: truncated CG iterations in all (one
                             data pass each)                                 */
} srp_info;

/* Fill *opt with the defaults listed above.  Returns SRP_EINVAL if NULL. */
int srp_default_options(srp_options* opt);

/* Thread-local text of the last error in this thread ("" if none). */
const char* srp_last_error(void);

/* sizeof(srp_options), sizeof(srp_info), sizeof(srp_request) and
 * sizeof(srp_result) as compiled into the library, for bindings to check
 * their layouts.  Host only; any pointer may be NULL. */
int srp_abi_sizes(size_t* options_bytes, size_t* info_bytes, size_t* request_bytes, size_t* result_bytes);

/* ---- sketches (Section 3; Appendix A) ---------------------------------
 * out = S A for an s x n sketch S drawn from `seed`, A n x d of `dtype`.
 * out is s x d, double for SRP_F64 input, float otherwise.
 *
 * CountSketch (Section 3): row i of A goes to bucket h(i) with sign g(i),
 *   w = SplitMix64 output i for `seed`; h(i) = ((w >> 32) * s) >> 32,
 *   g(i) = +1 if bit 0 of w is 0 else -1.  Deterministic summation order.
 * SRHT (Definition SRHT): S = sqrt(n'/s) R H D with n' = 2^ceil(log2 n),
 *   A zero-padded to n' rows, H the normalised Walsh-Hadamard matrix,
 *   D_i = +1 if bit 0 of SplitMix64(seed ^ 0x5352485444494147, i) is 0,
 *   R the s rows of smallest key SplitMix64(seed ^ 0x535248545357524F, r),
 *   in ascending row order.  Requires s <= n' <= 2^20.
 * SRP_FP8E4M3 input (codes from srp_stage_fp8): the sketch of the decoded,
 *   unscaled values, FP32; multiplying column j by scales[j] (exact) gives
 *   the sketch of the staged matrix.
 * Errors: SRP_EINVAL for n < 1, d < 1, s < 1, bad dtype or null pointers.
 */
int srp_countsketch(const void* A, int dtype, int64_t n, int d, int s,
                    uint64_t seed, void* out, void* stream);
int srp_srht(const void* A, int dtype, int64_t n, int d, int s,
             uint64_t seed, void* out, void* stream);
/* srp_countsketch for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments and the same output bits as
 * srp_countsketch, with no allocation of any kind.  Its scratch is a
 * library-owned device array of 44 MiB per GPU (held from the first launch
 * on that GPU until the process ends), which limits it to
 * n <= 4194304 rows and s <= 1048576 buckets (SRP_EINVAL beyond, before any
 * device work).  Stream-ordered and asynchronous: it returns once the work
 * is enqueued on `stream` (the output is ready when the stream reaches that
 * point) and does not synchronise.  Every call on one GPU shares that GPU's
 * array: calls on one stream run in order, but calls that overlap on one
 * GPU (other streams, other host threads) race on the scratch and give
 * undefined results.  Errors: as srp_countsketch, plus the limits above. */
int srp_countsketch_noalloc(const void* A, int dtype, int64_t n, int d, int s,
                            uint64_t seed, void* out, void* stream);
/* The s sampled SRHT rows (int64, ascending) for n rows and `seed`. */
int srp_srht_rows(int64_t n, int s, uint64_t seed, int64_t* rows,
                  void* stream);

/* ---- reduced-precision staging of the data ----------------------------
 * The low-precision forms of the sketch and of the data passes read staged
 * copies of X (row-major n x d).
 * srp_stage_bf16: out[i] = X[i] rounded to BF16 (nearest, ties to even),
 *   stored as uint16.
 * srp_stage_fp8: per column j the smallest power of two scales[j] (double,
 *   device) with max_i |X_ij| <= 448 scales[j]; out[i][j] = OCP FP8 E4M3
 *   code of X_ij / scales[j] (nearest, ties to even mantissa, saturating at
 *   +-448; 4 exponent bits, bias 7, 3 mantissa bits).  X is F32 or BF16.
 * Errors: SRP_EINVAL for null pointers, n < 1, d < 1 or a bad dtype.
 */
int srp_stage_bf16(const float* X, int64_t n, int d, uint16_t* out, void* stream);
int srp_stage_fp8(const void* X, int dtype, int64_t n, int d, uint8_t* out, double* scales, void* stream);

/* ---- preconditioner factor (Section 3; cost Table costs) --------------
 * From a sketch SA (s x d, dtype SRP_F64 or SRP_F32) compute in FP64 the
 * upper-triangular R with positive diagonal and R^T R = SA^T SA + lambda I,
 * and its inverse Rinv (both d x d, double, row-major; entries below the
 * diagonal are written as 0).  Rinv may be NULL.
 * Errors: SRP_ENOTSPD if the Gram is not positive definite (lambda = 0 with
 * a rank-deficient sketch), SRP_EINVAL for bad sizes.
 */
int srp_sketch_factor(const void* SA, int dtype, int s, int d, double lambda,
                      double* R, double* Rinv, void* stream);

/* ---- fused tall-skinny data pass (per-iteration products) -------------
 * For data blocks A0 (n x d0) and, if A1 != NULL, A1 (n x d1) of `dtype`,
 * and directions W0 (d0 x k), W1 (d1 x k) (double), compute with arithmetic
 * `compute` (SRP_F64 or SRP_F32):
 *   J0 = A0^T [A0 W0 | A1 W1]   (d0 x 2k, double)
 *   J1 = A1^T [A0 W0 | A1 W1]   (d1 x 2k, double)
 * (with A1 == NULL: J0 = A0^T A0 W0, d0 x k).  These are the products
 * X^T (X U), X^T (Y V), ... that the Riemannian gradient, projection and
 * retraction of Eq. gradCCA / Table 1 consume.  One read of the data.
 * compute = SRP_BF16 (BF16 data only): the products run on BF16 matrix
 *   cores with FP32 accumulation; W is rounded to BF16 and A_b W_b is
 *   rounded to BF16 before the second product.  A view narrower than 113
 *   columns (or rows that are not 4-byte aligned) is outside that
 *   kernel's row chunk: those shapes run the FP32-arithmetic pass on the
 *   same BF16 data (W and A_b W_b unrounded).
 * Limits: k <= 16 with two blocks, k <= 32 with one (k <= 16 for BF16
 * arithmetic); d0 + d1 <= 2048 (F32 / BF16 data) or <= 896 (F64
 * arithmetic).
 * Errors: SRP_EINVAL outside these limits or for a bad dtype / compute
 * pair (F64 data needs F64 arithmetic).
 */
int srp_gram_pass(const void* A0, const void* A1, int dtype, int compute,
                  int64_t n, int d0, int d1, int k, const double* W0,
                  const double* W1, double* J0, double* J1, void* stream);

/* Name of the kernel srp_gram_pass (and the solvers' iterations) run for
 * this shape, when the rows start on 16-byte boundaries (alignment only
 * changes the load width): "k_pass_quad" (FP32, two views of at most 1024
 * columns, 4x4 matrix-core blocks for the narrow products), "k_pass_quad1"
 * (FP32, one view, k <= 20, the same blocks), "k_pass_dma"
 * (FP32, rows streamed into LDS), "k_pass_bf" (BF16 matrix cores) or
 * "k_pass" (register-staged rows).  Static string; NULL outside the limits
 * above.  No device work.
 */
const char* srp_gram_pass_kernel(int dtype, int compute, int d0, int d1, int k);

/* ---- solvers ----------------------------------------------------------
 * cca_solve: top-k (lambda_x, lambda_y)-canonical correlations of X (n x dx)
 * and Y (n x dy) (Definition of regularised CCA, Section 4), by Algorithm
 * CCAopt: sketch X and Y with one S, factor M_xx and M_yy, warm start from
 * the sketched problem, then Riemannian CG on St_Sxx x St_Syy with metric
 * blkdiag(M_xx, M_yy) for the cost of Eq. costriemannianccaBrockett.
 * Outputs (device, double): U (dx x k), V (dy x k) with U^T Sxx U = I,
 * V^T Syy V = I, U^T Sxy V = diag(sigma); sigma (k) descending; column
 * pairs sign-normalised (largest |entry| of each U column positive).
 * tol: stop when ||grad f||_M <= tol * |f|.
 * Requires 1 <= k <= min(dx, dy), k <= 16, lambda >= 0, sketch_size >= 1.
 * A view with sketch_size < its width d (lambda > 0 required for it) keeps
 * its metric in Woodbury form (closing remark after Table costs): the
 * d x d M is neither formed nor factored; K = SA SA^T + lambda I_s is, and
 * M^-1 V = (V - SA^T K^-1 SA V) / lambda, so the metric costs O(s^2 d)
 * instead of O(s d^2); the warm start then iterates on the sketched
 * problem's pencil (no R^-1 to whiten with).
 * Returns SRP_ENOCONV (with the last iterate) at max_iter.
 */
int cca_solve(const void* X, const void* Y, int64_t n, int dx, int dy, int k,
              double lambda_x, double lambda_y, int sketch_size, double tol,
              int dtype, const srp_options* opt, void* stream, double* U,
              double* V, double* sigma, srp_info* info);

/* lda_solve: the k leading regularised FDA directions (Definition of FDA,
 * Section 5) of X (n x d) with int32 labels in [0, n_classes), by
 * Algorithm LDAopt: centre the classes (Xhat, S_B), sketch Xhat, factor M,
 * warm start, Riemannian CG on St_{S_w + lambda I} for Eq. lda_riemannian.
 * Outputs: W (d x k, double) with W^T (S_w + lambda I) W = I and
 * W^T S_B W = diag(rho); rho (k) descending.
 * Requires 2 <= n_classes <= 64, 1 <= k <= min(n_classes - 1, d),
 * k <= 32, every class non-empty, lambda >= 0, sketch_size >= 1
 * (sketch_size < d: the Woodbury form of M^-1 as for cca_solve, which
 * needs lambda > 0).
 */
int lda_solve(const void* X, const int32_t* labels, int64_t n, int d,
              int n_classes, int k, double lambda, int sketch_size,
              double tol, int dtype, const srp_options* opt, void* stream,
              double* W, double* rho, srp_info* info);

/* ---- sparse (CSR) data ----------------------------------------------
 * The paper states its costs in terms of nnz(X) and nnz(Y) (Section 3,
 * Table costs; the cost remarks of Sections 4.5 and 5.5): with the
 * CountSketch the preprocessing is O(nnz) and every data product is
 * O(nnz k).  These entry points take X (and Y) in CSR form.
 *
 * srp_csr: device arrays owned by the caller, unchanged until the call
 * returns.  row_ptr (int64, n_rows + 1, row_ptr[0] = 0, non-decreasing,
 * row_ptr[n_rows] = nnz); col_idx (int32, nnz; in [0, n_cols) and strictly
 * increasing within each row: sorted, no duplicates); values (nnz, dtype
 * SRP_F32 or SRP_F64).  Limits: 1 <= n_rows < 2^31, 1 <= n_cols <= 8192,
 * nnz < 2^31.  Every entry point checks the structure on the device first
 * and returns SRP_EINVAL for a malformed matrix.  All arithmetic on the
 * data is FP64 (the F32 values are widened).  The library builds a
 * column-major copy of each matrix for the products A^T P (nnz index and
 * value words, from its workspace).
 */
typedef struct srp_csr {
  int64_t n_rows;
  int n_cols;
  int dtype;
  int64_t nnz;
  const int64_t* row_ptr;
  const int32_t* col_idx;
  const void* values;
} srp_csr;

/* CountSketch (Section 3) of a CSR matrix: out (s x n_cols, double,
 * row-major) = S A with the h, g of srp_countsketch for `seed`; each
 * bucket's rows are summed in ascending row order, as srp_countsketch sums
 * the dense rows (zero entries add nothing).  O(nnz + n + s n_cols).
 * Errors: SRP_EINVAL for bad sizes or a malformed matrix. */
int srp_countsketch_csr(const srp_csr* A, int s, uint64_t seed, double* out, void* stream);

/* The data pass of srp_gram_pass for CSR blocks, FP64 arithmetic:
 * J0 = A0^T [A0 W0 | A1 W1] (n_cols0 x 2k), J1 = A1^T [A0 W0 | A1 W1]
 * (with A1 == NULL: J0 = A0^T A0 W0, n_cols0 x k).  The sums over a row
 * take its entries in column order, those over a column take its rows in
 * ascending order.  Requires (blocks x k) <= 64 and equal row counts.
 * O(nnz k). */
int srp_gram_pass_csr(const srp_csr* A0, const srp_csr* A1, int k, const double* W0, const double* W1,
                      double* J0, double* J1, void* stream);

/* cca_solve and lda_solve for CSR data (same outputs, conventions and
 * limits otherwise).  The sketch must be SRP_COUNTSKETCH (an SRHT mixes
 * every row, which is not O(nnz)), and the staged-sketch and BF16-phase
 * options are not available (SRP_EINVAL).  lda_solve_csr never forms the
 * centred Xhat: Xhat W = X W - (C W)[labels] row by row (C the class
 * means), Xhat^T (Xhat W) = X^T (Xhat W) since the class sums of Xhat's
 * rows vanish, and S Xhat = S X - (S E) C for the one-hot labels E. */
int cca_solve_csr(const srp_csr* X, const srp_csr* Y, int k, double lambda_x, double lambda_y,
                  int sketch_size, double tol, const srp_options* opt, void* stream, double* U,
                  double* V, double* sigma, srp_info* info);
int lda_solve_csr(const srp_csr* X, const int32_t* labels, int n_classes, int k, double lambda,
                  int sketch_size, double tol, const srp_options* opt, void* stream, double* W,
                  double* rho, srp_info* info);

/* Device workspace, in bytes, that one cca_solve / lda_solve with these
 * sizes allocates (sketches, R^-1 and M^-1, iterate and product buffers,
 * pass partials).  sketch_input_dtype: the dtype the sketch reads (the data
 * dtype, or srp_options.sketch_dtype when sketch_x is set).  Returns 0 for
 * sizes the solver rejects. */
size_t srp_cca_workspace_bytes(int64_t n, int dx, int dy, int k, int sketch_size, int dtype,
                               int sketch_kind, int sketch_input_dtype);
size_t srp_lda_workspace_bytes(int64_t n, int d, int n_classes, int k, int sketch_size, int dtype,
                               int sketch_kind);

/* ---- serving engine ----------------------------------------------------
 * Continuous batching of solves.  Not part of the paper's method: it is the
 * request loop around Algorithms CCAopt / LDAopt for a stream of problems
 * of mixed n, d and k.
 *
 * An engine owns one device-memory pool of hbm_budget_bytes, carved by a
 * first-fit allocator, and max_slots worker slots, each with its own HIP
 * stream (default priority) and host thread.  Submitted requests wait in
 * arrival (FIFO) order.  The head request is admitted as soon as a slot is
 * idle and its footprint (srp_request_footprint) fits in the pool; its
 * sketches, metric factor, iterate and product buffers (and staged copies)
 * then stay resident in that block until the solve ends, and the block
 * returns to the pool.  Admitted solves run concurrently, one per slot, so
 * their kernels overlap on the device; a request that arrives while others
 * run starts as soon as a slot and memory free up.
 *
 * Ownership: X, Y / labels, the outputs and any pointer inside req->opt
 * are caller memory that must stay valid until the request completes
 * (poll / wait returns its status).  Each solve gives the same result as
 * the synchronous call with the same arguments (the second CCA view runs
 * after the first on the slot's stream instead of on a side stream).
 * The engine functions are thread-safe. */
#define SRP_PROBLEM_CCA 0
#define SRP_PROBLEM_LDA 1

#define SRP_STAGE_NONE 0      /* solve on the data as given                   */
#define SRP_STAGE_BF16 1      /* F32 CCA data: the engine writes BF16 copies in
                                 its pool and runs the BF16 phase on them, then
                                 refines on X, Y (srp_options.lowp_*)          */
#define SRP_STAGE_BF16_FP8 2  /* as SRP_STAGE_BF16, and the sketch reads FP8
                                 E4M3 copies with column scales                */

typedef struct srp_request {
  int problem;            /* SRP_PROBLEM_CCA or SRP_PROBLEM_LDA              */
  const void* X;          /* device, n x dx (CCA) / n x d (FDA), `dtype`      */
  const void* Y;          /* CCA: device n x dy, `dtype`; FDA: int32 labels   */
  int64_t n;
  int dx;                 /* FDA: d                                           */
  int dy;                 /* FDA: number of classes                           */
  int k;
  double lambda_x;        /* FDA: lambda                                      */
  double lambda_y;        /* FDA: unused                                      */
  int sketch_size;
  double tol;
  int dtype;              /* SRP_F64, SRP_F32 or SRP_BF16                     */
  int stage;              /* SRP_STAGE_*                                      */
  srp_options opt;        /* by value; lowp_* and sketch_* are set by the
                             engine when stage != SRP_STAGE_NONE              */
  double* U;              /* device outputs as in cca_solve (FDA: W, rho in   */
  double* V;              /* U and sigma; V unused)                           */
  double* sigma;
} srp_request;

typedef struct srp_result {
  int status;             /* the solve's status (SRP_OK, SRP_ENOCONV, ...)    */
  int slot;               /* worker slot that ran it                          */
  double t_submit_ms;     /* engine clock: ms since srp_engine_create          */
  double t_start_ms;      /* admitted (workspace reserved)                    */
  double t_done_ms;       /* outputs complete on the device                   */
  size_t footprint_bytes;
  srp_info info;
  char message[160];      /* the solve's error message, "" on success         */
} srp_result;

typedef struct srp_engine srp_engine;

/* Creates an engine on `device` with a pool of hbm_budget_bytes (allocated
 * once, here) and 1 <= max_slots <= 16 slots. */
int srp_engine_create(int device, size_t hbm_budget_bytes, int max_slots, srp_engine** out);
/* As srp_engine_create, with flags:
 * SRP_ENGINE_GROUPED: grouped ticks.  The Riemannian CG iterations of the
 *   running solves advance together: each solve's data pass runs on its
 *   slot's stream, and each small step of an iteration (the line search's
 *   inner products, controller and update; M^-1 Z, the direction's inner
 *   products, controller and combination) runs for every solve in the tick
 *   as ONE launch (a grid dimension per solve) on the engine's own stream,
 *   between stream-event joins.  A solve's arithmetic is the same as alone
 *   (same kernels per solve, same order), so each result is the same as
 *   from the synchronous call.  Solves that cannot join (Woodbury metric,
 *   trust-region method) run their own launches.
 * Errors: SRP_EINVAL for unknown flags, as srp_engine_create otherwise. */
#define SRP_ENGINE_GROUPED 1
int srp_engine_create2(int device, size_t hbm_budget_bytes, int max_slots, int flags, srp_engine** out);
/* Grouped phases launched so far (0 without SRP_ENGINE_GROUPED). */
int srp_engine_ticks(srp_engine* e, uint64_t* ticks);
/* Bytes of the engine pool a request needs: the solve's workspace plus the
 * staged copies (stage).  0 if the request's sizes are invalid. */
size_t srp_request_footprint(const srp_request* req);
/* Queues a request (never blocks on the GPU).  *ticket identifies it.
 * SRP_EREJECTED: its footprint exceeds the whole pool; SRP_EINVAL: bad
 * sizes or null pointers; SRP_EBUSY: the engine is shutting down. */
int srp_engine_submit(srp_engine* e, const srp_request* req, uint64_t* ticket);
/* SRP_PENDING while the request is queued or running; otherwise fills *out
 * (if not NULL), returns the solve's status and forgets the ticket.
 * SRP_EINVAL for an unknown ticket. */
int srp_engine_poll(srp_engine* e, uint64_t ticket, srp_result* out);
/* Blocks until the request completes; then as srp_engine_poll. */
int srp_engine_wait(srp_engine* e, uint64_t ticket, srp_result* out);
/* Engine counters: requests queued now, running now, the largest number
 * that ran at once, pool bytes in use now and at most.  Any may be NULL. */
int srp_engine_stats(srp_engine* e, int* queued, int* running, int* peak_running, size_t* pool_used,
                     size_t* pool_peak);
/* Finishes every queued and running request, then frees the pool, the
 * streams and the threads.  Results not yet collected are dropped. */
int srp_engine_destroy(srp_engine* e);

#ifdef __cplusplus
}
#endif
#endif /* SRP_H */
