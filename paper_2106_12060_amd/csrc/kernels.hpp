// Internal launch interface between the host driver and the HIP kernels.
#pragma once
#include "common.hpp"

namespace srp {

int fill_i32(int* p, int64_t count, int v, hipStream_t st);
int fill_f64(double* p, int64_t count, double v, hipStream_t st);
int copy_f64(double* dst, const double* src, int64_t count, hipStream_t st);

// ---------------------------------------------------------- sketches
size_t countsketch_ws_bytes(int64_t n, int s);
int countsketch_run(const void* A, int dtype, int64_t n, int d, int s, uint64_t seed, void* out,
                    Arena& ws, hipStream_t st);
// Rows grouped by bucket (offsets[b] .. offsets[b+1] into sorted, rows
// ascending inside a bucket), from ws.
int countsketch_buckets(int64_t n, int s, uint64_t seed, Arena& ws, const int** offsets, const int** sorted,
                        hipStream_t st);
// offsets[0..count] = exclusive scan of in[0..count) (offsets[count] = total).
int scan_excl_i32(const int* in, int count, int* offsets, hipStream_t st);
size_t srht_ws_bytes(int64_t n, int d, int s, int dtype);
int srht_run(const void* A, int dtype, int64_t n, int d, int s, uint64_t seed, void* out, Arena& ws,
             hipStream_t st);
int srht_rows_run(int64_t n, int s, uint64_t seed, int64_t* rows, Arena& ws, hipStream_t st);
// The sampled rows of an SRHT and their grouping by low bits depend only on
// (n, s, seed): a plan computes them once (its arrays from `keep`, the
// selection's temporaries from `scratch`) and serves every matrix sketched
// with that S (both CCA views).
struct SrhtPlan {
  int64_t n = 0;
  int s = 0;
  uint64_t seed = 0;
  int64_t* rows = nullptr;
  int *goff = nullptr, *galpha = nullptr, *gslot = nullptr;
  uint32_t* dbits = nullptr;   // signs of D, one bit per row (1 = negated)
};
size_t srht_plan_bytes(int64_t n, int s);
int srht_plan_run(int64_t n, int s, uint64_t seed, SrhtPlan* plan, Arena& keep, Arena& scratch, hipStream_t st);
int srht_apply_run(const SrhtPlan& plan, const void* A, int dtype, int d, void* out, Arena& ws, hipStream_t st);

// ---------------------------------------------------- FP64 dense blocks
// C = alpha * op(A) op(B) + beta * C on row-major double matrices (A may be
// float).  op(A) is m x kk (A is m x kk, or kk x m when ta), op(B) is kk x n.
// upper_only skips 64x64 output tiles strictly below the block diagonal.
// ksplit > 1 splits kk into chunks written to C + z * c_split_stride (beta
// must be 0 then).
struct GemmArgs {
  int m, n, kk;
  double alpha, beta;
  const void* A; int64_t lda; bool ta; bool a_f32;
  const void* B; int64_t ldb; bool tb; bool b_f32;
  double* C; int64_t ldc;
  bool upper_only = false;
  int ksplit = 1;
  int64_t c_split_stride = 0;
};
int gemm_f64(const GemmArgs& g, hipStream_t st);
// C (m x nc) = op(A) (m x kk) B (kk x nc) for nc <= 64 (row-major, FP64
// arithmetic; op(A) = A^T when ta, A then kk x m; A FP64, or FP32 when
// a_f32).  ws holds the split-K partials (skinny_ws_bytes with the default
// slices).
size_t skinny_ws_bytes(int m, int kk, int nc);
struct SkinnyProb {
  int m, kk, nc;
  const void* A; int64_t lda; bool ta;
  const double* B; int64_t ldb;
  double* C; int64_t ldc;
  bool a_f32 = false;
};
// Up to four problems in one launch (all with the same ta and A type); ws
// holds the partials of each, in order.  slice: contraction length per
// partial (0: the default); when one slice covers every problem's
// contraction the products are written to C directly and ws may be null.
int gemm_skinny_batch(int nprob, const SkinnyProb* probs, double* ws, size_t ws_bytes, hipStream_t st,
                      int slice = 0);
int gemm_skinny_f64(int m, int kk, int nc, const double* A, int64_t lda, bool ta, const double* B, int64_t ldb,
                    double* C, int64_t ldc, double* ws, size_t ws_bytes, hipStream_t st);
// out[i] = sum_z parts[z * stride + i] (+ diag_add on the diagonal of a
// d x d matrix when d > 0), for count elements.
int sum_parts_f64(const double* parts, int nparts, int64_t stride, int64_t count, double* out,
                  int d, double diag_add, hipStream_t st);

// Gram of a sketch, Cholesky and inverse: R^T R = SA^T SA + lambda I.
// Hfull (optional, d x d): the full symmetric Gram SA^T SA, without lambda.
size_t factor_ws_bytes(int s, int d);
// aux (optional, not st): a second stream on which the column blocks of
// R^-1 run alongside the Cholesky (joined before return).
int sketch_factor_run(const void* SA, int dtype, int s, int d, double lambda, double* R, double* Rinv,
                      double* Minv, int* flag_dev, Arena& ws, hipStream_t st, double* Hfull = nullptr,
                      hipStream_t aux = nullptr);
// Per-device second streams for sketch_factor_run's aux (i = 0, 1; null on
// failure).
hipStream_t factor_aux_stream(int i);
// Split of an s-long Gram contraction over d0 x d1 outputs (about 256
// workgroups of 128 x 128 tiles).
int gram_split(int s, int d0, int d1);
// AT (cols x rows) = A^T for row-major A (rows x cols).
int transpose_f64(const double* A, int rows, int cols, double* AT, hipStream_t st);
// The same from an SRP_F64 or SRP_F32 matrix (FP32 entries widened).
int transpose_to_f64(const void* A, int dtype, int rows, int cols, double* AT, hipStream_t st);

// --------------------------------------------------------- data pass
// J_b = A_b^T [A_0 W_0 | A_1 W_1] (see srp_gram_pass).  Arithmetic in
// `compute` (SRP_F64 / SRP_F32).  With `ran`, a pass that runs (done not
// set) adds one to *ran on the device.
size_t pass_ws_bytes(int64_t n, int d0, int d1, int k, int compute);
const char* gram_pass_kernel_name(int dtype, int compute, int d0, int d1, int k);
int gram_pass_run(const void* A0, const void* A1, int dtype, int compute, int64_t n, int d0, int d1,
                  int k, const double* W0, const double* W1, double* J0, double* J1, const int* done,
                  Arena& ws, hipStream_t st, hipEvent_t before_pass = nullptr,
                  hipEvent_t after_pass = nullptr, int* ran = nullptr);
// FDA centring (Section 5.1): class counts and FP64 sums, Yhat rows
// sqrt(n_k)(m_k - m), and the materialised Xhat = X - m_{y_i} in the data
// type.  Returns SRP_EINVAL (via *bad) for labels out of range.
// Largest number of FDA classes: the centring kernels keep one LDS
// histogram bin and one 256-column accumulator row per class.
constexpr int kLdaMaxClasses = 64;
size_t lda_center_ws_bytes(int64_t n, int d, int c);
int lda_center_run(const void* X, const int32_t* labels, int dtype, int64_t n, int d, int c, void* Xhat,
                   double* Yhat, int* counts, int* bad, Arena& ws, hipStream_t st);
int pass_limits_ok(int dtype, int compute, int d0, int d1, int k, int nblocks);

// --------------------------------------------------------- sparse data
// CSR matrix in device memory (row pointers int64, n + 1 of them; column
// indices int32, strictly increasing within a row; values F32 or F64).
struct CsrView {
  int64_t n = 0;
  int d = 0;
  int64_t nnz = 0;
  const int64_t* ptr = nullptr;
  const int32_t* idx = nullptr;
  const void* val = nullptr;
  int dtype = SRP_F32;
};
// Its column-major copy: column j's rows (ascending) at ptr[j] .. ptr[j+1].
struct CscView {
  int d = 0;
  int64_t nnz = 0;
  int* ptr = nullptr;
  int32_t* idx = nullptr;
  void* val = nullptr;
  int dtype = SRP_F32;
  // the columns cut into segments of a fixed number of entries: segments
  // segptr[j] .. segptr[j+1] belong to column j, segcol[q] is q's column
  int nseg = 0;
  int* segptr = nullptr;
  int* segcol = nullptr;
};
// Widest CSR input: the CountSketch keeps one bucket's row of d doubles in
// LDS.
constexpr int kCsrMaxCols = 8192;
// Sets *bad (device) to 1 if A is not a well-formed CSR matrix.
int csr_validate(const CsrView& A, int* bad, hipStream_t st);
// Size and pointer checks, then csr_validate (bad: one device int);
// synchronises st; SRP_EINVAL naming `name` on failure.
int csr_check(const CsrView& A, const char* name, int* bad, hipStream_t st);
size_t csc_bytes(const CsrView& A);
size_t csc_scratch_bytes(const CsrView& A);
int csc_build(const CsrView& A, CscView* out, Arena& keep, Arena& scratch, hipStream_t st);
// out (rows x w, leading dimension ldo) = A D for D with leading dimension
// ldd, w <= 64; CSR form optionally minus sub[labels[r]] per row r.
// A set *done makes the launch a no-op.
int csr_times_dense(const CsrView& A, const double* D, int ldd, int w, double* out, int ldo, const double* sub,
                    const int32_t* labels, const int* done, hipStream_t st);
// The columns' products go through per-segment partials (partial:
// csc_partial_bytes(A, w) bytes), summed per column in segment order.
int64_t csc_max_segments(const CsrView& A);
size_t csc_partial_bytes(const CsrView& A, int w);
int csc_times_dense(const CscView& A, const double* D, int ldd, int w, double* out, int ldo, double* partial,
                    const int* done, hipStream_t st);
size_t countsketch_csr_ws_bytes(int64_t n, int s);
// out (s x d, FP64) = S A; with labels, se (s x c) = S E for the one-hot
// class matrix E (labels must be in range).
int countsketch_csr_run(const CsrView& A, int s, uint64_t seed, double* out, const int32_t* labels, int c,
                        double* se, Arena& ws, hipStream_t st);
int label_counts_run(int64_t n, int c, const int32_t* labels, int* counts, int* bad, hipStream_t st);
// sums (c x d) = class sums of A's rows, means (c x d) = class means and
// Yhat (c x d) rows sqrt(n_q)(m_q - m).
int fda_csr_stats_run(const CscView& A, int64_t n, int c, const int32_t* labels, const int* counts, double* sums,
                      double* means, double* Yhat, hipStream_t st);

// --------------------------------------------------------- staging
int stage_bf16_run(const float* X, int64_t n, int d, uint16_t* out, hipStream_t st);
size_t stage_fp8_ws_bytes(int d);
int stage_fp8_run(const void* X, int dtype, int64_t n, int d, uint8_t* out, double* scales, Arena& ws,
                  hipStream_t st);
// A (rows x d, FP32) column j times scales[j] (powers of two: exact).
int scale_cols_run(float* A, int64_t rows, int d, const double* scales, hipStream_t st);

// --------------------------------------------------------- solves
// Execution context of one solve.  side: stream for the second CCA view
// (null = both views in order on the main stream); ws / ws_bytes: a
// workspace the solve carves its buffers from (null = allocate from the
// stream-ordered pool and release on return).
struct TickGroup;
struct SolveCtx {
  hipStream_t side = nullptr;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  // the serving engine's grouped ticks (k <= 16 and k <= 32 solves): the
  // iteration's small kernels of every solve in a group run as one launch
  TickGroup* group[2] = {nullptr, nullptr};
};
// Groups of solves whose per-iteration small kernels run as grouped
// launches (driver.hip).  kc: 16 or 32 (the kernels' k bound).
TickGroup* tick_group_create(int kc, int* status);
void tick_group_destroy(TickGroup* g);
// Grouped ticks so far (the number of grouped phases launched).
uint64_t tick_group_ticks(const TickGroup* g);
size_t cca_ws_bytes(int64_t n, int dx, int dy, int k, int s, int dtype, int sketch_kind, int skin_dtype);
size_t lda_ws_bytes(int64_t n, int d, int c, int k, int s, int dtype, int sketch_kind);
size_t cca_csr_ws_bytes(const CsrView& X, const CsrView& Y, int k, int s);
size_t lda_csr_ws_bytes(const CsrView& X, int c, int k, int s);
int cca_solve_csr_impl(const CsrView& X, const CsrView& Y, int k, double lx, double ly, int s, double tol,
                       const srp_options* opt, hipStream_t st, double* U, double* V, double* sigma, srp_info* info,
                       const SolveCtx* ctx = nullptr);
int lda_solve_csr_impl(const CsrView& X, const int32_t* labels, int c, int k, double lam, int s, double tol,
                       const srp_options* opt, hipStream_t st, double* W, double* rho, srp_info* info,
                       const SolveCtx* ctx = nullptr);
int cca_solve_impl(const void* X, const void* Y, int64_t n, int dx, int dy, int k, double lx, double ly, int s,
                   double tol, int dtype, const srp_options* opt, hipStream_t st, double* U, double* V,
                   double* sigma, srp_info* info, const SolveCtx* ctx = nullptr);
int lda_solve_impl(const void* X, const int32_t* labels, int64_t n, int d, int c, int k, double lam, int s,
                   double tol, int dtype, const srp_options* opt, hipStream_t st, double* W, double* rho,
                   srp_info* info, const SolveCtx* ctx = nullptr);
const char* last_error();

}  // namespace srp
