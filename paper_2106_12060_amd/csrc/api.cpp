// C ABI entry points (declared in include/srp.h): argument checks, stream
// handling, workspace, and the synchronous-return convention.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "common.hpp"
#include "kernels.hpp"

using namespace srp;

namespace {
struct Scratch {
  void* p = nullptr;
  hipStream_t st;
  explicit Scratch(hipStream_t s) : st(s) {}
  ~Scratch() {
    if (p) {
      (void)hipFreeAsync(p, st);
      (void)hipStreamSynchronize(st);
    }
  }
};

int finish(hipStream_t st) {
  SRP_HIP(hipStreamSynchronize(st));
  return SRP_OK;
}

CsrView csr_view(const srp_csr& a) {
  CsrView v;
  v.n = a.n_rows;
  v.d = a.n_cols;
  v.nnz = a.nnz;
  v.ptr = a.row_ptr;
  v.idx = a.col_idx;
  v.val = a.values;
  v.dtype = a.dtype;
  return v;
}
}  // namespace

extern "C" {

int srp_default_options(srp_options* o) {
  if (!o) return SRP_EINVAL;
  memset(o, 0, sizeof(*o));
  o->sketch = SRP_COUNTSKETCH;
  o->seed = 12060;
  o->max_iter = 1000;
  o->warm_start_iters = 48;
  o->method = SRP_RCG;
  o->rtr_max_inner = 50;
  o->refresh_every = 25;
  o->check_every = 2;
  o->pass_compute = -1;
  o->final_f64 = 0;
  o->mu = nullptr;
  o->lowp_tol = 1e-3;
  o->lowp_max_iter = 200;
  o->sketch_dtype = SRP_F32;
  return SRP_OK;
}

const char* srp_last_error(void) { return srp::last_error(); }

size_t srp_cca_workspace_bytes(int64_t n, int dx, int dy, int k, int sketch_size, int dtype, int sketch_kind,
                               int sketch_input_dtype) {
  if (n < 1 || dx < 1 || dy < 1 || k < 1 || k > std::min(dx, dy) || sketch_size < 1) return 0;
  if (dtype < SRP_F64 || dtype > SRP_BF16 || sketch_input_dtype < SRP_F64 || sketch_input_dtype > SRP_FP8E4M3)
    return 0;
  if (sketch_kind != SRP_COUNTSKETCH && sketch_kind != SRP_SRHT) return 0;
  return cca_ws_bytes(n, dx, dy, k, sketch_size, dtype, sketch_kind, sketch_input_dtype);
}

size_t srp_lda_workspace_bytes(int64_t n, int d, int n_classes, int k, int sketch_size, int dtype, int sketch_kind) {
  if (n < 2 || d < 1 || n_classes < 2 || k < 1 || k > std::min(n_classes - 1, d) || sketch_size < 1) return 0;
  if (dtype < SRP_F64 || dtype > SRP_BF16) return 0;
  if (sketch_kind != SRP_COUNTSKETCH && sketch_kind != SRP_SRHT) return 0;
  return lda_ws_bytes(n, d, n_classes, k, sketch_size, dtype, sketch_kind);
}

int srp_abi_sizes(size_t* options_bytes, size_t* info_bytes, size_t* request_bytes, size_t* result_bytes) {
  if (options_bytes) *options_bytes = sizeof(srp_options);
  if (info_bytes) *info_bytes = sizeof(srp_info);
  if (request_bytes) *request_bytes = sizeof(srp_request);
  if (result_bytes) *result_bytes = sizeof(srp_result);
  return SRP_OK;
}

int srp_countsketch(const void* A, int dtype, int64_t n, int d, int s, uint64_t seed, void* out, void* stream) {
  clear_error();
  SRP_REQUIRE(A && out, "null pointer argument");
  SRP_REQUIRE(n >= 1 && n < (int64_t(1) << 31) && d >= 1 && s >= 1, "bad sizes");
  SRP_REQUIRE(dtype == SRP_F64 || dtype == SRP_F32 || dtype == SRP_BF16 || dtype == SRP_FP8E4M3, "bad dtype %d",
              dtype);
  hipStream_t st = (hipStream_t)stream;
  Scratch ws(st);
  const size_t bytes = countsketch_ws_bytes(n, s) + 1024;
  SRP_TRY(device_alloc(&ws.p, bytes, st));
  Arena ar{(char*)ws.p, bytes, 0};
  SRP_TRY(countsketch_run(A, dtype, n, d, s, seed, out, ar, st));
  return finish(st);
}

int srp_srht(const void* A, int dtype, int64_t n, int d, int s, uint64_t seed, void* out, void* stream) {
  clear_error();
  SRP_REQUIRE(A && out, "null pointer argument");
  SRP_REQUIRE(n >= 1 && d >= 1 && s >= 1, "bad sizes");
  SRP_REQUIRE(dtype == SRP_F64 || dtype == SRP_F32 || dtype == SRP_BF16 || dtype == SRP_FP8E4M3, "bad dtype %d",
              dtype);
  int64_t np = 2;
  while (np < n) np <<= 1;
  SRP_REQUIRE(np <= (int64_t(1) << 20) && s <= np, "SRHT needs s <= n' <= 2^20");
  hipStream_t st = (hipStream_t)stream;
  Scratch ws(st);
  const size_t bytes = srht_ws_bytes(n, d, s, dtype) + 1024;
  SRP_TRY(device_alloc(&ws.p, bytes, st));
  Arena ar{(char*)ws.p, bytes, 0};
  SRP_TRY(srht_run(A, dtype, n, d, s, seed, out, ar, st));
  return finish(st);
}

int srp_stage_bf16(const float* X, int64_t n, int d, uint16_t* out, void* stream) {
  clear_error();
  SRP_REQUIRE(X && out, "null pointer argument");
  SRP_REQUIRE(n >= 1 && d >= 1, "bad sizes");
  hipStream_t st = (hipStream_t)stream;
  SRP_TRY(stage_bf16_run(X, n, d, out, st));
  return finish(st);
}

int srp_stage_fp8(const void* X, int dtype, int64_t n, int d, uint8_t* out, double* scales, void* stream) {
  clear_error();
  SRP_REQUIRE(X && out && scales, "null pointer argument");
  SRP_REQUIRE(n >= 1 && d >= 1, "bad sizes");
  SRP_REQUIRE(dtype == SRP_F32 || dtype == SRP_BF16, "stage_fp8: data must be F32 or BF16");
  hipStream_t st = (hipStream_t)stream;
  Scratch ws(st);
  const size_t bytes = stage_fp8_ws_bytes(d) + 1024;
  SRP_TRY(device_alloc(&ws.p, bytes, st));
  Arena ar{(char*)ws.p, bytes, 0};
  SRP_TRY(stage_fp8_run(X, dtype, n, d, out, scales, ar, st));
  return finish(st);
}

int srp_srht_rows(int64_t n, int s, uint64_t seed, int64_t* rows, void* stream) {
  clear_error();
  SRP_REQUIRE(rows, "null pointer argument");
  SRP_REQUIRE(n >= 1 && s >= 1, "bad sizes");
  int64_t np = 2;
  while (np < n) np <<= 1;
  SRP_REQUIRE(np <= (int64_t(1) << 20) && s <= np, "SRHT needs s <= n' <= 2^20");
  hipStream_t st = (hipStream_t)stream;
  Scratch ws(st);
  const size_t bytes = srht_ws_bytes(n, 1, s, SRP_F32) + 1024;
  SRP_TRY(device_alloc(&ws.p, bytes, st));
  Arena ar{(char*)ws.p, bytes, 0};
  SRP_TRY(srht_rows_run(n, s, seed, rows, ar, st));
  return finish(st);
}

int srp_sketch_factor(const void* SA, int dtype, int s, int d, double lambda, double* R, double* Rinv,
                      void* stream) {
  clear_error();
  SRP_REQUIRE(SA && R, "null pointer argument");
  SRP_REQUIRE(s >= 1 && d >= 1, "bad sizes");
  SRP_REQUIRE(dtype == SRP_F64 || dtype == SRP_F32, "sketch dtype must be SRP_F64 or SRP_F32");
  SRP_REQUIRE(lambda >= 0.0, "lambda must be >= 0");
  hipStream_t st = (hipStream_t)stream;
  Scratch ws(st);
  const size_t bytes = factor_ws_bytes(s, d) + bytes_of<int>(4) + bytes_of<double>((size_t)d * d) + 2048;
  SRP_TRY(device_alloc(&ws.p, bytes, st));
  Arena ar{(char*)ws.p, bytes, 0};
  int* flag = ar.take<int>(4);
  double* X = Rinv ? Rinv : ar.take<double>((size_t)d * d);
  SRP_TRY(fill_i32(flag, 1, 0, st));
  SRP_TRY(sketch_factor_run(SA, dtype, s, d, lambda, R, X, nullptr, flag, ar, st, nullptr,
                            factor_aux_stream(0)));
  int h = 0;
  SRP_HIP(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  SRP_TRY(finish(st));
  if (h) {
    set_error("sketched Gram is not positive definite");
    return SRP_ENOTSPD;
  }
  return SRP_OK;
}

int srp_gram_pass(const void* A0, const void* A1, int dtype, int compute, int64_t n, int d0, int d1, int k,
                  const double* W0, const double* W1, double* J0, double* J1, void* stream) {
  clear_error();
  SRP_REQUIRE(A0 && W0 && J0, "null pointer argument");
  SRP_REQUIRE(!A1 || (W1 && J1 && d1 >= 1), "second block needs W1, J1 and d1 >= 1");
  SRP_REQUIRE(n >= 1 && d0 >= 1 && k >= 1, "bad sizes");
  SRP_REQUIRE(compute == SRP_F64 || compute == SRP_F32 || compute == SRP_BF16,
              "compute must be SRP_F64, SRP_F32 or SRP_BF16");
  if (!A1) d1 = 0;
  SRP_REQUIRE(pass_limits_ok(dtype, compute, d0, d1, k, A1 ? 2 : 1), "unsupported shape for the data pass");
  hipStream_t st = (hipStream_t)stream;
  Scratch ws(st);
  const size_t bytes = pass_ws_bytes(n, d0, d1, k, compute) + 2048;
  SRP_TRY(device_alloc(&ws.p, bytes, st));
  Arena ar{(char*)ws.p, bytes, 0};
  SRP_TRY(gram_pass_run(A0, A1, dtype, compute, n, d0, d1, k, W0, W1, J0, J1, nullptr, ar, st));
  return finish(st);
}

int srp_countsketch_csr(const srp_csr* A, int s, uint64_t seed, double* out, void* stream) {
  clear_error();
  SRP_REQUIRE(A && out, "null pointer argument");
  SRP_REQUIRE(s >= 1, "bad sizes");
  hipStream_t st = (hipStream_t)stream;
  const CsrView v = csr_view(*A);
  Scratch ws(st);
  const size_t bytes = countsketch_csr_ws_bytes(std::max<int64_t>(v.n, 1), s) + bytes_of<int>(4) + 1024;
  SRP_TRY(device_alloc(&ws.p, bytes, st));
  Arena ar{(char*)ws.p, bytes, 0};
  int* bad = ar.take<int>(4);
  SRP_TRY(csr_check(v, "A", bad, st));
  SRP_TRY(countsketch_csr_run(v, s, seed, out, nullptr, 0, nullptr, ar, st));
  return finish(st);
}

int srp_gram_pass_csr(const srp_csr* A0, const srp_csr* A1, int k, const double* W0, const double* W1, double* J0,
                      double* J1, void* stream) {
  clear_error();
  SRP_REQUIRE(A0 && W0 && J0, "null pointer argument");
  SRP_REQUIRE(!A1 || (W1 && J1), "second block needs W1 and J1");
  const int nb = A1 ? 2 : 1;
  SRP_REQUIRE(k >= 1 && nb * k <= 64, "need 1 <= k and (blocks x k) <= 64");
  hipStream_t st = (hipStream_t)stream;
  CsrView v[2] = {csr_view(*A0), A1 ? csr_view(*A1) : CsrView{}};
  SRP_REQUIRE(!A1 || v[1].n == v[0].n, "A0 and A1 must have the same number of rows");
  const int ldp = nb * k;
  Scratch ws(st);
  size_t bytes = bytes_of<int>(4) + bytes_of<double>((size_t)std::max<int64_t>(v[0].n, 1) * ldp) + 2048;
  size_t scr = 0;
  for (int b = 0; b < nb; ++b) {
    SRP_REQUIRE(v[b].n >= 1 && v[b].d >= 1, "bad sizes");
    bytes += csc_bytes(v[b]) + csc_partial_bytes(v[b], ldp);
    scr = std::max(scr, csc_scratch_bytes(v[b]));
  }
  bytes += scr;
  SRP_TRY(device_alloc(&ws.p, bytes, st));
  Arena ar{(char*)ws.p, bytes, 0};
  int* bad = ar.take<int>(4);
  SRP_TRY(csr_check(v[0], "A0", bad, st));
  if (A1) SRP_TRY(csr_check(v[1], "A1", bad, st));
  double* P = ar.take<double>((size_t)v[0].n * ldp);
  CscView c[2];
  char* sbase = ar.base + ar.used;
  ar.used += (scr + 255) & ~size_t(255);
  double* part[2] = {nullptr, nullptr};
  for (int b = 0; b < nb; ++b) {
    Arena t{sbase, scr, 0};
    SRP_TRY(csc_build(v[b], &c[b], ar, t, st));
    part[b] = (double*)ar.take<char>(csc_partial_bytes(v[b], ldp));
    if (!part[b]) { set_error("workspace layout overflow"); return SRP_ENOMEM; }
  }
  const double* Wb[2] = {W0, W1};
  double* Jb[2] = {J0, J1};
  for (int b = 0; b < nb; ++b)
    SRP_TRY(csr_times_dense(v[b], Wb[b], k, k, P + b * k, ldp, nullptr, nullptr, nullptr, st));
  for (int b = 0; b < nb; ++b) SRP_TRY(csc_times_dense(c[b], P, ldp, ldp, Jb[b], ldp, part[b], nullptr, st));
  return finish(st);
}

const char* srp_gram_pass_kernel(int dtype, int compute, int d0, int d1, int k) {
  return gram_pass_kernel_name(dtype, compute, d0, d1, k);
}

int cca_solve(const void* X, const void* Y, int64_t n, int dx, int dy, int k, double lambda_x, double lambda_y,
              int sketch_size, double tol, int dtype, const srp_options* opt, void* stream, double* U, double* V,
              double* sigma, srp_info* info) {
  return cca_solve_impl(X, Y, n, dx, dy, k, lambda_x, lambda_y, sketch_size, tol, dtype, opt, (hipStream_t)stream,
                        U, V, sigma, info);
}

int lda_solve(const void* X, const int32_t* labels, int64_t n, int d, int n_classes, int k, double lambda,
              int sketch_size, double tol, int dtype, const srp_options* opt, void* stream, double* W, double* rho,
              srp_info* info) {
  return lda_solve_impl(X, labels, n, d, n_classes, k, lambda, sketch_size, tol, dtype, opt, (hipStream_t)stream, W,
                        rho, info);
}

int cca_solve_csr(const srp_csr* X, const srp_csr* Y, int k, double lambda_x, double lambda_y, int sketch_size,
                  double tol, const srp_options* opt, void* stream, double* U, double* V, double* sigma,
                  srp_info* info) {
  clear_error();
  SRP_REQUIRE(X && Y, "null pointer argument");
  return cca_solve_csr_impl(csr_view(*X), csr_view(*Y), k, lambda_x, lambda_y, sketch_size, tol, opt,
                            (hipStream_t)stream, U, V, sigma, info);
}

int lda_solve_csr(const srp_csr* X, const int32_t* labels, int n_classes, int k, double lambda, int sketch_size,
                  double tol, const srp_options* opt, void* stream, double* W, double* rho, srp_info* info) {
  clear_error();
  SRP_REQUIRE(X, "null pointer argument");
  return lda_solve_csr_impl(csr_view(*X), labels, n_classes, k, lambda, sketch_size, tol, opt, (hipStream_t)stream, W,
                            rho, info);
}

}  // extern "C"
