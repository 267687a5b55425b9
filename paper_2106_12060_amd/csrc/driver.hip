// Host driver: Algorithm CCAopt and Algorithm LDAopt on one HIP stream.
//
//   sketch (CountSketch / SRHT, one S for X and Y)
//   -> M_b = (S A_b)^T (S A_b) + lam_b I, R_b, M_b^-1 = R_b^-1 R_b^-T (FP64)
//   -> warm start: the exact solution of the sketched problem (exact-cca /
//      exact-fda of the sketch): block subspace iteration with Rayleigh-Ritz
//      (CCA), one small eigensolve (FDA)
//   -> qf_B of the warm start, then Riemannian CG on the full data with the
//      metric M (one fused data pass per iteration)
//   -> FP64 retraction, Rayleigh-Ritz rotation of the k x k block, sign
//      convention.
// All iteration state stays on the device; the host only enqueues kernels
// and polls a convergence flag every `check_every` iterations.
#include "common.hpp"
#include "kernels.hpp"
#include "solver.hpp"
#include "rtr.hpp"

#include <algorithm>
#include <chrono>
#include <utility>
#include <vector>
#include <cstdarg>
#include <cstring>
#include <atomic>
#include <map>
#include <mutex>
#include <condition_variable>

namespace srp {

// ------------------------------------------------------------ errors
static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}
void clear_error() { g_err[0] = 0; }
const char* last_error() { return g_err; }

int num_cus() {
  static std::atomic<int> cached{0};
  int c = cached.load(std::memory_order_relaxed);
  if (c) return c;
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
    c = v;
  else
    c = 256;
  cached.store(c, std::memory_order_relaxed);
  return c;
}

int allow_dynamic_lds(const void* fn, size_t bytes) {
  static std::mutex mu;
  static std::map<std::pair<int, const void*>, size_t> limits;
  int dev = 0;
  SRP_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  size_t& cur = limits[{dev, fn}];
  if (bytes > cur) {
    SRP_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    cur = bytes;
  }
  return SRP_OK;
}

int device_alloc(void** p, size_t bytes, hipStream_t s) {
  static std::mutex mu;
  static bool tuned[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < 64) {
    std::lock_guard<std::mutex> lock(mu);
    hipMemPool_t pool;
    if (!tuned[dev] && hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
      uint64_t thr = UINT64_MAX;
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
    tuned[dev] = true;
  }
  hipError_t e = hipMallocAsync(p, bytes, s);
  if (e != hipSuccess) {
    set_error("device allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? SRP_ENOMEM : SRP_EDEVICE;
  }
  return SRP_OK;
}

int device_free(void* p, hipStream_t s) {
  if (p) SRP_HIP(hipFreeAsync(p, s));
  return SRP_OK;
}

// Owns one stream-ordered workspace allocation.
struct Workspace {
  void* base = nullptr;
  hipStream_t st = nullptr;
  ~Workspace() {
    if (base) (void)hipFreeAsync(base, st);
  }
};

// ------------------------------------------------------------ timers
struct PhaseTimer {
  hipStream_t st;
  std::chrono::steady_clock::time_point t0;
  explicit PhaseTimer(hipStream_t s) : st(s) { t0 = std::chrono::steady_clock::now(); }
  double lap_ms() {
    (void)hipStreamSynchronize(st);
    auto t1 = std::chrono::steady_clock::now();
    double ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    t0 = t1;
    return ms;
  }
};

// A second stream per device (default priority) for work that is
// independent of the caller's stream: CCA sketches and factors the Y view on
// it while the X view runs on the caller's stream.
static hipStream_t side_stream() {
  static std::mutex mu;
  static hipStream_t streams[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  if (!streams[dev] && hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking) != hipSuccess)
    streams[dev] = nullptr;
  return streams[dev];
}

// Two more streams per device (default priority) for the column blocks of
// R^-1 that run alongside each view's Cholesky (sketch_factor_run).
hipStream_t factor_aux_stream(int i) {
  static std::mutex mu;
  static hipStream_t streams[64][2] = {};
  int dev = 0;
  if (i < 0 || i > 1 || hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  if (!streams[dev][i] && hipStreamCreateWithFlags(&streams[dev][i], hipStreamNonBlocking) != hipSuccess)
    streams[dev][i] = nullptr;
  return streams[dev][i];
}

// The factor's second stream for a solve: only when the solve may fork
// (ctx == null: the synchronous entry points); a context without a side
// stream (the serving engine) keeps every view's work on its own stream.
static hipStream_t factor_aux(const SolveCtx* ctx, int i) { return ctx ? nullptr : factor_aux_stream(i); }

// Fork/join of the side stream around a block of independent work.
struct SideFork {
  hipEvent_t fork = nullptr, join = nullptr;
  hipStream_t side = nullptr, main = nullptr;
  bool open = false;
  ~SideFork() {
    // an early error return still joins, so the workspace is released (on
    // the caller's stream) only after the side stream's work
    if (open) (void)end(main);
    if (fork) (void)hipEventDestroy(fork);
    if (join) (void)hipEventDestroy(join);
  }
  // ctx == null: the per-device side stream; ctx->side == null: no fork,
  // the "side" work runs in order on st itself.
  int begin(hipStream_t st, const SolveCtx* ctx = nullptr) {
    main = st;
    if (ctx && !ctx->side) {
      side = st;
      return SRP_OK;
    }
    side = ctx ? ctx->side : side_stream();
    if (!side) { set_error("could not create a side stream"); return SRP_EDEVICE; }
    SRP_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
    SRP_HIP(hipEventCreateWithFlags(&join, hipEventDisableTiming));
    SRP_HIP(hipEventRecord(fork, st));
    SRP_HIP(hipStreamWaitEvent(side, fork, 0));
    open = true;
    return SRP_OK;
  }
  int end(hipStream_t st) {
    if (!open) return SRP_OK;
    open = false;
    SRP_HIP(hipEventRecord(join, side));
    SRP_HIP(hipStreamWaitEvent(st, join, 0));
    return SRP_OK;
  }
};

// ----------------------------------------------------------- the solver
struct RcgProblem {
  int nb = 1, k = 1, lda_cost = 0;
  int dtype = SRP_F32;      // element type of the data matrices
  int compute = SRP_F32;    // arithmetic of the fused passes
  const void* A[2] = {nullptr, nullptr};
  int64_t n = 0;
  int d[2] = {0, 0};
  double lam[2] = {0.0, 0.0};
  const double* Minv[2] = {nullptr, nullptr};
  const double* Yhat = nullptr;  // FDA: c x d rows sqrt(n_j)(m_j - m); S_B = Yhat^T Yhat
  int c = 0;
  const struct SparseData* sp = nullptr;   // CSR data (A unused): products in FP64 from the sparse forms
  const struct Woodbury* wb[2] = {nullptr, nullptr};   // block b's M^-1 in Woodbury form (Minv[b] unused)
};

// M^-1 for a sketch with fewer rows than columns (s < d, lambda > 0; the
// closing remark after Table costs): M = SA^T SA + lam I (d x d) is never
// formed or factored.  K = SA SA^T + lam I_s (s x s) is, in O(s^2 d + s^3),
// and by the Sherman-Morrison-Woodbury identity
//   M^-1 V = (V - SA^T K^-1 SA V) / lam,
// O(s d w + s^2 w) for w columns.
struct Woodbury {
  const void* SA = nullptr;   // the sketch, s x d (FP64 or FP32)
  bool f32 = false;
  int s = 0, d = 0;
  double lam = 0.0;
  const double* Kinv = nullptr;   // s x s
  double* t1 = nullptr;           // s x 64
  double* t2 = nullptr;           // s x 64
  double* skw = nullptr;          // split-K partials of its skinny products
  size_t skw_bytes = 0;
};

// Workspace a Woodbury block keeps for the whole solve (t1, t2, partials).
static size_t woodbury_keep_bytes(int s, int d) {
  return 2 * bytes_of<double>((size_t)s * 64) +
         std::max({skinny_ws_bytes(s, d, 64), skinny_ws_bytes(s, s, 64), skinny_ws_bytes(d, s, 64)}) + 1024;
}
// Scratch of its factorisation: SA^T in FP64 and the factor's own.
static size_t woodbury_factor_scratch(int s, int d) {
  return bytes_of<double>((size_t)d * s) + factor_ws_bytes(d, s) + 1024;
}

// K = SA SA^T + lam I_s is the Gram of SA^T (d x s) plus lam I: the sketch
// factor of SA^T gives K's Cholesky factor (KR) and K^-1.
static int woodbury_factor(const void* SA, int sk_dtype, int s, int d, double lam, double* KR, double* Kinv,
                           int* flag, Arena& scratch, Arena& keep, Woodbury* W, hipStream_t st) {
  double* SAt = scratch.take<double>((size_t)d * s);
  if (!SAt) { set_error("Woodbury factor: workspace too small"); return SRP_ENOMEM; }
  SRP_TRY(transpose_to_f64(SA, sk_dtype, s, d, SAt, st));
  Arena sub{scratch.base + scratch.used, scratch.cap - scratch.used, 0};
  SRP_TRY(sketch_factor_run(SAt, SRP_F64, d, s, lam, KR, nullptr, Kinv, flag, sub, st));
  W->SA = SA;
  W->f32 = sk_dtype != SRP_F64;
  W->s = s;
  W->d = d;
  W->lam = lam;
  W->Kinv = Kinv;
  W->t1 = keep.take<double>((size_t)s * 64);
  W->t2 = keep.take<double>((size_t)s * 64);
  W->skw_bytes = std::max({skinny_ws_bytes(s, d, 64), skinny_ws_bytes(s, s, 64), skinny_ws_bytes(d, s, 64)});
  W->skw = (double*)keep.take<char>(W->skw_bytes);
  if (!W->skw) { set_error("Woodbury form: workspace too small"); return SRP_ENOMEM; }
  return SRP_OK;
}

// out (d_b x w, row-major, w <= 64) = M_b^-1 V.
static int minv_apply(const RcgProblem& P, int b, const double* V, int w, double* out, double* skw, size_t skw_bytes,
                      hipStream_t st) {
  const int d = P.d[b];
  if (!P.wb[b]) return gemm_skinny_f64(d, d, w, P.Minv[b], d, false, V, w, out, w, skw, skw_bytes, st);
  const Woodbury& W = *P.wb[b];
  SkinnyProb p1{W.s, d, w, W.SA, d, false, V, w, W.t1, w};   // SA V
  p1.a_f32 = W.f32;
  SRP_TRY(gemm_skinny_batch(1, &p1, W.skw, W.skw_bytes, st));
  SRP_TRY(gemm_skinny_f64(W.s, W.s, w, W.Kinv, W.s, false, W.t1, w, W.t2, w, W.skw, W.skw_bytes, st));
  SkinnyProb p3{d, W.s, w, W.SA, d, true, W.t2, w, out, w};   // SA^T K^-1 SA V
  p3.a_f32 = W.f32;
  SRP_TRY(gemm_skinny_batch(1, &p3, W.skw, W.skw_bytes, st));
  RtrLinArgs la{};
  la.k = w;
  la.side[0] = RtrLinSide{out, V, 1.0 / W.lam, out, -1.0 / W.lam, nullptr, d};
  return rtr_lin(la, 1, st);
}

// Sparse data of a solve: the CSR views and their CSC copies; FDA adds the
// labels and the class means, whose products give the centred ones.
struct SparseData {
  CsrView csr[2];
  CscView csc[2];
  const int32_t* labels = nullptr;
  const double* means = nullptr;   // c x d class means
  double* T = nullptr;             // c x k: means W
  double* partial[2] = {nullptr, nullptr};   // per-segment partials of A_b^T P
};

struct RcgBuffers {
  double *U[2], *Ks[2], *Kc[2], *xi[2], *gold[2], *J[2], *Jc[2], *Z[2], *Wz[2];
  double* Pn = nullptr;      // two-pass route: n x 2k
  double* skw = nullptr;     // split-K partials of the skinny products
  size_t skw_bytes = 0;
  double* Tc = nullptr;      // FDA: Yhat W (c x k)
  double* parts = nullptr;   // two-pass route: split-k partials
  int ksplit = 1;
  SolverCtrl* ctrl;
  double* kk;
  double* part;
  double* mu;
  char* pass_ws;
  size_t pass_ws_bytes;
  // optional timing of the fused passes over the full data; *ran counts
  // the timed launches that did the work (a launch that finds the
  // converged flag set returns at once)
  bool time_passes = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>>* events = nullptr;
  int* ran_all = nullptr;   // two counters: main passes, BF16-phase passes
  int* ran = nullptr;
  char* rtr_ws = nullptr;   // the trust-region solver's vectors
  size_t rtr_ws_bytes = 0;
  TickGroup* group[2] = {nullptr, nullptr};   // grouped ticks (engine), for k <= 16 / k <= 32
};

__global__ void k_count_pass(const int* __restrict__ done, int* __restrict__ ran) {
  if (!(done && *done)) ++*ran;
}

static size_t kk_bytes() { return bytes_of<double>((size_t)(2 * KK_NSLOTS + 9) * KK_STRIDE); }

static int twopass_ksplit(int64_t n) {
  int64_t ks = (n + 1023) / 1024;
  if (ks > 128) ks = 128;
  if (ks < 1) ks = 1;
  return (int)ks;
}

static size_t skinny_bytes(int nb, int k, const int* d, int c) {
  size_t b = 0;
  for (int s = 0; s < nb; ++s) b += skinny_ws_bytes(d[s], d[s], 2 * k) + 256;
  if (c > 0) b = std::max({b, skinny_ws_bytes(c, d[0], k), skinny_ws_bytes(d[0], c, k)});
  return b;
}

static size_t rtr_ws_bytes(int nb, int k, const int* d);

static size_t rcg_buffers_bytes(int nb, int k, int64_t nmax, const int* d, int dtype, int c = 0) {
  size_t b = skinny_bytes(nb, k, d, c) + bytes_of<double>((size_t)std::max(c, 1) * k);
  for (int s = 0; s < nb; ++s) {
    const size_t dk = (size_t)d[s] * k;
    b += 6 * bytes_of<double>(dk) + bytes_of<double>((size_t)d[s] * nb * k) + 2 * bytes_of<double>(2 * dk);
  }
  b += bytes_of<SolverCtrl>(1) + kk_bytes() + partial_bytes(k, std::max(d[0], nb == 2 ? d[1] : 0)) +
       bytes_of<double>(KMAX) + bytes_of<int>(2);
  const size_t pw = std::max(pass_ws_bytes(nmax, d[0], nb == 2 ? d[1] : 0, k, SRP_F64),
                             pass_ws_bytes(nmax, d[0], nb == 2 ? d[1] : 0, k, SRP_F32));
  b += (pw + 255) & ~size_t(255);
  // two-pass FP64 route
  const int ks = twopass_ksplit(nmax);
  b += bytes_of<double>((size_t)nmax * nb * k);
  b += bytes_of<double>((size_t)ks * std::max(d[0], nb == 2 ? d[1] : 0) * nb * k);
  b += rtr_ws_bytes(nb, std::min(k, kRtrK), d);
  (void)dtype;
  return b;
}

static int rcg_buffers_take(RcgBuffers& B, Arena& ar, int nb, int k, int64_t nmax, const int* d, int c = 0) {
  B.skw_bytes = skinny_bytes(nb, k, d, c);
  B.skw = (double*)ar.take<char>(B.skw_bytes);
  B.Tc = ar.take<double>((size_t)std::max(c, 1) * k);
  for (int s = 0; s < nb; ++s) {
    const size_t dk = (size_t)d[s] * k;
    B.U[s] = ar.take<double>(dk);
    B.Ks[s] = ar.take<double>(dk);
    B.Kc[s] = ar.take<double>(dk);
    B.xi[s] = ar.take<double>(dk);
    B.gold[s] = ar.take<double>(dk);
    B.Jc[s] = ar.take<double>(dk);
    B.J[s] = ar.take<double>((size_t)d[s] * nb * k);
    B.Z[s] = ar.take<double>(2 * dk);
    B.Wz[s] = ar.take<double>(2 * dk);
    if (!B.Wz[s]) return SRP_ENOMEM;
  }
  for (int s = nb; s < 2; ++s) {
    B.U[s] = B.Ks[s] = B.Kc[s] = B.xi[s] = B.gold[s] = B.Jc[s] = B.J[s] = B.Z[s] = B.Wz[s] = nullptr;
  }
  B.ctrl = ar.take<SolverCtrl>(1);
  B.kk = (double*)ar.take<char>(kk_bytes());
  B.part = (double*)ar.take<char>(partial_bytes(k, std::max(d[0], nb == 2 ? d[1] : 0)));
  B.mu = ar.take<double>(KMAX);
  B.ran_all = ar.take<int>(2);
  B.pass_ws_bytes = std::max(pass_ws_bytes(nmax, d[0], nb == 2 ? d[1] : 0, k, SRP_F64),
                             pass_ws_bytes(nmax, d[0], nb == 2 ? d[1] : 0, k, SRP_F32));
  B.pass_ws = ar.take<char>(B.pass_ws_bytes);
  B.ksplit = twopass_ksplit(nmax);
  B.Pn = ar.take<double>((size_t)nmax * nb * k);
  B.parts = ar.take<double>((size_t)B.ksplit * std::max(d[0], nb == 2 ? d[1] : 0) * nb * k);
  B.rtr_ws_bytes = rtr_ws_bytes(nb, std::min(k, kRtrK), d);
  B.rtr_ws = ar.take<char>(B.rtr_ws_bytes);
  if (!B.ctrl || !B.kk || !B.part || !B.mu || !B.pass_ws || !B.Pn || !B.parts || !B.skw || !B.Tc || !B.ran_all ||
      !B.rtr_ws)
    return SRP_ENOMEM;
  return SRP_OK;
}

static ProbView make_view(const RcgProblem& P, RcgBuffers& B) {
  ProbView v{};
  v.nb = P.nb;
  v.k = P.k;
  v.lda_cost = P.lda_cost;
  for (int s = 0; s < P.nb; ++s) {
    SideView& q = v.s[s];
    q.d = P.d[s];
    q.lam = P.lam[s];
    q.U = B.U[s];
    q.Ks = B.Ks[s];
    q.Kc = B.Kc[s];
    q.xi = B.xi[s];
    q.gold = B.gold[s];
    q.J = B.J[s];
    q.jld = P.nb * P.k;
    q.js_off = s * P.k;
    q.jc_off = (P.nb == 2) ? (1 - s) * P.k : 0;
    q.Jc_sep = P.lda_cost ? B.Jc[s] : nullptr;
    q.Z = B.Z[s];
    q.Wz = B.Wz[s];
  }
  v.mu = B.mu;
  v.ctrl = B.ctrl;
  v.kk = B.kk;
  v.part = B.part;
  v.part_slices = partial_slices(std::max(P.d[0], P.nb == 2 ? P.d[1] : 0));
  // eigenvectors of the projection's k x k system to relative off-diagonal
  // 1e-15 (a looser stop for FP32 passes stalled clustered problems)
  v.eig_tol2 = 1e-30;
  return v;
}

// J_b = A_b^T [A_0 W_0 | A_1 W_1] with FP64 arithmetic in two reads of the
// data; used where the fused pass has no FP64 instance for the shape.  The
// skinny products take it when A fits their 32-bit offsets: P = A W row
// blocks over the whole contraction (no partials), then A^T P split over
// the rows into at most ksplit partials; else the generic GEMM.
static int twopass_f64(const RcgProblem& P, RcgBuffers& B, double* const* W, hipStream_t st) {
  const int k = P.k, nb = P.nb, ldp = nb * k;
  if (P.dtype == SRP_BF16) {
    set_error("two-pass FP64 route does not take BF16 data");
    return SRP_EINVAL;
  }
  const bool f32 = (P.dtype == SRP_F32);
  const int64_t esz = f32 ? 4 : 8;
  bool skinny = ldp <= 64 && P.n * ldp * 8 < (int64_t(1) << 31);
  for (int s = 0; s < nb; ++s) skinny = skinny && P.n * P.d[s] * esz < (int64_t(1) << 31);
  if (skinny) {
    SkinnyProb pr[2];
    for (int s = 0; s < nb; ++s) {
      pr[s] = SkinnyProb{(int)P.n, P.d[s], k, P.A[s], P.d[s], false, W[s], k, B.Pn + s * k, ldp};
      pr[s].a_f32 = f32;
    }
    SRP_TRY(gemm_skinny_batch(nb, pr, nullptr, 0, st, std::max(P.d[0], nb == 2 ? P.d[1] : 0)));
    const int64_t rows_per = (P.n + B.ksplit - 1) / B.ksplit;
    const int slice = (int)((rows_per + 31) / 32 * 32);
    const size_t ws = bytes_of<double>((size_t)B.ksplit * std::max(P.d[0], nb == 2 ? P.d[1] : 0) * ldp);
    for (int s = 0; s < nb; ++s) {
      SkinnyProb q{P.d[s], (int)P.n, ldp, P.A[s], P.d[s], true, B.Pn, ldp, B.J[s], ldp};
      q.a_f32 = f32;
      SRP_TRY(gemm_skinny_batch(1, &q, B.parts, ws, st, slice));
    }
    return SRP_OK;
  }
  for (int s = 0; s < nb; ++s) {
    GemmArgs g{};
    g.m = (int)P.n; g.n = k; g.kk = P.d[s]; g.alpha = 1.0; g.beta = 0.0;
    g.A = P.A[s]; g.lda = P.d[s]; g.ta = false; g.a_f32 = f32;
    g.B = W[s]; g.ldb = k; g.tb = false; g.b_f32 = false;
    g.C = B.Pn + s * k; g.ldc = ldp;
    SRP_TRY(gemm_f64(g, st));
  }
  for (int s = 0; s < nb; ++s) {
    const int64_t cnt = (int64_t)P.d[s] * ldp;
    GemmArgs g{};
    g.m = P.d[s]; g.n = ldp; g.kk = (int)P.n; g.alpha = 1.0; g.beta = 0.0;
    g.A = P.A[s]; g.lda = P.d[s]; g.ta = true; g.a_f32 = f32;
    g.B = B.Pn; g.ldb = ldp; g.tb = false; g.b_f32 = false;
    g.C = B.parts; g.ldc = ldp; g.ksplit = B.ksplit; g.c_split_stride = cnt;
    SRP_TRY(gemm_f64(g, st));
    SRP_TRY(sum_parts_f64(B.parts, B.ksplit, cnt, cnt, B.J[s], 0, 0.0, st));
  }
  return SRP_OK;
}

// Products of CSR data, FP64: P_b = A_b W_b (n x k each, side by side in
// B.Pn), then J_b = A_b^T [P_0 | P_1] from the CSC copies.  FDA: the rows
// of Xhat = X - E C (E the one-hot labels, C the class means) give
// Xhat W = X W - (C W)[labels] per row, and Xhat^T (Xhat W) = X^T (Xhat W)
// because the class sums of the rows of Xhat vanish (E^T Xhat = 0): the
// centred products cost nnz(X) k + c d k, without an n x d Xhat.
static int sparse_pass(const RcgProblem& P, RcgBuffers& B, double* const* W, const int* done, hipStream_t st) {
  const SparseData& S = *P.sp;
  const int k = P.k, nb = P.nb, ldp = nb * k;
  for (int b = 0; b < nb; ++b) {
    const double* sub = nullptr;
    if (S.labels) {
      SRP_TRY(gemm_skinny_f64(P.c, P.d[0], k, S.means, P.d[0], false, W[0], k, S.T, k, B.skw, B.skw_bytes, st));
      sub = S.T;
    }
    SRP_TRY(csr_times_dense(S.csr[b], W[b], k, k, B.Pn + b * k, ldp, sub, S.labels, done, st));
  }
  for (int b = 0; b < nb; ++b)
    SRP_TRY(csc_times_dense(S.csc[b], B.Pn, ldp, ldp, B.J[b], ldp, S.partial[b], done, st));
  return SRP_OK;
}

// Data products along directions W (d_b x k): fills J (and FDA's S_B W).
static int data_pass(const RcgProblem& P, RcgBuffers& B, double* const* W, int compute, const int* done,
                     hipStream_t st) {
  if (P.sp) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (B.time_passes && B.events) {
      SRP_HIP(hipEventCreate(&e0));
      SRP_HIP(hipEventCreate(&e1));
      SRP_HIP(hipEventRecord(e0, st));
    }
    SRP_TRY(sparse_pass(P, B, W, done, st));
    if (e0) {
      SRP_HIP(hipEventRecord(e1, st));
      B.events->push_back({e0, e1});
      if (B.ran) {
        hipLaunchKernelGGL(k_count_pass, dim3(1), dim3(1), 0, st, done, B.ran);
        SRP_LAUNCH_CHECK();
      }
    }
  } else if (compute == SRP_F64 && !pass_limits_ok(P.dtype, SRP_F64, P.d[0], P.d[1], P.k, P.nb)) {
    SRP_TRY(twopass_f64(P, B, W, st));
  } else {
    Arena pw{B.pass_ws, B.pass_ws_bytes, 0};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (B.time_passes && B.events) {
      SRP_HIP(hipEventCreate(&e0));
      SRP_HIP(hipEventCreate(&e1));
    }
    SRP_TRY(gram_pass_run(P.A[0], P.nb == 2 ? P.A[1] : nullptr, P.dtype, compute, P.n, P.d[0], P.d[1], P.k, W[0],
                          P.nb == 2 ? W[1] : nullptr, B.J[0], P.nb == 2 ? B.J[1] : nullptr, done, pw, st, e0, e1,
                          e0 ? B.ran : nullptr));
    if (e0) B.events->push_back({e0, e1});
  }
  if (P.lda_cost) {   // S_B W = Yhat^T (Yhat W): c-row factor instead of the d x d matrix
    SRP_TRY(gemm_skinny_f64(P.c, P.d[0], P.k, P.Yhat, P.d[0], false, W[0], P.k, B.Tc, P.k, B.skw, B.skw_bytes, st));
    SRP_TRY(gemm_skinny_f64(P.d[0], P.c, P.k, P.Yhat, P.d[0], true, B.Tc, P.k, B.Jc[0], P.k, B.skw, B.skw_bytes, st));
  }
  return SRP_OK;
}

static int apply_minv(const RcgProblem& P, RcgBuffers& B, hipStream_t st) {
  if (P.wb[0] || P.wb[1]) {
    for (int b = 0; b < P.nb; ++b) SRP_TRY(minv_apply(P, b, B.Z[b], 2 * P.k, B.Wz[b], B.skw, B.skw_bytes, st));
    return SRP_OK;
  }
  SkinnyProb pr[2];
  for (int s = 0; s < P.nb; ++s)
    pr[s] = SkinnyProb{P.d[s], P.d[s], 2 * P.k, P.Minv[s], P.d[s], false, B.Z[s], 2 * P.k, B.Wz[s], 2 * P.k};
  return gemm_skinny_batch(P.nb, pr, B.skw, B.skw_bytes, st);
}

// Gradient, transported direction and new CG direction at the current point.
static int direction_step(const RcgProblem& P, RcgBuffers& B, const ProbView& v, hipStream_t st) {
  SRP_TRY(apply_minv(P, B, st));
  SRP_TRY(launch_dir_partials(v, st));
  SRP_TRY(launch_ctrl_dir(v, st));
  SRP_TRY(launch_combine(v, st));
  return SRP_OK;
}

// ------------------------------------------------------ grouped ticks
// The serving engine runs several solves at once.  Their data passes are
// their own (each on its solve's stream), but the small kernels of an
// iteration (the line search's partials and controller, the update; then
// M^-1 Z, the direction's partials and controller, the combination) are
// latency-bound, a few microseconds of work behind a launch each.  A tick
// group runs each of those steps for every member as one launch.  All of a
// member's iteration work goes to the group's one stream while it is a
// member (no cross-stream joins inside an iteration): an iteration is two
// phases, a member queues its phase work (data pass; refresh) and posts
// the phase, and the phase fires, queuing the grouped kernels behind every
// member's work, when every member has posted it.  Members join and leave
// between iterations (their own stream and the group's joined by events).
// Each member's arithmetic is the same as alone.
struct TickMember {
  int slot = -1;
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr;
  ProbView v{};
  PartialArgs ls{}, dir{};
  const RcgProblem* P = nullptr;
  int ntr = 0;
  size_t lds_ls = 0, lds_dir = 0;
  int dmax = 0;
  size_t skw_need = 0;   // the M^-1 Z products' partials
};

struct TickGroup {
  explicit TickGroup(int kc) : kc_(kc) {}
  ~TickGroup() {
    if (st_) (void)hipStreamSynchronize(st_);
    if (views_) (void)hipFree(views_);
    if (ls_) (void)hipFree(ls_);
    if (dir_) (void)hipFree(dir_);
    if (skw_) (void)hipFree(skw_);
    if (ev_) (void)hipEventDestroy(ev_);
    if (st_) (void)hipStreamDestroy(st_);
  }
  int init() {
    SRP_HIP(hipStreamCreateWithFlags(&st_, hipStreamNonBlocking));
    SRP_HIP(hipEventCreateWithFlags(&ev_, hipEventDisableTiming));
    SRP_HIP(hipMalloc((void**)&views_, sizeof(ProbView) * kGroupMax));
    SRP_HIP(hipMalloc((void**)&ls_, sizeof(PartialArgs) * kGroupMax));
    SRP_HIP(hipMalloc((void**)&dir_, sizeof(PartialArgs) * kGroupMax));
    skw_bytes_ = size_t(32) << 20;
    SRP_HIP(hipMalloc((void**)&skw_, skw_bytes_));
    return SRP_OK;
  }
  // A solve can join when its M^-1 products fit the group's partials
  // (two views per chunk of four problems).
  bool fits(const TickMember& m) const { return m.skw_need * 2 <= skw_bytes_; }
  int join(TickMember& m) {
    std::unique_lock<std::mutex> lk(mu_);
    cv_.wait(lk, [&] { return phase_ == 0; });
    int slot = -1;
    for (int i = 0; i < kGroupMax && slot < 0; ++i)
      if (!used_[i]) slot = i;
    if (slot < 0) return SRP_EBUSY;
    used_[slot] = true;
    m.slot = slot;
    SRP_HIP(hipMemcpyAsync(views_ + slot, &m.v, sizeof(ProbView), hipMemcpyHostToDevice, st_));
    SRP_HIP(hipMemcpyAsync(ls_ + slot, &m.ls, sizeof(PartialArgs), hipMemcpyHostToDevice, st_));
    SRP_HIP(hipMemcpyAsync(dir_ + slot, &m.dir, sizeof(PartialArgs), hipMemcpyHostToDevice, st_));
    SRP_HIP(hipStreamSynchronize(st_));
    members_.push_back(&m);
    return SRP_OK;
  }
  // Leaves between iterations (or, on an error, in the middle of one: the
  // phase the others have posted then fires without it).
  int leave(TickMember& m) {
    std::unique_lock<std::mutex> lk(mu_);
    members_.erase(std::remove(members_.begin(), members_.end(), &m), members_.end());
    used_[m.slot] = false;
    m.slot = -1;
    int rc = SRP_OK;
    if (!members_.empty() && posted_.size() == members_.size()) rc = fire();
    cv_.notify_all();
    return rc != SRP_OK ? rc : err_;
  }
  // The group's stream: a member's iteration loop queues all its work
  // (data passes, refreshes, polls) there while it is a member.
  hipStream_t stream() const { return st_; }
  // Post phase `ph` of the current iteration for m (its work for the phase
  // already queued on the group's stream); returns once the grouped
  // launches of that phase are queued behind it.
  int post(TickMember& m, int ph) {
    std::unique_lock<std::mutex> lk(mu_);
    cv_.wait(lk, [&] { return phase_ == ph; });
    posted_.push_back(&m);
    const uint64_t g = gen_;
    if (posted_.size() == members_.size()) {
      const int rc = fire();
      if (rc != SRP_OK) err_ = rc;
      cv_.notify_all();
    } else {
      cv_.wait(lk, [&] { return gen_ != g; });
    }
    return err_;
  }
  uint64_t ticks() const { return gen_; }

 private:
  int fire() {
    GroupSel sel{};
    sel.n = (int)posted_.size();
    int slices = 1, dmax = 1, kmax = 1;
    size_t lds = 0;
    for (int i = 0; i < sel.n; ++i) {
      TickMember* m = posted_[i];
      sel.idx[i] = m->slot;
      sel.aux[i] = m->ntr;
      slices = std::max(slices, m->v.part_slices);
      dmax = std::max(dmax, m->dmax);
      kmax = std::max(kmax, m->v.k);
      lds = std::max(lds, phase_ == 0 ? m->lds_ls : m->lds_dir);
    }
    if (phase_ == 0) {
      SRP_TRY(launch_partials_g(ls_, sel, slices, (int64_t)(2 * kmax) * (6 * kmax), st_));
      SRP_TRY(launch_ctrl_ls_g(views_, sel, lds, kc_, st_));
      SRP_TRY(launch_update_g(views_, sel, 0, dmax, kc_, st_));
    } else {
      // M^-1 Z of every member's views, four problems per launch
      std::vector<SkinnyProb> pr;
      for (int i = 0; i < sel.n; ++i) {
        const RcgProblem& P = *posted_[i]->P;
        for (int b = 0; b < P.nb; ++b)
          pr.push_back(SkinnyProb{P.d[b], P.d[b], 2 * P.k, P.Minv[b], P.d[b], false, posted_[i]->v.s[b].Z,
                                  2 * P.k, posted_[i]->v.s[b].Wz, 2 * P.k});
      }
      for (size_t q = 0; q < pr.size(); q += 4) {
        const int np = (int)std::min<size_t>(4, pr.size() - q);
        SRP_TRY(gemm_skinny_batch(np, pr.data() + q, skw_, skw_bytes_, st_));
      }
      SRP_TRY(launch_partials_g(dir_, sel, slices, (int64_t)(2 * kmax) * (4 * kmax), st_));
      SRP_TRY(launch_ctrl_dir_g(views_, sel, lds, kc_, st_));
      SRP_TRY(launch_combine_g(views_, sel, (int64_t)dmax * kmax, kc_, st_));
    }
    posted_.clear();
    phase_ = 1 - phase_;
    ++gen_;
    return SRP_OK;
  }

  std::mutex mu_;
  std::condition_variable cv_;
  int phase_ = 0;
  uint64_t gen_ = 0;
  int err_ = SRP_OK;
  std::vector<TickMember*> members_, posted_;
  bool used_[kGroupMax] = {};
  hipStream_t st_ = nullptr;
  hipEvent_t ev_ = nullptr;
  ProbView* views_ = nullptr;
  PartialArgs* ls_ = nullptr;
  PartialArgs* dir_ = nullptr;
  double* skw_ = nullptr;
  size_t skw_bytes_ = 0;
  int kc_;
};

TickGroup* tick_group_create(int kc, int* status) {
  auto* g = new TickGroup(kc);
  const int rc = g->init();
  if (status) *status = rc;
  if (rc != SRP_OK) {
    delete g;
    return nullptr;
  }
  return g;
}

void tick_group_destroy(TickGroup* g) { delete g; }

uint64_t tick_group_ticks(const TickGroup* g) { return g ? g->ticks() : 0; }

// The member record of a solve (its grouped-launch parameters), or false
// when the solve cannot take part (Woodbury metric, too large).
static bool tick_member(const RcgProblem& P, const ProbView& v, hipStream_t st, TickMember* m) {
  if (P.wb[0] || P.wb[1]) return false;
  m->st = st;
  m->v = v;
  m->P = &P;
  fill_partial_args(v, 0, &m->ls);
  fill_partial_args(v, 1, &m->dir);
  m->ntr = ctrl_ls_shape(P.k, P.nb, &m->lds_ls);
  if (m->ntr < 1) return false;
  m->lds_dir = ctrl_dir_lds(P.k, P.nb);
  m->dmax = std::max(P.d[0], P.nb == 2 ? P.d[1] : 0);
  m->skw_need = 0;
  for (int b = 0; b < P.nb; ++b) m->skw_need += skinny_ws_bytes(P.d[b], P.d[b], 2 * P.k) + 256;
  return true;
}

struct RcgResult {
  int status = SRP_OK;
  int iterations = 0;
  int passes = 0;
  double f = 0.0, gg = 0.0;
};

static int read_ctrl(SolverCtrl* dev, SolverCtrl* host, hipStream_t st) {
  SRP_HIP(hipMemcpyAsync(host, dev, sizeof(SolverCtrl), hipMemcpyDeviceToHost, st));
  SRP_HIP(hipStreamSynchronize(st));
  return SRP_OK;
}

// Convergence polls without draining the stream: the flag is copied into
// pinned host memory behind an event, and the host reads it only after it
// has queued the next batch of iterations (those return at once on the
// device once the flag is set).  The pinned words are pooled: one per solve
// running at a time, kept for reuse until the process ends.
class FlagPoll {
 public:
  ~FlagPoll() {
    if (pending_) (void)hipEventSynchronize(ev_);   // no copy in flight into a pooled word
    if (ev_) (void)hipEventDestroy(ev_);
    if (h_) {
      std::lock_guard<std::mutex> g(mu());
      pool().push_back(h_);
    }
  }
  int init() {
    {
      std::lock_guard<std::mutex> g(mu());
      if (!pool().empty()) { h_ = pool().back(); pool().pop_back(); }
    }
    if (!h_) SRP_HIP(hipHostMalloc((void**)&h_, 64, hipHostMallocDefault));
    SRP_HIP(hipEventCreateWithFlags(&ev_, hipEventDisableTiming));
    return SRP_OK;
  }
  // Queue a copy of *done (device) taken after the work queued so far.
  int post(const int* done, hipStream_t st) {
    SRP_HIP(hipMemcpyAsync(h_, done, sizeof(int), hipMemcpyDeviceToHost, st));
    SRP_HIP(hipEventRecord(ev_, st));
    pending_ = true;
    return SRP_OK;
  }
  // Wait for the last posted copy; *set = its value (false if none posted).
  int read(bool* set) {
    *set = false;
    if (!pending_) return SRP_OK;
    SRP_HIP(hipEventSynchronize(ev_));
    pending_ = false;
    *set = *h_ != 0;
    return SRP_OK;
  }
 private:
  static std::mutex& mu() { static std::mutex m; return m; }
  static std::vector<int*>& pool() { static std::vector<int*> v; return v; }
  int* h_ = nullptr;
  hipEvent_t ev_ = nullptr;
  bool pending_ = false;
};

// Runs Riemannian CG from qf_B(start).  On return B.U holds the final point.
static int rcg_run(const RcgProblem& P, RcgBuffers& B, double* const* start, int max_iter, double tol,
                   int check_every, int refresh_every, bool finalize, bool final_f64, double* sigma_out,
                   RcgResult& res, hipStream_t st) {
  const int k = P.k, nb = P.nb;
  ProbView v = make_view(P, B);
  for (int s = 0; s < nb; ++s) {
    const int64_t dk = (int64_t)P.d[s] * k;
    SRP_TRY(fill_f64(B.U[s], dk, 0.0, st));
    SRP_TRY(fill_f64(B.Ks[s], dk, 0.0, st));
    SRP_TRY(fill_f64(B.Kc[s], dk, 0.0, st));
    SRP_TRY(fill_f64(B.gold[s], dk, 0.0, st));
    SRP_TRY(copy_f64(B.xi[s], start[s], dk, st));
  }
  SRP_TRY(launch_ctrl_init(B.ctrl, tol, max_iter, st));
  int passes = 0;
  // qf_B(start): a data pass along the start point, step t = 1 from U = 0.
  SRP_TRY(data_pass(P, B, B.xi, P.compute, nullptr, st));
  ++passes;
  SRP_TRY(launch_ls_partials(v, st));
  SRP_TRY(launch_ctrl_ls(v, st));
  SRP_TRY(launch_update(v, 0, st));
  SRP_TRY(direction_step(P, B, v, st));
  const int* done = &B.ctrl->done;
  SolverCtrl hc{};
  FlagPoll poll;
  SRP_TRY(poll.init());
  int passes_posted = passes;   // passes queued when the pending flag copy was
  // grouped ticks (serving engine): this solve's small kernels run in the
  // group's launches
  TickGroup* grp = B.group[k <= 16 ? 0 : 1];
  TickMember mem;
  struct Ev {
    hipEvent_t e = nullptr;
    ~Ev() { if (e) (void)hipEventDestroy(e); }
  } mev;
  bool grouped = false;
  const hipStream_t own = st;
  if (grp && max_iter > 0 && tick_member(P, v, st, &mem) && grp->fits(mem)) {
    SRP_HIP(hipEventCreateWithFlags(&mev.e, hipEventDisableTiming));
    mem.ev = mev.e;
    SRP_TRY(grp->join(mem));
    grouped = true;
    // the loop's work goes to the group's stream, after this solve's own
    SRP_HIP(hipEventRecord(mev.e, own));
    SRP_HIP(hipStreamWaitEvent(grp->stream(), mev.e, 0));
    st = grp->stream();
  }
  // on an early return: leave, and make the solve's own stream wait for the
  // work it queued on the group's stream (its buffers stay in use until then)
  struct Leave {
    TickGroup* g = nullptr;
    TickMember* m = nullptr;
    hipStream_t own = nullptr;
    ~Leave() {
      if (!g) return;
      (void)g->leave(*m);
      if (hipEventRecord(m->ev, g->stream()) == hipSuccess) (void)hipStreamWaitEvent(own, m->ev, 0);
    }
  } leave_guard{grouped ? grp : nullptr, &mem, own};
  for (int it = 1; it <= max_iter; ++it) {
    SRP_TRY(data_pass(P, B, B.xi, P.compute, done, st));
    ++passes;
    if (grouped) {
      SRP_TRY(grp->post(mem, 0));
    } else {
      SRP_TRY(launch_ls_partials(v, st));
      SRP_TRY(launch_ctrl_ls(v, st));
      SRP_TRY(launch_update(v, 0, st));
    }
    if (refresh_every > 0 && it % refresh_every == 0) {
      SRP_TRY(data_pass(P, B, B.U, P.compute, done, st));
      ++passes;
      SRP_TRY(launch_update(v, 1, st));
    }
    if (grouped) SRP_TRY(grp->post(mem, 1));
    else SRP_TRY(direction_step(P, B, v, st));
    if (it % check_every == 0 || it == max_iter) {
      // the flag posted one batch ago: if set, this batch ran as no-ops
      bool was_done = false;
      const int prev = passes_posted;
      SRP_TRY(poll.read(&was_done));
      if (was_done) {
        passes = prev;
        break;
      }
      SRP_TRY(poll.post(done, st));
      passes_posted = passes;
    }
  }
  if (grouped) {   // leave before the finish, so the group's ticks do not wait for it
    leave_guard.g = nullptr;
    SRP_TRY(grp->leave(mem));
    SRP_HIP(hipEventRecord(mev.e, st));
    SRP_HIP(hipStreamWaitEvent(own, mev.e, 0));
    st = own;
  }
  SRP_TRY(read_ctrl(B.ctrl, &hc, st));
  res.status = hc.status;
  res.iterations = hc.iter;
  res.f = hc.f;
  res.gg = hc.gg;
  if (hc.status == SRP_ENOTSPD) {
    set_error("Cholesky breakdown in the retraction (Gram not positive definite)");
    res.passes = passes;
    return SRP_OK;
  }
  if (finalize) {
    SRP_TRY(data_pass(P, B, B.U, final_f64 ? SRP_F64 : P.compute, nullptr, st));
    ++passes;
    SRP_TRY(launch_update(v, 2, st));
    SRP_TRY(launch_final_partials(v, st));
    SRP_TRY(launch_ctrl_final(v, sigma_out, st));
    SRP_TRY(launch_apply_rot(v, st));
    SRP_TRY(launch_sign_fix(v, st));
    SolverCtrl fc{};
    SRP_TRY(read_ctrl(B.ctrl, &fc, st));
    res.f = fc.f;
    if (fc.status == SRP_ENOTSPD) {
      res.status = SRP_ENOTSPD;
      set_error("Cholesky breakdown in the final retraction");
    }
  }
  res.passes = passes;
  return SRP_OK;
}

// ------------------------------------------------- trust region
// Riemannian trust-region with a truncated CG inner solver (Steihaug-Toint),
// in the metric g(xi, eta) = tr(xi^T M eta) of Table 1.  The Hessian of
// Table 1 applied to a tangent vector reads, with S_g the symmetric solution
// of the gradient's projection (X^T grad_E f - X^T M grad f = S_g),
//   Hess f[d] = Pi_Z(M^-1 (D^2 f[d] - B d S_g)),
// which for CCA is Eq. HessCCA (D^2 f[d] = -[Sxy d_V N; Sxy^T d_U N]) and
// for FDA Eq. LDAhess (D^2 f[d] = -S_B d N).  One fused data pass along d
// gives B d and the cross product; the projection reuses P = (BZ)^T M^-1 BZ,
// factored once per outer iteration.  Every tangent vector v is carried
// with its image M v (M Pi(M^-1 h) = h - BZ S_h), so the metric's inner
// products are plain traces.  The trial point's retraction Gram and cost
// come from products accumulated along the inner iterations (B eta and the
// cross product of eta are sums of the passes along the CG directions): no
// extra data pass.
struct RtrState {
  double *BZ[2], *MiK[2], *e[2], *w[2], *grad[2], *Mg[2], *r[2], *Mr[2], *dl[2], *Mdl[2];
  double *eta[2], *Meta[2], *Beta[2], *Ceta[2], *MHeta[2], *h[2], *wh[2], *Hd[2], *MHd[2], *Bd[2], *Cd[2], *tmp[2];
  double *P[2], *Q[2], *lam[2], *Sg[2], *Cg[2], *Sh[2], *Ch[2], *E[2], *F[2], *Lit[2], *X0[4], *Nm;
  double* dots;     // device scalars
  double* hdots;    // pinned host copy
};

static size_t rtr_ws_bytes(int nb, int k, const int* d) {
  size_t b = 0;
  for (int s = 0; s < nb; ++s) b += 22 * bytes_of<double>((size_t)d[s] * k);
  b += (2 * 11 + 5) * bytes_of<double>((size_t)kRtrK * kRtrK) + bytes_of<double>(16);
  return b + 64 * 256;
}

static int rtr_take(RtrState& R, Arena& a, int nb, int k, const int* d) {
  for (int s = 0; s < 2; ++s) {
    double** vecs[] = {&R.BZ[s], &R.MiK[s], &R.e[s], &R.w[s], &R.grad[s], &R.Mg[s], &R.r[s], &R.Mr[s], &R.dl[s],
                       &R.Mdl[s], &R.eta[s], &R.Meta[s], &R.Beta[s], &R.Ceta[s], &R.MHeta[s], &R.h[s], &R.wh[s],
                       &R.Hd[s], &R.MHd[s], &R.Bd[s], &R.Cd[s], &R.tmp[s]};
    for (double** v : vecs) *v = s < nb ? a.take<double>((size_t)d[s] * k) : nullptr;
    double** mats[] = {&R.P[s], &R.Q[s], &R.lam[s], &R.Sg[s], &R.Cg[s], &R.Sh[s], &R.Ch[s], &R.E[s], &R.F[s],
                       &R.Lit[s]};
    for (double** m : mats) *m = s < nb ? a.take<double>((size_t)kRtrK * kRtrK) : nullptr;
  }
  for (int q = 0; q < 4; ++q) R.X0[q] = a.take<double>((size_t)kRtrK * kRtrK);
  R.Nm = a.take<double>((size_t)kRtrK * kRtrK);
  R.dots = a.take<double>(16);
  if (!R.dots || !R.tmp[nb - 1]) { set_error("trust region: workspace too small"); return SRP_ENOMEM; }
  return SRP_OK;
}

struct RtrResult {
  int status = SRP_OK, outer = 0, inner = 0, passes = 0;
  double f = 0.0, gg = 0.0;
};

static int rtr_run(const RcgProblem& P, RcgBuffers& B, RtrState& R, const double* mu_host, int max_outer,
                   int max_inner, double tol, int refresh_every, RtrResult& res, hipStream_t st) {
  const int k = P.k, nb = P.nb;
  const int* d = P.d;
  const double cs = P.lda_cost ? 0.5 : 1.0;   // f = cs tr(Z_0^T e_0)
  auto lin = [&](double* const* out, double a, double* const* A, double c, double* const* C,
                 double* const* K) -> int {
    RtrLinArgs la{};
    la.k = k;
    for (int b = 0; b < nb; ++b) {
      la.side[b] = RtrLinSide{out[b], A ? A[b] : nullptr, a, C ? C[b] : nullptr, c, K ? K[b] : nullptr, d[b]};
    }
    return rtr_lin(la, nb, st);
  };
  // C_b = op(X_b)^T Y_b (k x k) for both blocks, one launch
  auto gram = [&](double* const* X, double* const* Y, double* const* Cout) -> int {
    SkinnyProb pr[2];
    for (int b = 0; b < nb; ++b) pr[b] = SkinnyProb{k, d[b], k, X[b], k, true, Y[b], k, Cout[b], k};
    return gemm_skinny_batch(nb, pr, B.skw, B.skw_bytes, st);
  };
  auto minv = [&](double* const* X, double* const* Out) -> int {
    if (P.wb[0] || P.wb[1]) {
      for (int b = 0; b < nb; ++b) SRP_TRY(minv_apply(P, b, X[b], k, Out[b], B.skw, B.skw_bytes, st));
      return SRP_OK;
    }
    SkinnyProb pr[2];
    for (int b = 0; b < nb; ++b) pr[b] = SkinnyProb{d[b], d[b], k, P.Minv[b], d[b], false, X[b], k, Out[b], k};
    return gemm_skinny_batch(nb, pr, B.skw, B.skw_bytes, st);
  };
  auto dots = [&](int np, double* const* X0, double* const* Y0, double* const* X1, double* const* Y1,
                  double* const* X2, double* const* Y2, double* const* X3, double* const* Y3, int nbp = 0) -> int {
    RtrDotArgs da{};
    da.k = k; da.nb = nbp ? nbp : nb; da.np = np; da.out = R.dots;
    da.d[0] = d[0]; da.d[1] = nb == 2 ? d[1] : 0;
    double* const* xs[4] = {X0, X1, X2, X3};
    double* const* ys[4] = {Y0, Y1, Y2, Y3};
    for (int p = 0; p < np; ++p)
      for (int b = 0; b < da.nb; ++b) { da.X[p][b] = xs[p][b]; da.Y[p][b] = ys[p][b]; }
    SRP_TRY(rtr_dots(da, st));
    SRP_HIP(hipMemcpyAsync(R.hdots, R.dots, sizeof(double) * np, hipMemcpyDeviceToHost, st));
    SRP_HIP(hipStreamSynchronize(st));
    return SRP_OK;
  };
  // the pass along dirs: B dirs (with lambda) into Bout, cross products into Cout
  auto pass = [&](double* const* dirs, double* const* Bout, double* const* Cout) -> int {
    SRP_TRY(data_pass(P, B, dirs, P.compute, nullptr, st));
    ++res.passes;
    // J_b = A_b^T [A_0 d_0 | A_1 d_1]: block b of it (plus lambda d_b) is
    // B_b d_b, the other block the cross product (FDA: S_B d from Jc)
    RtrLinArgs la{}, lc{};
    la.k = lc.k = k;
    for (int b = 0; b < nb; ++b) {
      la.side[b] = RtrLinSide{Bout[b], B.J[b] + b * k, 1.0, dirs[b], P.lam[b], nullptr, d[b], nb * k, 0};
      if (P.lda_cost) lc.side[b] = RtrLinSide{Cout[b], B.Jc[b], 1.0, nullptr, 0.0, nullptr, d[b], 0, 0};
      else lc.side[b] = RtrLinSide{Cout[b], B.J[b] + (1 - b) * k, 1.0, nullptr, 0.0, nullptr, d[b], nb * k, 0};
    }
    SRP_TRY(rtr_lin(la, nb, st));
    SRP_TRY(rtr_lin(lc, nb, st));
    return SRP_OK;
  };
  // N as a diagonal matrix
  {
    double Nh[kRtrK * kRtrK] = {};
    for (int i = 0; i < k; ++i) Nh[i * k + i] = mu_host[i];
    SRP_HIP(hipMemcpyAsync(R.Nm, Nh, sizeof(double) * k * k, hipMemcpyHostToDevice, st));
  }
  double* Nm2[2] = {R.Nm, R.Nm};
  const double Dbar = std::sqrt((double)k * nb), rho_prime = 0.1;
  double Delta = Dbar / 8.0;
  int accepted = 0;
  double f = 0.0, gg = 0.0;
  for (int outer = 0; outer <= max_outer; ++outer) {
    // gradient at Z: BZ = Ks + lam Z, e = -Kc N, S_g, grad, M grad
    for (int b = 0; b < nb; ++b) {
      RtrLinArgs la{};
      la.k = k;
      la.side[0] = RtrLinSide{R.BZ[b], B.Ks[b], 1.0, B.U[b], P.lam[b], nullptr, d[b]};
      SRP_TRY(rtr_lin(la, 1, st));
    }
    SRP_TRY(lin(R.e, 0.0, nullptr, -1.0, B.Kc, Nm2));
    SRP_TRY(minv(R.BZ, R.MiK));
    SRP_TRY(minv(R.e, R.w));
    SRP_TRY(gram(R.BZ, R.MiK, R.P));
    for (int b = 0; b < nb; ++b) SRP_TRY(launch_rr_eig(R.P[b], k, k, R.Q[b], R.lam[b], st));
    SRP_TRY(gram(R.BZ, R.w, R.Cg));
    {
      RtrSylvArgs sa{};
      sa.k = k;
      for (int b = 0; b < nb; ++b) { sa.Q[b] = R.Q[b]; sa.lam[b] = R.lam[b]; sa.C[b] = R.Cg[b]; sa.S[b] = R.Sg[b]; }
      SRP_TRY(rtr_sylv(sa, nb, st));
    }
    SRP_TRY(lin(R.grad, 1.0, R.w, -1.0, R.MiK, R.Sg));
    SRP_TRY(lin(R.Mg, 1.0, R.e, -1.0, R.BZ, R.Sg));
    // f needs block 0 only, ||grad||^2 both blocks
    {
      double* const* Z0 = B.U;
      SRP_TRY(dots(1, Z0, R.e, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 1));
      f = cs * R.hdots[0];
    }
    SRP_TRY(dots(1, R.grad, R.Mg, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr));
    gg = R.hdots[0];
    res.f = f;
    res.gg = gg;
    res.outer = outer;
    if (!(std::isfinite(f) && std::isfinite(gg))) { res.status = SRP_ENOTSPD; return SRP_OK; }
    if (std::sqrt(std::max(gg, 0.0)) <= tol * std::fabs(f)) { res.status = SRP_OK; return SRP_OK; }
    if (outer == max_outer) { res.status = SRP_ENOCONV; return SRP_OK; }
    // truncated CG on the model  f + <grad, eta> + 1/2 <eta, Hess eta>, ||eta|| <= Delta
    SRP_TRY(lin(R.eta, 0.0, nullptr, 0.0, nullptr, nullptr));
    SRP_TRY(lin(R.Meta, 0.0, nullptr, 0.0, nullptr, nullptr));
    SRP_TRY(lin(R.Beta, 0.0, nullptr, 0.0, nullptr, nullptr));
    SRP_TRY(lin(R.Ceta, 0.0, nullptr, 0.0, nullptr, nullptr));
    SRP_TRY(lin(R.MHeta, 0.0, nullptr, 0.0, nullptr, nullptr));
    SRP_TRY(lin(R.r, 1.0, R.grad, 0.0, nullptr, nullptr));
    SRP_TRY(lin(R.Mr, 1.0, R.Mg, 0.0, nullptr, nullptr));
    SRP_TRY(lin(R.dl, -1.0, R.grad, 0.0, nullptr, nullptr));
    SRP_TRY(lin(R.Mdl, -1.0, R.Mg, 0.0, nullptr, nullptr));
    double rr = gg, ee = 0.0, ed = 0.0, dd = gg;
    const double r0 = std::sqrt(gg);
    bool boundary = false;
    for (int j = 0; j < max_inner; ++j) {
      ++res.inner;
      SRP_TRY(pass(R.dl, R.Bd, R.Cd));
      // h = -Cd N - Bd S_g ; Hd = Pi(M^-1 h) ; M Hd = h - BZ S_h
      SRP_TRY(lin(R.tmp, 0.0, nullptr, 1.0, R.Cd, Nm2));
      SRP_TRY(lin(R.h, -1.0, R.tmp, -1.0, R.Bd, R.Sg));
      SRP_TRY(minv(R.h, R.wh));
      SRP_TRY(gram(R.BZ, R.wh, R.Ch));
      {
        RtrSylvArgs sa{};
        sa.k = k;
        for (int b = 0; b < nb; ++b) { sa.Q[b] = R.Q[b]; sa.lam[b] = R.lam[b]; sa.C[b] = R.Ch[b]; sa.S[b] = R.Sh[b]; }
        SRP_TRY(rtr_sylv(sa, nb, st));
      }
      SRP_TRY(lin(R.Hd, 1.0, R.wh, -1.0, R.MiK, R.Sh));
      SRP_TRY(lin(R.MHd, 1.0, R.h, -1.0, R.BZ, R.Sh));
      SRP_TRY(dots(1, R.dl, R.MHd, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr));
      const double kappa = R.hdots[0];
      const double alpha = rr / kappa;
      double step = alpha;
      bool stop_boundary = false;
      if (!(kappa > 0.0) || ee + 2.0 * alpha * ed + alpha * alpha * dd >= Delta * Delta) {
        // to the boundary: the positive root of ee + 2 t ed + t^2 dd = Delta^2
        step = (-ed + std::sqrt(std::max(0.0, ed * ed + dd * (Delta * Delta - ee)))) / dd;
        stop_boundary = true;
      }
      SRP_TRY(lin(R.eta, 1.0, R.eta, step, R.dl, nullptr));
      SRP_TRY(lin(R.Meta, 1.0, R.Meta, step, R.Mdl, nullptr));
      SRP_TRY(lin(R.Beta, 1.0, R.Beta, step, R.Bd, nullptr));
      SRP_TRY(lin(R.Ceta, 1.0, R.Ceta, step, R.Cd, nullptr));
      SRP_TRY(lin(R.MHeta, 1.0, R.MHeta, step, R.MHd, nullptr));
      if (stop_boundary) { boundary = true; break; }
      SRP_TRY(lin(R.r, 1.0, R.r, alpha, R.Hd, nullptr));
      SRP_TRY(lin(R.Mr, 1.0, R.Mr, alpha, R.MHd, nullptr));
      SRP_TRY(dots(4, R.r, R.Mr, R.eta, R.Meta, R.eta, R.Mr, R.r, R.Mdl));
      const double rr_new = R.hdots[0], ee_new = R.hdots[1], er = R.hdots[2], rd_old = R.hdots[3];
      if (std::sqrt(std::max(rr_new, 0.0)) <= r0 * std::min(r0, 0.1)) break;   // theta = 1, kappa = 0.1
      const double beta = rr_new / rr;
      const double ed_old = ed + alpha * dd;   // <eta_new, d_old>
      ed = -er + beta * ed_old;
      dd = rr_new - 2.0 * beta * rd_old + beta * beta * dd;
      ee = ee_new;
      rr = rr_new;
      SRP_TRY(lin(R.dl, -1.0, R.r, beta, R.dl, nullptr));
      SRP_TRY(lin(R.Mdl, -1.0, R.Mr, beta, R.Mdl, nullptr));
    }
    // model decrease and the trial point
    SRP_TRY(dots(2, R.eta, R.Mg, R.eta, R.MHeta, nullptr, nullptr, nullptr, nullptr));
    const double mdec = -(R.hdots[0] + 0.5 * R.hdots[1]);
    // Gram of Z + eta from the carried products, the current Z^T B Z
    // included (not taken as I), so rounding in the constraint does not
    // accumulate over accepted steps
    SRP_TRY(lin(R.tmp, 0.5, B.U, 1.0, R.eta, nullptr));
    SRP_TRY(gram(R.BZ, R.tmp, R.E));
    SRP_TRY(gram(R.eta, R.Beta, R.F));
    {
      SkinnyProb pr[4];
      pr[0] = SkinnyProb{k, d[0], k, B.U[0], k, true, B.Kc[0], k, R.X0[0], k};
      pr[1] = SkinnyProb{k, d[0], k, B.U[0], k, true, R.Ceta[0], k, R.X0[1], k};
      pr[2] = SkinnyProb{k, d[0], k, R.eta[0], k, true, B.Kc[0], k, R.X0[2], k};
      pr[3] = SkinnyProb{k, d[0], k, R.eta[0], k, true, R.Ceta[0], k, R.X0[3], k};
      SRP_TRY(gemm_skinny_batch(4, pr, B.skw, B.skw_bytes, st));
    }
    {
      RtrTrialArgs ta{};
      ta.k = k; ta.nb = nb; ta.mu = B.mu; ta.cost_scale = cs; ta.out = R.dots;
      for (int b = 0; b < nb; ++b) { ta.E[b] = R.E[b]; ta.F[b] = R.F[b]; ta.Lit[b] = R.Lit[b]; }
      for (int q = 0; q < 4; ++q) ta.X0[q] = R.X0[q];
      SRP_TRY(rtr_trial(ta, st));
      SRP_HIP(hipMemcpyAsync(R.hdots, R.dots, sizeof(double) * 2, hipMemcpyDeviceToHost, st));
      SRP_HIP(hipStreamSynchronize(st));
    }
    const double fplus = R.hdots[0];
    const bool breakdown = R.hdots[1] != 0.0;
    // near the solution both decreases fall to the rounding level of f: a
    // shift of a few hundred ulps of |f| on both makes the ratio tend to 1
    // there instead of to noise (the regularised ratio of Absil, Baker and
    // Gallivan's trust-region code)
    const double reg = 1e3 * 2.220446049250313e-16 * std::max(1.0, std::fabs(f));
    const double rho = breakdown ? -1.0 : (f - fplus + reg) / (mdec + reg);
    if (rho < 0.25) Delta *= 0.25;
    else if (rho > 0.75 && boundary) Delta = std::min(2.0 * Delta, Dbar);
    if (rho > rho_prime && !breakdown) {
      // accept: Z <- (Z + eta) L^-T; Ks <- (Ks + B eta - lam eta) L^-T;
      // Kc_b <- (Kc_b + Ceta_b) L_o^-T (o: the other block; FDA: itself)
      SRP_TRY(lin(R.tmp, 1.0, B.U, 1.0, R.eta, nullptr));
      SRP_TRY(lin(B.U, 0.0, nullptr, 1.0, R.tmp, R.Lit));
      for (int b = 0; b < nb; ++b) {
        RtrLinArgs la{};
        la.k = k;
        la.side[0] = RtrLinSide{R.tmp[b], B.Ks[b], 1.0, R.Beta[b], 1.0, nullptr, d[b]};
        SRP_TRY(rtr_lin(la, 1, st));
        la.side[0] = RtrLinSide{R.tmp[b], R.tmp[b], 1.0, R.eta[b], -P.lam[b], nullptr, d[b]};
        SRP_TRY(rtr_lin(la, 1, st));
      }
      SRP_TRY(lin(B.Ks, 0.0, nullptr, 1.0, R.tmp, R.Lit));
      SRP_TRY(lin(R.tmp, 1.0, B.Kc, 1.0, R.Ceta, nullptr));
      double* Lo[2] = {R.Lit[nb == 2 ? 1 : 0], R.Lit[0]};
      SRP_TRY(lin(B.Kc, 0.0, nullptr, 1.0, R.tmp, Lo));
      ++accepted;
      if (refresh_every > 0 && accepted % refresh_every == 0) {   // products from the data again
        SRP_TRY(pass(B.U, R.Bd, B.Kc));
        for (int b = 0; b < nb; ++b) {
          RtrLinArgs la{};
          la.k = k;
          la.side[0] = RtrLinSide{B.Ks[b], R.Bd[b], 1.0, B.U[b], -P.lam[b], nullptr, d[b]};
          SRP_TRY(rtr_lin(la, 1, st));
        }
      }
    }
  }
  return SRP_OK;
}

// --------------------------------------------------------- CCA / FDA
struct CommonArgs {
  int k;
  double tol;
  srp_options opt;
};

static int sketch_any(int kind, const void* A, int dtype, int64_t n, int d, int s, uint64_t seed, void* out,
                      Arena& ar, hipStream_t st, const SrhtPlan* plan = nullptr) {
  Arena sub{ar.base + ar.used, ar.cap - ar.used, 0};
  if (kind == SRP_SRHT) {
    if (plan) return srht_apply_run(*plan, A, dtype, d, out, sub, st);
    return srht_run(A, dtype, n, d, s, seed, out, sub, st);
  }
  return countsketch_run(A, dtype, n, d, s, seed, out, sub, st);
}

static size_t sketch_ws(int kind, int64_t n, int d, int s, int dtype) {
  return kind == SRP_SRHT ? srht_ws_bytes(n, d, s, dtype) : countsketch_ws_bytes(n, s);
}

// ------------------------------------------------------- warm start
// The exact solution of the sketched problem: Algorithms CCAopt and LDAopt
// start from exact-cca(SX, SY) / exact-fda(SX) (sketch-and-solve), then
// qf_B of it.  M_b = (S A_b)^T (S A_b) + lam_b I and M_b^-1 are at hand.
struct WarmStart {
  int kind = 0;                  // 0: none (Gaussian start), 1: CCA, 2: FDA, 3: CCA with a Woodbury block
  int iters = 0;                 // CCA: block subspace iterations
  const double* Hxy = nullptr;   // CCA: (S X)^T (S Y), dx x dy
  const double* Rinv[2] = {nullptr, nullptr};   // CCA: R_x^-1, R_y^-1 (upper)
  const double* Yhat = nullptr;  // FDA: c x d between-class factor
  int c = 0;
  const void* SA[2] = {nullptr, nullptr};   // CCA with a Woodbury block: the sketches S X, S Y
  bool sa_f32 = false;
  int s = 0;
  char* ws = nullptr;            // scratch (warm_ws_bytes)
  size_t ws_bytes = 0;
};

// Block width of the CCA subspace iteration: 32 columns for k <= 12, else
// 64 (the spectrum of the sketched problem is flat past its leading
// correlations, so a block a few times k wide converges in a few products;
// the Rayleigh-Ritz eigensolve and the Cholesky-QR cost grow with the
// block's square and cube), at most min(dx, dy).
static int warm_block(int dx, int dy, int k) { return std::max(k, std::min(k <= 12 ? 32 : 64, std::min(dx, dy))); }
// Subspace iterations per product: the block is multiplied by (C^T C)^4.
constexpr int kWarmPower = 4;

static int warm_cca_iters(int dx, int dy, int k, int iters) {
  if (warm_block(dx, dy, k) == std::min(dx, dy)) return 1;   // the block spans C^T C's range
  return (std::max(1, iters) + kWarmPower - 1) / kWarmPower * kWarmPower;
}

// Most contraction splits of the dense warm-start products (their partials
// take this many d x d blocks of the workspace).
constexpr int kWarmSplit = 4;

// C = op(A)... : out (m x n) = A^T B for A kk x m, B kk x n (FP64), split
// over the contraction into `parts` (the big-tile GEMM), summed in order:
// enough splits for about 256 workgroups of 128 x 128 tiles, each at least
// 256 rows of the contraction (at d = 1000: 64 tiles, 4 splits).
static int gemm_atb(int m, int n, int kk, const double* A, int64_t lda, const double* Bm, int64_t ldb, double* out,
                    double* parts, size_t parts_bytes, hipStream_t st) {
  const int64_t cnt = (int64_t)m * n;
  const int64_t tiles = (int64_t)((m + 127) / 128) * ((n + 127) / 128);
  int64_t ks = std::min<int64_t>((256 + tiles - 1) / tiles, std::max(1, kk / 256));
  ks = std::min<int64_t>(ks, (int64_t)(parts_bytes / bytes_of<double>((size_t)cnt)));
  const int nsplit = (int)std::max<int64_t>(1, ks);
  GemmArgs g{};
  g.m = m; g.n = n; g.kk = kk; g.alpha = 1.0; g.beta = 0.0;
  g.A = A; g.lda = lda; g.ta = true; g.a_f32 = false;
  g.B = Bm; g.ldb = ldb; g.tb = false; g.b_f32 = false;
  if (nsplit == 1) {
    g.C = out; g.ldc = n;
    return gemm_f64(g, st);
  }
  g.C = parts; g.ldc = n; g.ksplit = nsplit; g.c_split_stride = cnt;
  SRP_TRY(gemm_f64(g, st));
  return sum_parts_f64(parts, nsplit, cnt, cnt, out, 0, 0.0, st);
}

static size_t warm_ws_bytes(int nb, int k, const int* d, int c) {
  if (nb == 2) {
    const int dx = d[0], dy = d[1], q = warm_block(dx, dy, k), dm = std::max(dx, dy);
    const size_t dense = (3 + kWarmSplit) * bytes_of<double>((size_t)dm * dm);  // E, B1, B2, parts
    return dense + bytes_of<double>((size_t)(3 * dy + 2 * dx) * q + 64 * 64 + q * q + q * k + 64) +
           bytes_of<int>(4) + skinny_ws_bytes(dm, dm, q) + 16 * 256;
  }
  const int dd = d[0];
  return bytes_of<double>((size_t)2 * dd * c + c * c + c * k + 64) + bytes_of<int>(4) +
         skinny_ws_bytes(std::max(dd, c), dd, c) + 8 * 256;
}

// CCA.  The sketched correlations are the singular values of
// C = R_x^-T H_xy R_y^-1 (H_xy = (SX)^T (SY), R^T R = M), and the
// sketched weights are U = R_x^-1 P_k, V = R_y^-1 W_k for the singular
// pairs (P, W) of C.  The dense FP64 products are all of the A^T B form
// of the big-tile GEMM:
//   E = (R_x^-1)^T H_xy,  F = E^T E,  K^T = F^T R_y^-1,  S = (R_y^-1)^T K^T
// so S = C^T C (symmetric, eigenvalues sigma^2), then S^2 and S^4 by
// squaring.  Block subspace iteration W <- qf(S^4 W) (Cholesky-QR) then
// advances four iterations per product.  Rayleigh-Ritz on the block: with
// V = R_y^-1 W and P = E V = C W, the q x q matrix P^T P = W^T S W has
// eigenvectors Q, and V Q_k, R_x^-1 P Q_k are the right and left weights
// (up to positive column scales, which the qf start point removes).
static int warm_cca(const RcgProblem& P, const WarmStart& w, double* const* out, int* flag, uint64_t seed,
                    const double* Rix, const double* Riy, hipStream_t st) {
  const int dx = P.d[0], dy = P.d[1], k = P.k, q = warm_block(dx, dy, k), dm = std::max(dx, dy);
  const int ldq = cholqr_block(q);
  Arena a{w.ws, w.ws_bytes, 0};
  double* E = a.take<double>((size_t)dm * dm);
  double* B1 = a.take<double>((size_t)dm * dm);
  double* B2 = a.take<double>((size_t)dm * dm);
  const size_t parts_bytes = kWarmSplit * bytes_of<double>((size_t)dm * dm);
  double* parts = (double*)a.take<char>(parts_bytes);
  double* W = a.take<double>((size_t)dy * q);
  double* Wn = a.take<double>((size_t)dy * q);
  double* V = a.take<double>((size_t)dy * q);
  double* Pm = a.take<double>((size_t)dx * q);
  double* PQ = a.take<double>((size_t)dx * q);
  double* G = a.take<double>((size_t)q * q);
  double* Bm = a.take<double>((size_t)64 * 64);
  double* Q = a.take<double>((size_t)q * k);
  double* ev = a.take<double>(64);
  const size_t skb = skinny_ws_bytes(dm, dm, q);
  double* skw = (double*)a.take<char>(skb);
  if (!skw) { set_error("warm start: workspace too small"); return SRP_ENOMEM; }
  auto mm = [&](int m, int kk, int nc, const double* A, int64_t lda, bool ta, const double* Bp, int64_t ldb,
                double* C) { return gemm_skinny_f64(m, kk, nc, A, lda, ta, Bp, ldb, C, nc, skw, skb, st); };
  // dense products
  SRP_TRY(gemm_atb(dx, dy, dx, Rix, dx, w.Hxy, dy, E, parts, parts_bytes, st));    // R_x^-T H_xy
  SRP_TRY(gemm_atb(dy, dy, dx, E, dy, E, dy, B1, parts, parts_bytes, st));         // F = E^T E
  SRP_TRY(gemm_atb(dy, dy, dy, B1, dy, Riy, dy, B2, parts, parts_bytes, st));      // K^T = F R_y^-1
  SRP_TRY(gemm_atb(dy, dy, dy, Riy, dy, B2, dy, B1, parts, parts_bytes, st));      // S = R_y^-T K^T
  const int iters = warm_cca_iters(dx, dy, k, w.iters);
  const double* Sp = B1;
  if (iters >= kWarmPower) {
    SRP_TRY(gemm_atb(dy, dy, dy, B1, dy, B1, dy, B2, parts, parts_bytes, st));     // S^2
    SRP_TRY(gemm_atb(dy, dy, dy, B2, dy, B2, dy, B1, parts, parts_bytes, st));     // S^4
  }
  const int steps = iters >= kWarmPower ? iters / kWarmPower : iters;
  // W = qf(G0) for a seeded Gaussian G0, then W <- qf(S^p W)
  SRP_TRY(launch_gauss_fill(Wn, (int64_t)dy * q, seed ^ 0x5741524D53544152ull, st));
  for (int it = 0; it <= steps; ++it) {
    if (it > 0) SRP_TRY(mm(dy, dy, q, Sp, dy, false, W, q, Wn));
    SRP_TRY(mm(q, dy, q, Wn, q, true, Wn, q, G));
    SRP_TRY(launch_cholqr_factor(G, q, Bm, flag, st));
    SRP_TRY(gemm_skinny_f64(dy, q, q, Wn, q, false, Bm, ldq, W, q, skw, skb, st));
  }
  // Rayleigh-Ritz on the block
  SRP_TRY(mm(dy, dy, q, Riy, dy, false, W, q, V));       // V = R_y^-1 W
  SRP_TRY(mm(dx, dy, q, E, dy, false, V, q, Pm));        // P = E V = C W
  SRP_TRY(mm(q, dx, q, Pm, q, true, Pm, q, G));          // P^T P = W^T S W
  SRP_TRY(launch_rr_eig(G, q, k, Q, ev, st));
  SRP_TRY(gemm_skinny_f64(dx, q, k, Pm, q, false, Q, k, PQ, k, skw, skb, st));
  SRP_TRY(gemm_skinny_f64(dx, dx, k, Rix, dx, false, PQ, k, out[0], k, skw, skb, st));
  SRP_TRY(gemm_skinny_f64(dy, q, k, V, q, false, Q, k, out[1], k, skw, skb, st));
  return SRP_OK;
}

// CCA when a block's metric is in Woodbury form (no R^-1 to whiten with).
// The sketched weights solve H v = sigma M_x u, H^T u = sigma M_y v for
// H = (S X)^T (S Y), so v is an eigenvector of A = M_y^-1 H^T M_x^-1 H,
// which is self-adjoint in the M_y inner product.  Block subspace
// iteration V <- qf_My(A V) (H and H^T applied as two skinny products
// through the s x q middle, M^-1 by minv_apply), then Rayleigh-Ritz:
// with U = M_x^-1 H V, V^T M_y A V = (H V)^T U (q x q), whose top
// eigenvectors Q give V Q and U Q (U Q = M_x^-1 H V Q: the left weights up
// to positive column scales, which the qf start removes).
static int warm_cca_pencil(const RcgProblem& P, const WarmStart& w, double* const* out, int* flag, uint64_t seed,
                           hipStream_t st) {
  const int dx = P.d[0], dy = P.d[1], k = P.k, s = w.s, q = warm_block(dx, dy, k), dm = std::max(dx, dy);
  const int ldq = cholqr_block(q);
  Arena a{w.ws, w.ws_bytes, 0};
  double* V = a.take<double>((size_t)dy * q);
  double* Vn = a.take<double>((size_t)dy * q);
  double* Z = a.take<double>((size_t)dy * q);
  double* U = a.take<double>((size_t)dx * q);
  double* H = a.take<double>((size_t)dx * q);
  double* T = a.take<double>((size_t)s * q);
  double* G = a.take<double>((size_t)q * q);
  double* G2 = a.take<double>((size_t)q * q);
  double* Bm = a.take<double>((size_t)64 * 64);
  double* Q = a.take<double>((size_t)q * k);
  double* ev = a.take<double>(64);
  const size_t skb = std::max({skinny_ws_bytes(dm, dm, q), skinny_ws_bytes(s, dm, q), skinny_ws_bytes(dm, s, q),
                               skinny_ws_bytes(q, dm, q), skinny_ws_bytes(q, s, q)});
  double* skw = (double*)a.take<char>(skb);
  if (!skw) { set_error("warm start: workspace too small"); return SRP_ENOMEM; }
  const bool f32 = w.sa_f32;
  // C (m x nc) = op(A) B for a sketch A (FP32 or FP64)
  auto mmS = [&](int m, int kk, int nc, const void* A, int64_t lda, bool ta, const double* Bp, int64_t ldb,
                 double* C) {
    SkinnyProb pr{m, kk, nc, A, lda, ta, Bp, ldb, C, nc};
    pr.a_f32 = f32;
    return gemm_skinny_batch(1, &pr, skw, skb, st);
  };
  auto mm = [&](int m, int kk, int nc, const double* A, int64_t lda, bool ta, const double* Bp, int64_t ldb,
                double* C) { return gemm_skinny_f64(m, kk, nc, A, lda, ta, Bp, ldb, C, nc, skw, skb, st); };
  // Vout = qf_My(Vin): G = (S Y Vin)^T (S Y Vin) + lam_y Vin^T Vin, L^-T by Cholesky-QR
  auto qf_y = [&](const double* Vin, double* Vout) -> int {
    SRP_TRY(mmS(s, dy, q, w.SA[1], dy, false, Vin, q, T));
    SRP_TRY(mm(q, s, q, T, q, true, T, q, G));
    SRP_TRY(mm(q, dy, q, Vin, q, true, Vin, q, G2));
    RtrLinArgs la{};
    la.k = q;
    la.side[0] = RtrLinSide{G, G, 1.0, G2, P.lam[1], nullptr, q};
    SRP_TRY(rtr_lin(la, 1, st));
    SRP_TRY(launch_cholqr_factor(G, q, Bm, flag, st));
    return gemm_skinny_f64(dy, q, q, Vin, q, false, Bm, ldq, Vout, q, skw, skb, st);
  };
  // Hout = H V = (S X)^T (S Y V)
  auto apply_h = [&](const double* Vin, double* Hout) -> int {
    SRP_TRY(mmS(s, dy, q, w.SA[1], dy, false, Vin, q, T));
    return mmS(dx, s, q, w.SA[0], dx, true, T, q, Hout);
  };
  SRP_TRY(launch_gauss_fill(Vn, (int64_t)dy * q, seed ^ 0x5741524D53544152ull, st));
  SRP_TRY(qf_y(Vn, V));
  const int iters = std::max(1, w.iters);
  for (int it = 0; it < iters; ++it) {
    SRP_TRY(apply_h(V, H));
    SRP_TRY(minv_apply(P, 0, H, q, U, skw, skb, st));
    SRP_TRY(mmS(s, dx, q, w.SA[0], dx, false, U, q, T));       // S X U
    SRP_TRY(mmS(dy, s, q, w.SA[1], dy, true, T, q, Z));        // H^T U
    SRP_TRY(minv_apply(P, 1, Z, q, Vn, skw, skb, st));
    SRP_TRY(qf_y(Vn, V));
  }
  SRP_TRY(apply_h(V, H));
  SRP_TRY(minv_apply(P, 0, H, q, U, skw, skb, st));
  SRP_TRY(mm(q, dx, q, H, q, true, U, q, G));                  // (H V)^T M_x^-1 (H V)
  SRP_TRY(launch_rr_eig(G, q, k, Q, ev, st));
  SRP_TRY(gemm_skinny_f64(dx, q, k, U, q, false, Q, k, out[0], k, skw, skb, st));
  SRP_TRY(gemm_skinny_f64(dy, q, k, V, q, false, Q, k, out[1], k, skw, skb, st));
  return SRP_OK;
}

// FDA.  The sketched problem S_B w = rho M w with S_B = Yhat^T Yhat has its
// solutions in the range of M^-1 Yhat^T: w = M^-1 Yhat^T p with
// (Yhat M^-1 Yhat^T) p = rho p, a c x c eigenproblem.
static int warm_lda(const RcgProblem& P, const WarmStart& w, double* const* out, hipStream_t st) {
  const int d = P.d[0], k = P.k, c = w.c;
  Arena a{w.ws, w.ws_bytes, 0};
  double* Yt = a.take<double>((size_t)d * c);
  double* T = a.take<double>((size_t)d * c);
  double* K = a.take<double>((size_t)c * c);
  double* Q = a.take<double>((size_t)c * k);
  double* ev = a.take<double>(64);
  const size_t skb = skinny_ws_bytes(std::max(d, c), d, c);
  double* skw = (double*)a.take<char>(skb);
  if (!skw) { set_error("warm start: workspace too small"); return SRP_ENOMEM; }
  SRP_TRY(transpose_f64(w.Yhat, c, d, Yt, st));
  SRP_TRY(minv_apply(P, 0, Yt, c, T, skw, skb, st));                                  // M^-1 Yhat^T
  SRP_TRY(gemm_skinny_f64(c, d, c, w.Yhat, d, false, T, c, K, c, skw, skb, st));        // Yhat M^-1 Yhat^T
  SRP_TRY(launch_rr_eig(K, c, k, Q, ev, st));
  SRP_TRY(gemm_skinny_f64(d, c, k, T, c, false, Q, k, out[0], k, skw, skb, st));
  return SRP_OK;
}

// The trust-region tail: qf_B of the start point (a data pass, step t = 1),
// trust-region iterations to tol, then the finish of the CG tail (FP64
// Rayleigh-Ritz rotation and sign convention from a pass along the point).
static int rtr_tail(RcgProblem& full, RcgBuffers& B, const CommonArgs& ca, double* const* start,
                    double* const* outW, double* sigma_out, srp_info* info, double ms_warm, int warm_iters,
                    PhaseTimer& tm, hipStream_t st) {
  const int k = full.k, nb = full.nb;
  RcgResult r0;
  SRP_TRY(rcg_run(full, B, start, 0, ca.tol, 1, 0, false, false, nullptr, r0, st));
  if (r0.status == SRP_ENOTSPD) return SRP_ENOTSPD;
  RtrState R{};
  Arena a{B.rtr_ws, B.rtr_ws_bytes, 0};
  SRP_TRY(rtr_take(R, a, nb, k, full.d));
  SRP_HIP(hipHostMalloc((void**)&R.hdots, 16 * sizeof(double), hipHostMallocDefault));
  struct Pinned { double* p; ~Pinned() { if (p) (void)hipHostFree(p); } } pin{R.hdots};
  double mu_h[KMAX];
  for (int i = 0; i < k; ++i) mu_h[i] = ca.opt.mu ? ca.opt.mu[i] : (double)(k - i);
  RtrResult rr;
  SRP_TRY(rtr_run(full, B, R, mu_h, ca.opt.max_iter, std::max(1, ca.opt.rtr_max_inner), ca.tol, ca.opt.refresh_every,
                  rr, st));
  for (int s = 0; s < nb; ++s) SRP_TRY(copy_f64(outW[s], B.U[s], (int64_t)full.d[s] * k, st));
  RcgResult rf;
  const bool f64_finish = ca.opt.final_f64 != 0;
  SRP_TRY(rcg_run(full, B, outW, 0, ca.tol, 1, 0, true, f64_finish, sigma_out, rf, st));
  for (int s = 0; s < nb; ++s) SRP_TRY(copy_f64(outW[s], B.U[s], (int64_t)full.d[s] * k, st));
  const double ms_iter = tm.lap_ms();
  int status = rr.status;
  if (rf.status == SRP_ENOTSPD) status = SRP_ENOTSPD;
  if (info) {
    info->status = status;
    info->iterations = rr.outer;
    info->inner_iterations = rr.inner;
    info->warm_iterations = warm_iters;
    info->passes = rr.passes + r0.passes + rf.passes;
    info->f = rf.f;
    info->grad_norm = rr.gg > 0 ? std::sqrt(rr.gg) : 0.0;
    info->ms_warm = ms_warm;
    info->ms_iterate = ms_iter;
  }
  return status;
}

// Shared tail of both solvers once the data, sketches and metric exist.
static int solve_tail(RcgProblem& full, const WarmStart& warm, RcgBuffers& B, const CommonArgs& ca,
                      double* const* outW, double* sigma_out, srp_info* info, PhaseTimer& tm, hipStream_t st) {
  const int k = full.k, nb = full.nb;
  // start point: the exact solution of the sketched problem, or (no warm
  // start, or its block factor broke down) a seeded Gaussian matrix; the
  // iteration begins at qf_B of it
  double* start[2] = {outW[0], nb == 2 ? outW[1] : nullptr};
  int warm_iters = 0;
  bool gauss = warm.kind == 0;
  if (!gauss) {
    int* wflag = B.ran_all;   // not yet in use: cleared before the timed passes
    SRP_TRY(fill_i32(wflag, 1, 0, st));
    if (warm.kind == 1) {
      SRP_TRY(warm_cca(full, warm, outW, wflag, ca.opt.seed, warm.Rinv[0], warm.Rinv[1], st));
      warm_iters = warm_cca_iters(full.d[0], full.d[1], k, warm.iters);
    } else if (warm.kind == 3) {
      SRP_TRY(warm_cca_pencil(full, warm, outW, wflag, ca.opt.seed, st));
      warm_iters = std::max(1, warm.iters);
    } else {
      SRP_TRY(warm_lda(full, warm, outW, st));
      warm_iters = 1;
    }
    int hflag = 0;
    SRP_HIP(hipMemcpyAsync(&hflag, wflag, sizeof(int), hipMemcpyDeviceToHost, st));
    SRP_HIP(hipStreamSynchronize(st));
    if (hflag) {   // a singular sketched block (e.g. zero cross-covariance): Gaussian start
      gauss = true;
      warm_iters = 0;
    }
  }
  if (gauss)
    for (int s = 0; s < nb; ++s)
      SRP_TRY(launch_gauss_fill(start[s], (int64_t)full.d[s] * k, ca.opt.seed ^ (0x5741524D53544152ull + s), st));
  const double ms_warm = tm.lap_ms();
  if (ca.opt.time_passes) SRP_TRY(fill_i32(B.ran_all, 2, 0, st));
  // low-precision phase (CCA): BF16 data, BF16 matrix-core passes
  int lowp_iters = 0, lowp_status = SRP_OK;
  double ms_lowp = 0.0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> lowp_events;
  if (ca.opt.lowp_x && full.nb == 2) {
    if (start[0] != outW[0]) {   // keep the phase's start point (Z is scratch of rcg_run)
      for (int s = 0; s < nb; ++s) SRP_TRY(copy_f64(outW[s], start[s], (int64_t)full.d[s] * k, st));
      start[0] = outW[0];
      start[1] = outW[1];
    }
    B.time_passes = ca.opt.time_passes != 0;
    B.events = &lowp_events;
    B.ran = B.ran_all + 1;
    RcgProblem lp = full;
    lp.A[0] = ca.opt.lowp_x;
    lp.A[1] = ca.opt.lowp_y;
    lp.dtype = SRP_BF16;
    lp.compute = SRP_BF16;
    RcgResult rl;
    SRP_TRY(rcg_run(lp, B, start, std::max(1, ca.opt.lowp_max_iter), ca.opt.lowp_tol,
                    std::max(1, ca.opt.check_every), ca.opt.refresh_every, false, false, nullptr, rl, st));
    B.time_passes = false;
    B.events = nullptr;
    B.ran = nullptr;
    lowp_status = rl.status;
    // A retraction Gram from BF16 products can lose definiteness when the
    // data's columns span many decades (the products' rounding is relative
    // to |A|^T |A W|, not to the Gram).  The phase only accelerates: on a
    // breakdown the iteration continues on the main data from the point the
    // phase started at (still in outW).
    if (rl.status != SRP_ENOTSPD) {
      for (int s = 0; s < nb; ++s) SRP_TRY(copy_f64(outW[s], B.U[s], (int64_t)full.d[s] * k, st));
      start[0] = outW[0];
      start[1] = outW[1];
    }
    lowp_iters = rl.iterations;
    ms_lowp = tm.lap_ms();
  }
  if (ca.opt.method == SRP_RTR) return rtr_tail(full, B, ca, start, outW, sigma_out, info, ms_warm, warm_iters,
                                                 tm, st);
  RcgResult r;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  B.time_passes = ca.opt.time_passes != 0;
  B.events = &events;
  B.ran = B.ran_all;
  // final_f64 > 0 with lower-precision passes: close with that many
  // iterations whose data products run in FP64 arithmetic, from the point
  // the FP32 (or BF16) iteration reached; the finishing pass is FP64 too.
  // final_f64 < 0: only the finishing pass runs in FP64.
  const bool refine = ca.opt.final_f64 > 0 && full.compute != SRP_F64;
  SRP_TRY(rcg_run(full, B, start, ca.opt.max_iter, ca.tol, std::max(1, ca.opt.check_every),
                  ca.opt.refresh_every, !refine, ca.opt.final_f64 != 0, sigma_out, r, st));
  for (int s = 0; s < nb; ++s) SRP_TRY(copy_f64(outW[s], B.U[s], (int64_t)full.d[s] * k, st));
  if (refine && r.status != SRP_ENOTSPD) {
    RcgProblem f64 = full;
    f64.compute = SRP_F64;
    double* rstart[2] = {outW[0], nb == 2 ? outW[1] : nullptr};
    RcgResult r2;
    SRP_TRY(rcg_run(f64, B, rstart, ca.opt.final_f64, ca.tol, std::max(1, ca.opt.check_every),
                    ca.opt.refresh_every, true, true, sigma_out, r2, st));
    for (int s = 0; s < nb; ++s) SRP_TRY(copy_f64(outW[s], B.U[s], (int64_t)full.d[s] * k, st));
    r.iterations += r2.iterations;
    r.passes += r2.passes;
    r.f = r2.f;
    r.gg = r2.gg;
    // the closing phase has a fixed budget: reaching it is not a failure
    if (r2.status == SRP_ENOTSPD) r.status = SRP_ENOTSPD;
  }
  const double ms_iter = tm.lap_ms() + ms_lowp;
  double pass_ms = 0.0;
  for (auto& e : events) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e.first, e.second) == hipSuccess) pass_ms += ms;
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  B.time_passes = false;
  B.events = nullptr;
  B.ran = nullptr;
  int ran_h[2] = {0, 0};
  if (ca.opt.time_passes) {
    SRP_HIP(hipMemcpyAsync(ran_h, B.ran_all, sizeof(ran_h), hipMemcpyDeviceToHost, st));
    SRP_HIP(hipStreamSynchronize(st));
  }
  double lowp_pass_ms = 0.0;
  for (auto& e : lowp_events) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e.first, e.second) == hipSuccess) lowp_pass_ms += ms;
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  if (info) {
    info->lowp_pass_ms = lowp_pass_ms;
    info->lowp_pass_launches = ran_h[1];
    info->pass_ms = pass_ms;
    info->pass_launches = ran_h[0];
    info->status = r.status;
    info->iterations = r.iterations;
    info->warm_iterations = warm_iters;
    info->passes = r.passes;
    info->f = r.f;
    info->grad_norm = r.gg > 0 ? std::sqrt(r.gg) : 0.0;
    info->ms_warm = ms_warm;
    info->ms_iterate = ms_iter;
    info->lowp_iterations = lowp_iters;
    info->lowp_status = lowp_status;
    info->ms_lowp = ms_lowp;
  }
  return r.status;
}

static int check_options(const srp_options& o) {
  SRP_REQUIRE(o.sketch == SRP_COUNTSKETCH || o.sketch == SRP_SRHT, "unknown sketch kind %d", o.sketch);
  SRP_REQUIRE(o.max_iter >= 0 && o.warm_start_iters >= 0 && o.refresh_every >= 0, "negative iteration option");
  SRP_REQUIRE(o.pass_compute == SRP_F64 || o.pass_compute == SRP_F32 || o.pass_compute == -1,
              "pass_compute must be SRP_F64 or SRP_F32");
  SRP_REQUIRE(o.method == SRP_RCG || o.method == SRP_RTR, "unknown method %d", o.method);
  SRP_REQUIRE(o.method == SRP_RCG || o.lowp_x == nullptr, "the trust-region method has no BF16 phase");
  return SRP_OK;
}

static int setup_mu(const srp_options& o, int k, double* mu_dev, hipStream_t st) {
  double mu[KMAX];
  for (int i = 0; i < k; ++i) mu[i] = o.mu ? o.mu[i] : (double)(k - i);
  // Equal weights (N = I) give the unweighted trace cost: the top-k subspace
  // is its critical set and the closing Rayleigh-Ritz rotation orders it.
  for (int i = 0; i < k; ++i)
    SRP_REQUIRE(mu[i] > 0.0 && (i == 0 || mu[i] <= mu[i - 1]), "mu must be positive and non-increasing");
  SRP_HIP(hipMemcpyAsync(mu_dev, mu, sizeof(double) * k, hipMemcpyHostToDevice, st));
  SRP_HIP(hipStreamSynchronize(st));
  return SRP_OK;
}

// Scratch of one CCA view's sketch and factor.  Both views get the larger
// of the two needs: the factor's split-K partials do not grow monotonically
// with d (fewer upper tiles take a deeper split).
static size_t cca_view_scratch(int64_t n, int dx, int dy, int k, int s, int dtype, int sketch_kind) {
  const int dd[2] = {dx, dy};
  size_t m = std::max({sketch_ws(sketch_kind, n, dx, s, dtype), sketch_ws(sketch_kind, n, dy, s, dtype),
                       factor_ws_bytes(s, dx), factor_ws_bytes(s, dy), warm_ws_bytes(2, k, dd, 0)});
  for (int d : dd)
    if (s < d) m = std::max(m, woodbury_factor_scratch(s, d));
  return m;
}

size_t cca_ws_bytes(int64_t n, int dx, int dy, int k, int s, int dtype, int sketch_kind, int skin_dtype) {
  const int sk_dtype = skin_dtype == SRP_F64 ? SRP_F64 : SRP_F32;
  const size_t ssz = dtype_size(sk_dtype);
  const int dd[2] = {dx, dy};
  size_t bytes = 0;
  bytes += 2 * (((size_t)s * std::max(dx, dy) * ssz + 255) & ~size_t(255));  // SX, SY
  bytes += 2 * bytes_of<double>((size_t)dx * dx) + 2 * bytes_of<double>((size_t)dy * dy);  // R, Minv (x) ...
  bytes += 2 * bytes_of<double>((size_t)std::max(dx, dy) * std::max(dx, dy));
  bytes += bytes_of<int>(4);
  bytes += bytes_of<double>((size_t)dx * dy);   // cross Gram of the sketches
  if (sketch_kind == SRP_SRHT) bytes += srht_plan_bytes(n, s) + 1024;   // shared sampled rows
  const size_t scratch = cca_view_scratch(n, dx, dy, k, s, dtype, sketch_kind);
  bytes += rcg_buffers_bytes(2, k, std::max<int64_t>(n, s), dd, dtype);
  bytes += 2 * ((scratch + 255) & ~size_t(255)) + 4096;   // one scratch per view (the views run concurrently)
  for (int d : dd)
    if (s < d) bytes += woodbury_keep_bytes(s, d);
  return bytes;
}

size_t lda_ws_bytes(int64_t n, int d, int c, int k, int s, int dtype, int sketch_kind) {
  const int sk_dtype = dtype == SRP_F64 ? SRP_F64 : SRP_F32;
  const size_t esz = dtype_size(dtype), ssz = dtype_size(sk_dtype);
  const int dd[2] = {d, 0};
  size_t bytes = 0;
  bytes += (((size_t)n * d * esz + 255) & ~size_t(255));          // Xhat
  bytes += (((size_t)s * d * ssz + 255) & ~size_t(255));          // sketch
  bytes += 3 * bytes_of<double>((size_t)d * d);                    // R, Rinv, Minv
  bytes += bytes_of<double>((size_t)c * d) + bytes_of<int>(c) + bytes_of<int>(4);
  size_t scratch = std::max({sketch_ws(sketch_kind, n, d, s, dtype), factor_ws_bytes(s, d),
                             lda_center_ws_bytes(n, d, c), warm_ws_bytes(1, k, dd, c)});
  if (s < d) scratch = std::max(scratch, woodbury_factor_scratch(s, d)) + woodbury_keep_bytes(s, d);
  bytes += rcg_buffers_bytes(1, k, std::max<int64_t>(n, s), dd, dtype, c);
  bytes += scratch + 4096;
  return bytes;
}

// The solve's workspace: the context's buffer when it has one (it must be
// large enough), else a stream-ordered allocation released on return.
static int take_workspace(Workspace& W, size_t bytes, const SolveCtx* ctx, hipStream_t st, void** base) {
  if (ctx && ctx->ws) {
    SRP_REQUIRE(ctx->ws_bytes >= bytes, "workspace of %zu bytes is smaller than the %zu needed", ctx->ws_bytes,
                bytes);
    *base = ctx->ws;
    return SRP_OK;
  }
  W.st = st;
  SRP_TRY(device_alloc(&W.base, bytes, st));
  *base = W.base;
  return SRP_OK;
}

int cca_solve_impl(const void* X, const void* Y, int64_t n, int dx, int dy, int k, double lx, double ly, int s,
                   double tol, int dtype, const srp_options* optp, hipStream_t st, double* U, double* V,
                   double* sigma, srp_info* info, const SolveCtx* ctx) {
  clear_error();
  srp_options opt;
  srp_default_options(&opt);
  if (optp) opt = *optp;
  SRP_TRY(check_options(opt));
  SRP_REQUIRE(X && Y && U && V && sigma, "null pointer argument");
  SRP_REQUIRE(dtype == SRP_F64 || dtype == SRP_F32 || dtype == SRP_BF16, "bad dtype %d", dtype);
  SRP_REQUIRE(n >= 1 && n < (int64_t(1) << 31), "n out of range");
  SRP_REQUIRE(dx >= 1 && dy >= 1, "dx, dy must be positive");
  SRP_REQUIRE(k >= 1 && k <= std::min(dx, dy) && k <= 16, "need 1 <= k <= min(dx, dy), k <= 16");
  SRP_REQUIRE(lx >= 0.0 && ly >= 0.0, "lambda must be >= 0");
  SRP_REQUIRE(tol >= 0.0, "tol must be >= 0");
  // s < d: the view's metric in Woodbury form, which needs lambda > 0
  const bool wbx = s < dx, wby = s < dy;
  SRP_REQUIRE(s >= 1 && (!wbx || lx > 0.0) && (!wby || ly > 0.0),
              "sketch_size < d needs lambda > 0 for that view (the Woodbury form of M^-1)");
  int compute = opt.pass_compute == -1 ? (dtype == SRP_F64 ? SRP_F64 : SRP_F32) : opt.pass_compute;
  // FP64 arithmetic falls back to two GEMM reads of the data where the fused pass has no instance
  const bool f64_ok = opt.final_f64 == 0 || dtype != SRP_BF16;
  SRP_REQUIRE(f64_ok, "FP64 closing iterations need F32 or F64 data");
  SRP_REQUIRE(pass_limits_ok(dtype, compute, dx, dy, k, 2) || (compute == SRP_F64 && dtype != SRP_BF16),
              "unsupported shape for the data pass (dx+dy=%d)", dx + dy);
  const bool staged = opt.sketch_x != nullptr;
  if (staged) {
    SRP_REQUIRE(opt.sketch_y, "sketch_x and sketch_y go together");
    SRP_REQUIRE(opt.sketch_dtype == SRP_F32 || opt.sketch_dtype == SRP_BF16 || opt.sketch_dtype == SRP_FP8E4M3,
                "bad sketch_dtype %d", opt.sketch_dtype);
    SRP_REQUIRE(opt.sketch_dtype != SRP_FP8E4M3 || (opt.sketch_scale_x && opt.sketch_scale_y),
                "FP8 sketch input needs its column scales");
  }
  const void* skin_x = staged ? opt.sketch_x : X;
  const void* skin_y = staged ? opt.sketch_y : Y;
  const int skin_dtype = staged ? opt.sketch_dtype : dtype;
  const int sk_dtype = skin_dtype == SRP_F64 ? SRP_F64 : SRP_F32;
  SRP_REQUIRE(pass_limits_ok(sk_dtype, compute, dx, dy, k, 2) || compute == SRP_F64,
              "unsupported shape for the sketch pass");
  if (opt.lowp_x) {
    SRP_REQUIRE(opt.lowp_y, "lowp_x and lowp_y go together");
    SRP_REQUIRE(pass_limits_ok(SRP_BF16, SRP_BF16, dx, dy, k, 2), "unsupported shape for the BF16 pass");
  }
  if (opt.sketch == SRP_SRHT) {
    int64_t np = 2;
    while (np < n) np <<= 1;
    SRP_REQUIRE(np <= (int64_t(1) << 20) && s <= np, "SRHT needs s <= n' <= 2^20");
  }
  PhaseTimer tm(st);
  // workspace
  const size_t ssz = dtype_size(sk_dtype);
  const int dd[2] = {dx, dy};
  const size_t bytes = cca_ws_bytes(n, dx, dy, k, s, dtype, opt.sketch, skin_dtype);
  const size_t scratch = cca_view_scratch(n, dx, dy, k, s, dtype, opt.sketch);
  Workspace W;
  void* wbase = nullptr;
  SRP_TRY(take_workspace(W, bytes, ctx, st, &wbase));
  Arena ar{(char*)wbase, bytes, 0};
  void* SX = ar.take<char>((size_t)s * dx * ssz);
  void* SY = ar.take<char>((size_t)s * dy * ssz);
  double* Rx = ar.take<double>((size_t)dx * dx);
  double* Ry = ar.take<double>((size_t)dy * dy);
  double* Mx = ar.take<double>((size_t)dx * dx);
  double* My = ar.take<double>((size_t)dy * dy);
  double* Rinv = ar.take<double>((size_t)std::max(dx, dy) * std::max(dx, dy));
  double* Rinv2 = ar.take<double>((size_t)std::max(dx, dy) * std::max(dx, dy));
  int* flag = ar.take<int>(4);
  // cross Gram (S X)^T (S Y) of the sketches, for the warm start
  double* Hxy = ar.take<double>((size_t)dx * dy);
  const bool warm = opt.warm_start_iters > 0;
  RcgBuffers B{};
  if (!flag || !Rinv2 || !Hxy || rcg_buffers_take(B, ar, 2, k, std::max<int64_t>(n, s), dd) != SRP_OK) {
    set_error("workspace layout overflow");
    return SRP_ENOMEM;
  }
  if (ctx) {
    B.group[0] = ctx->group[0];
    B.group[1] = ctx->group[1];
  }
  Arena wkeep[2];
  Woodbury wbs[2];
  for (int b = 0; b < 2; ++b)
    if (s < dd[b]) {
      const size_t kb = woodbury_keep_bytes(s, dd[b]);
      wkeep[b] = Arena{ar.take<char>(kb), kb, 0};
      if (!wkeep[b].base) { set_error("workspace layout overflow"); return SRP_ENOMEM; }
    }
  SRP_TRY(setup_mu(opt, k, B.mu, st));
  SRP_TRY(fill_i32(flag, 1, 0, st));
  // 1-2. sketches (same S for X and Y) and metric factors: the Y view on the
  // side stream, concurrently with the X view (separate scratch)
  const size_t scr = (scratch + 255) & ~size_t(255);
  Arena sx{ar.base + ar.used, scr, 0};
  Arena sy{ar.base + ar.used + scr, scr, 0};
  if (ar.used + 2 * scr > ar.cap) { set_error("workspace layout overflow"); return SRP_ENOMEM; }
  // SRHT: the sampled rows (one S for both views) once, before the fork
  SrhtPlan plan;
  const SrhtPlan* planp = nullptr;
  if (opt.sketch == SRP_SRHT) {
    Arena keep{ar.base + ar.used + 2 * scr, ar.cap - ar.used - 2 * scr, 0};
    Arena tmp{sx.base, sx.cap, 0};
    SRP_TRY(srht_plan_run(n, s, opt.seed, &plan, keep, tmp, st));
    planp = &plan;
  }
  SideFork fk;
  SRP_TRY(fk.begin(st, ctx));
  SRP_TRY(sketch_any(opt.sketch, skin_y, skin_dtype, n, dy, s, opt.seed, SY, sy, fk.side, planp));
  if (staged && skin_dtype == SRP_FP8E4M3) SRP_TRY(scale_cols_run((float*)SY, s, dy, opt.sketch_scale_y, fk.side));
  {
    Arena sub{sy.base, sy.cap, 0};
    if (wby) SRP_TRY(woodbury_factor(SY, sk_dtype, s, dy, ly, Ry, My, flag, sub, wkeep[1], &wbs[1], fk.side));
    else SRP_TRY(sketch_factor_run(SY, sk_dtype, s, dy, ly, Ry, Rinv2, My, flag, sub, fk.side, nullptr,
                                   factor_aux(ctx, 1)));
  }
  SRP_TRY(sketch_any(opt.sketch, skin_x, skin_dtype, n, dx, s, opt.seed, SX, sx, st, planp));
  if (staged && skin_dtype == SRP_FP8E4M3) SRP_TRY(scale_cols_run((float*)SX, s, dx, opt.sketch_scale_x, st));
  const double ms_sketch = tm.lap_ms();   // X view's sketch (Y's runs alongside)
  {
    Arena sub{sx.base, sx.cap, 0};
    if (wbx) SRP_TRY(woodbury_factor(SX, sk_dtype, s, dx, lx, Rx, Mx, flag, sub, wkeep[0], &wbs[0], st));
    else SRP_TRY(sketch_factor_run(SX, sk_dtype, s, dx, lx, Rx, Rinv, Mx, flag, sub, st, nullptr, factor_aux(ctx, 0)));
  }
  SRP_TRY(fk.end(st));
  const bool pencil = wbx || wby;   // no R^-1 for a Woodbury view: the warm start iterates on the pencil
  if (warm && !pencil) {   // cross Gram (S X)^T (S Y), split over the s rows in the X view's scratch
    const int64_t cnt = (int64_t)dx * dy;
    int ks = gram_split(s, dx, dy);
    ks = (int)std::max<int64_t>(1, std::min<int64_t>(ks, (int64_t)(scr / bytes_of<double>((size_t)cnt))));
    double* parts = (double*)sx.base;
    GemmArgs g{};
    g.m = dx; g.n = dy; g.kk = s; g.alpha = 1.0; g.beta = 0.0;
    g.A = SX; g.lda = dx; g.ta = true; g.a_f32 = sk_dtype != SRP_F64;
    g.B = SY; g.ldb = dy; g.tb = false; g.b_f32 = sk_dtype != SRP_F64;
    g.C = parts; g.ldc = dy; g.ksplit = ks; g.c_split_stride = cnt;
    SRP_TRY(gemm_f64(g, st));
    SRP_TRY(sum_parts_f64(parts, ks, cnt, cnt, Hxy, 0, 0.0, st));
  }
  int hflag = 0;
  SRP_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  SRP_HIP(hipStreamSynchronize(st));
  if (hflag) {
    set_error("sketched Gram is not positive definite (lambda = 0 with rank-deficient data?)");
    if (info) info->status = SRP_ENOTSPD;
    return SRP_ENOTSPD;
  }
  const double ms_factor = tm.lap_ms();
  // 3. problems
  RcgProblem full;
  full.nb = 2; full.k = k; full.lda_cost = 0; full.dtype = dtype; full.compute = compute;
  full.A[0] = X; full.A[1] = Y; full.n = n; full.d[0] = dx; full.d[1] = dy;
  full.lam[0] = lx; full.lam[1] = ly; full.Minv[0] = Mx; full.Minv[1] = My;
  full.wb[0] = wbx ? &wbs[0] : nullptr;
  full.wb[1] = wby ? &wbs[1] : nullptr;
  WarmStart ws;
  if (warm && pencil) {
    ws.kind = 3; ws.iters = opt.warm_start_iters; ws.SA[0] = SX; ws.SA[1] = SY; ws.sa_f32 = sk_dtype != SRP_F64;
    ws.s = s; ws.ws = sx.base; ws.ws_bytes = sx.cap;
  } else if (warm) {   // the X view's scratch is free once the cross Gram is summed
    ws.kind = 1; ws.iters = opt.warm_start_iters; ws.Hxy = Hxy; ws.Rinv[0] = Rinv; ws.Rinv[1] = Rinv2;
    ws.ws = sx.base; ws.ws_bytes = sx.cap;
  }
  CommonArgs ca{k, tol, opt};
  double* outW[2] = {U, V};
  if (info) {
    memset(info, 0, sizeof(*info));
    info->ms_sketch = ms_sketch;
    info->ms_factor = ms_factor;
  }
  int rc = solve_tail(full, ws, B, ca, outW, sigma, info, tm, st);
  SRP_HIP(hipStreamSynchronize(st));
  if (info) {
    info->status = rc;
    info->ms_total = info->ms_sketch + info->ms_factor + info->ms_warm + info->ms_iterate;
    double sum = 0.0, hs[KMAX];
    if (hipMemcpy(hs, sigma, sizeof(double) * k, hipMemcpyDeviceToHost) == hipSuccess)
      for (int i = 0; i < k; ++i) sum += hs[i];
    info->objective = sum;
  }
  if (rc == SRP_ENOCONV) set_error("max_iter reached before the gradient tolerance");
  return rc;
}

int lda_solve_impl(const void* X, const int32_t* labels, int64_t n, int d, int c, int k, double lam, int s,
                   double tol, int dtype, const srp_options* optp, hipStream_t st, double* Wout, double* rho,
                   srp_info* info, const SolveCtx* ctx) {
  clear_error();
  srp_options opt;
  srp_default_options(&opt);
  if (optp) opt = *optp;
  SRP_TRY(check_options(opt));
  SRP_REQUIRE(X && labels && Wout && rho, "null pointer argument");
  SRP_REQUIRE(dtype == SRP_F64 || dtype == SRP_F32 || dtype == SRP_BF16, "bad dtype %d", dtype);
  SRP_REQUIRE(n >= 2 && n < (int64_t(1) << 31), "n out of range");
  SRP_REQUIRE(c >= 2 && c <= kLdaMaxClasses && d >= 1, "need 2 <= n_classes <= %d and d >= 1", kLdaMaxClasses);
  SRP_REQUIRE(k >= 1 && k <= std::min(c - 1, d) && k <= KMAX, "need 1 <= k <= min(c-1, d), k <= 32");
  SRP_REQUIRE(opt.method != SRP_RTR || k <= kRtrK, "the trust-region method needs k <= %d", kRtrK);
  SRP_REQUIRE(lam >= 0.0 && tol >= 0.0, "lambda and tol must be >= 0");
  const bool wbm = s < d;   // the metric in Woodbury form
  SRP_REQUIRE(s >= 1 && (!wbm || lam > 0.0), "sketch_size < d needs lambda > 0 (the Woodbury form of M^-1)");
  int compute = opt.pass_compute == -1 ? (dtype == SRP_F64 ? SRP_F64 : SRP_F32) : opt.pass_compute;
  SRP_REQUIRE(opt.final_f64 == 0 || dtype != SRP_BF16, "FP64 closing iterations need F32 or F64 data");
  SRP_REQUIRE(pass_limits_ok(dtype, compute, d, 0, k, 1) || (compute == SRP_F64 && dtype != SRP_BF16),
              "unsupported shape for the data pass (d=%d)", d);
  const int sk_dtype = dtype == SRP_F64 ? SRP_F64 : SRP_F32;
  if (opt.sketch == SRP_SRHT) {
    int64_t np = 2;
    while (np < n) np <<= 1;
    SRP_REQUIRE(np <= (int64_t(1) << 20) && s <= np, "SRHT needs s <= n' <= 2^20");
  }
  PhaseTimer tm(st);
  const size_t esz = dtype_size(dtype), ssz = dtype_size(sk_dtype);
  const int dd[2] = {d, 0};
  const size_t bytes = lda_ws_bytes(n, d, c, k, s, dtype, opt.sketch);
  Workspace Wk;
  void* wbase = nullptr;
  SRP_TRY(take_workspace(Wk, bytes, ctx, st, &wbase));
  Arena ar{(char*)wbase, bytes, 0};
  void* Xhat = ar.take<char>((size_t)n * d * esz);
  void* SXh = ar.take<char>((size_t)s * d * ssz);
  double* R = ar.take<double>((size_t)d * d);
  double* Rinv = ar.take<double>((size_t)d * d);
  double* Minv = ar.take<double>((size_t)d * d);
  const bool warm = opt.warm_start_iters > 0;
  double* Yhat = ar.take<double>((size_t)c * d);
  int* counts = ar.take<int>(c);
  int* flag = ar.take<int>(4);
  RcgBuffers B{};
  if (!flag || rcg_buffers_take(B, ar, 1, k, std::max<int64_t>(n, s), dd, c) != SRP_OK) {
    set_error("workspace layout overflow");
    return SRP_ENOMEM;
  }
  if (ctx) {
    B.group[0] = ctx->group[0];
    B.group[1] = ctx->group[1];
  }
  SRP_TRY(setup_mu(opt, k, B.mu, st));
  // 1. centring; S_B = Yhat^T Yhat stays factored
  {
    Arena sub{ar.base + ar.used, ar.cap - ar.used, 0};
    SRP_TRY(lda_center_run(X, labels, dtype, n, d, c, Xhat, Yhat, counts, flag + 1, sub, st));
  }
  int hc[kLdaMaxClasses];
  int hbad = 0;
  SRP_HIP(hipMemcpyAsync(&hbad, flag + 1, sizeof(int), hipMemcpyDeviceToHost, st));
  SRP_HIP(hipMemcpyAsync(hc, counts, sizeof(int) * c, hipMemcpyDeviceToHost, st));
  SRP_HIP(hipStreamSynchronize(st));
  SRP_REQUIRE(!hbad, "label out of range [0, %d)", c);
  for (int q = 0; q < c; ++q) SRP_REQUIRE(hc[q] > 0, "class %d is empty", q);
  // 2. sketch of Xhat and metric factor
  SRP_TRY(sketch_any(opt.sketch, Xhat, dtype, n, d, s, opt.seed, SXh, ar, st));
  const double ms_sketch = tm.lap_ms();
  SRP_TRY(fill_i32(flag, 1, 0, st));
  Woodbury wbs;
  if (wbm) {
    const size_t kb = woodbury_keep_bytes(s, d);
    Arena keep{ar.take<char>(kb), kb, 0};
    Arena sub{ar.base + ar.used, ar.cap - ar.used, 0};
    if (!keep.base) { set_error("workspace layout overflow"); return SRP_ENOMEM; }
    SRP_TRY(woodbury_factor(SXh, sk_dtype, s, d, lam, R, Minv, flag, sub, keep, &wbs, st));
  } else {
    Arena sub{ar.base + ar.used, ar.cap - ar.used, 0};
    SRP_TRY(sketch_factor_run(SXh, sk_dtype, s, d, lam, R, Rinv, Minv, flag, sub, st, nullptr, factor_aux(ctx, 0)));
  }
  int hflag = 0;
  SRP_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  SRP_HIP(hipStreamSynchronize(st));
  if (hflag) {
    set_error("sketched Gram is not positive definite (lambda = 0 with rank-deficient data?)");
    if (info) info->status = SRP_ENOTSPD;
    return SRP_ENOTSPD;
  }
  const double ms_factor = tm.lap_ms();
  RcgProblem full;
  full.nb = 1; full.k = k; full.lda_cost = 1; full.dtype = dtype; full.compute = compute;
  full.A[0] = Xhat; full.n = n; full.d[0] = d; full.lam[0] = lam; full.Minv[0] = Minv; full.Yhat = Yhat;
  full.c = c;
  full.wb[0] = wbm ? &wbs : nullptr;
  WarmStart ws;
  if (warm) {   // scratch past the solve's buffers (the sketch's and factor's, now free)
    ws.kind = 2; ws.Yhat = Yhat; ws.c = c;
    ws.ws = ar.base + ar.used; ws.ws_bytes = ar.cap - ar.used;
  }
  CommonArgs ca{k, tol, opt};
  double* outW[2] = {Wout, nullptr};
  if (info) {
    memset(info, 0, sizeof(*info));
    info->ms_sketch = ms_sketch;
    info->ms_factor = ms_factor;
  }
  int rc = solve_tail(full, ws, B, ca, outW, rho, info, tm, st);
  SRP_HIP(hipStreamSynchronize(st));
  if (info) {
    info->status = rc;
    info->ms_total = info->ms_sketch + info->ms_factor + info->ms_warm + info->ms_iterate;
    double sum = 0.0, hs[KMAX];
    if (hipMemcpy(hs, rho, sizeof(double) * k, hipMemcpyDeviceToHost) == hipSuccess)
      for (int i = 0; i < k; ++i) sum += hs[i];
    info->objective = sum;
  }
  if (rc == SRP_ENOCONV) set_error("max_iter reached before the gradient tolerance");
  return rc;
}

// ------------------------------------------------------- CSR inputs
// The sparse forms of Algorithms CCAopt and LDAopt: the CountSketch reads
// nnz entries (an SRHT would mix every row: it is not offered), the data
// products are the O(nnz k) sparse-times-skinny products, and the rest of
// the solve (factor, warm start, iteration, finish) is the dense one.  All
// data arithmetic is FP64.
static int csr_common_checks(const srp_options& opt) {
  SRP_REQUIRE(opt.sketch == SRP_COUNTSKETCH, "CSR input takes the CountSketch (an SRHT touches every row)");
  SRP_REQUIRE(!opt.sketch_x && !opt.lowp_x, "CSR input has no staged sketch input or BF16 phase");
  return SRP_OK;
}

static size_t csr_scratch(const CsrView* A, int nv, int s, int k, int c) {
  size_t m = 0;
  int dd[2] = {A[0].d, nv == 2 ? A[1].d : 0};
  for (int b = 0; b < nv; ++b) {
    m = std::max({m, csc_scratch_bytes(A[b]), countsketch_csr_ws_bytes(A[b].n, s), factor_ws_bytes(s, A[b].d)});
    if (s < A[b].d) m = std::max(m, woodbury_factor_scratch(s, A[b].d));
  }
  m = std::max(m, warm_ws_bytes(nv, k, dd, c));
  if (nv == 2) m = std::max(m, bytes_of<double>((size_t)dd[0] * dd[1]));
  return m + 4096;
}

size_t cca_csr_ws_bytes(const CsrView& X, const CsrView& Y, int k, int s) {
  const int dx = X.d, dy = Y.d, dm = std::max(dx, dy);
  const int dd[2] = {dx, dy};
  const CsrView v[2] = {X, Y};
  size_t b = bytes_of<double>((size_t)s * dx) + bytes_of<double>((size_t)s * dy);
  b += 2 * bytes_of<double>((size_t)dx * dx) + 2 * bytes_of<double>((size_t)dy * dy);   // R, M^-1
  b += 2 * bytes_of<double>((size_t)dm * dm) + bytes_of<int>(4) + bytes_of<double>((size_t)dx * dy);
  b += csc_bytes(X) + csc_bytes(Y) + csc_partial_bytes(X, 2 * k) + csc_partial_bytes(Y, 2 * k);
  b += rcg_buffers_bytes(2, k, std::max<int64_t>(X.n, s), dd, SRP_F64);
  for (int q = 0; q < 2; ++q)
    if (s < dd[q]) b += woodbury_keep_bytes(s, dd[q]);
  return b + csr_scratch(v, 2, s, k, 0) + 4096;
}

size_t lda_csr_ws_bytes(const CsrView& X, int c, int k, int s) {
  const int d = X.d;
  const int dd[2] = {d, 0};
  size_t b = bytes_of<double>((size_t)s * d) + bytes_of<double>((size_t)s * c);
  b += 3 * bytes_of<double>((size_t)d * d) + 3 * bytes_of<double>((size_t)c * d) + bytes_of<double>((size_t)c * k);
  b += bytes_of<int>(c) + bytes_of<int>(4) + csc_bytes(X) + csc_partial_bytes(X, k);
  b += rcg_buffers_bytes(1, k, std::max<int64_t>(X.n, s), dd, SRP_F64, c);
  if (s < d) b += woodbury_keep_bytes(s, d);
  return b + csr_scratch(&X, 1, s, k, c) + 4096;
}

static void finish_info(srp_info* info, int rc, const double* vals, int k) {
  if (!info) return;
  info->status = rc;
  info->ms_total = info->ms_sketch + info->ms_factor + info->ms_warm + info->ms_iterate;
  double sum = 0.0, hs[KMAX];
  if (hipMemcpy(hs, vals, sizeof(double) * k, hipMemcpyDeviceToHost) == hipSuccess)
    for (int i = 0; i < k; ++i) sum += hs[i];
  info->objective = sum;
}

int cca_solve_csr_impl(const CsrView& X, const CsrView& Y, int k, double lx, double ly, int s, double tol,
                       const srp_options* optp, hipStream_t st, double* U, double* V, double* sigma, srp_info* info,
                       const SolveCtx* ctx) {
  clear_error();
  srp_options opt;
  srp_default_options(&opt);
  if (optp) opt = *optp;
  SRP_TRY(check_options(opt));
  SRP_TRY(csr_common_checks(opt));
  SRP_REQUIRE(U && V && sigma, "null pointer argument");
  SRP_REQUIRE(X.n == Y.n, "X and Y must have the same number of rows");
  const int64_t n = X.n;
  const int dx = X.d, dy = Y.d;
  SRP_REQUIRE(k >= 1 && k <= std::min(dx, dy) && k <= 16, "need 1 <= k <= min(dx, dy), k <= 16");
  SRP_REQUIRE(lx >= 0.0 && ly >= 0.0 && tol >= 0.0, "lambda and tol must be >= 0");
  const bool wbv[2] = {s < dx, s < dy};
  SRP_REQUIRE(s >= 1 && (!wbv[0] || lx > 0.0) && (!wbv[1] || ly > 0.0),
              "sketch_size < d needs lambda > 0 for that view (the Woodbury form of M^-1)");
  PhaseTimer tm(st);
  const size_t bytes = cca_csr_ws_bytes(X, Y, k, s);
  const CsrView views[2] = {X, Y};
  const size_t scr = csr_scratch(views, 2, s, k, 0);
  Workspace W;
  void* wbase = nullptr;
  SRP_TRY(take_workspace(W, bytes, ctx, st, &wbase));
  Arena ar{(char*)wbase, bytes, 0};
  int* flag = ar.take<int>(4);
  SRP_TRY(csr_check(X, "X", flag, st));
  SRP_TRY(csr_check(Y, "Y", flag, st));
  const int dd[2] = {dx, dy}, dm = std::max(dx, dy);
  double* SX = ar.take<double>((size_t)s * dx);
  double* SY = ar.take<double>((size_t)s * dy);
  double* Rx = ar.take<double>((size_t)dx * dx);
  double* Ry = ar.take<double>((size_t)dy * dy);
  double* Mx = ar.take<double>((size_t)dx * dx);
  double* My = ar.take<double>((size_t)dy * dy);
  double* Rinv = ar.take<double>((size_t)dm * dm);
  double* Rinv2 = ar.take<double>((size_t)dm * dm);
  double* Hxy = ar.take<double>((size_t)dx * dy);
  SparseData sd;
  sd.csr[0] = X;
  sd.csr[1] = Y;
  RcgBuffers B{};
  if (!Hxy || rcg_buffers_take(B, ar, 2, k, std::max<int64_t>(n, s), dd) != SRP_OK) {
    set_error("workspace layout overflow");
    return SRP_ENOMEM;
  }
  Arena wkeep[2];
  Woodbury wbs[2];
  for (int b = 0; b < 2; ++b)
    if (wbv[b]) {
      const size_t kb = woodbury_keep_bytes(s, dd[b]);
      wkeep[b] = Arena{ar.take<char>(kb), kb, 0};
      if (!wkeep[b].base) { set_error("workspace layout overflow"); return SRP_ENOMEM; }
    }
  SRP_TRY(setup_mu(opt, k, B.mu, st));
  if (ar.used + scr > ar.cap) { set_error("workspace layout overflow"); return SRP_ENOMEM; }
  Arena keep{ar.base + ar.used, ar.cap - ar.used - scr, 0};
  char* scratch_base = ar.base + ar.cap - scr;
  // CSC copies, sketches (one S for both views) and metric factors; the
  // steps share one scratch area in stream order
  for (int b = 0; b < 2; ++b) {
    Arena t{scratch_base, scr, 0};
    SRP_TRY(csc_build(views[b], &sd.csc[b], keep, t, st));
    sd.partial[b] = (double*)keep.take<char>(csc_partial_bytes(views[b], 2 * k));
  }
  if (!sd.partial[1]) { set_error("workspace layout overflow"); return SRP_ENOMEM; }
  SRP_TRY(fill_i32(flag, 1, 0, st));
  for (int b = 0; b < 2; ++b) {
    Arena t{scratch_base, scr, 0};
    SRP_TRY(countsketch_csr_run(views[b], s, opt.seed, b ? SY : SX, nullptr, 0, nullptr, t, st));
  }
  const double ms_sketch = tm.lap_ms();
  {
    Arena t{scratch_base, scr, 0};
    if (wbv[0]) SRP_TRY(woodbury_factor(SX, SRP_F64, s, dx, lx, Rx, Mx, flag, t, wkeep[0], &wbs[0], st));
    else SRP_TRY(sketch_factor_run(SX, SRP_F64, s, dx, lx, Rx, Rinv, Mx, flag, t, st, nullptr, factor_aux(ctx, 0)));
  }
  {
    Arena t{scratch_base, scr, 0};
    if (wbv[1]) SRP_TRY(woodbury_factor(SY, SRP_F64, s, dy, ly, Ry, My, flag, t, wkeep[1], &wbs[1], st));
    else SRP_TRY(sketch_factor_run(SY, SRP_F64, s, dy, ly, Ry, Rinv2, My, flag, t, st, nullptr, factor_aux(ctx, 0)));
  }
  const bool warm = opt.warm_start_iters > 0;
  const bool pencil = wbv[0] || wbv[1];
  if (warm && !pencil) {
    const int64_t cnt = (int64_t)dx * dy;
    int ks = gram_split(s, dx, dy);
    ks = (int)std::max<int64_t>(1, std::min<int64_t>(ks, (int64_t)(scr / bytes_of<double>((size_t)cnt))));
    double* parts = (double*)scratch_base;
    GemmArgs g{};
    g.m = dx; g.n = dy; g.kk = s; g.alpha = 1.0; g.beta = 0.0;
    g.A = SX; g.lda = dx; g.ta = true; g.a_f32 = false;
    g.B = SY; g.ldb = dy; g.tb = false; g.b_f32 = false;
    g.C = parts; g.ldc = dy; g.ksplit = ks; g.c_split_stride = cnt;
    SRP_TRY(gemm_f64(g, st));
    SRP_TRY(sum_parts_f64(parts, ks, cnt, cnt, Hxy, 0, 0.0, st));
  }
  int hflag = 0;
  SRP_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  SRP_HIP(hipStreamSynchronize(st));
  if (hflag) {
    set_error("sketched Gram is not positive definite (lambda = 0 with rank-deficient data?)");
    if (info) info->status = SRP_ENOTSPD;
    return SRP_ENOTSPD;
  }
  const double ms_factor = tm.lap_ms();
  RcgProblem full;
  full.nb = 2; full.k = k; full.lda_cost = 0; full.dtype = SRP_F64; full.compute = SRP_F64;
  full.n = n; full.d[0] = dx; full.d[1] = dy;
  full.lam[0] = lx; full.lam[1] = ly; full.Minv[0] = Mx; full.Minv[1] = My;
  full.sp = &sd;
  full.wb[0] = wbv[0] ? &wbs[0] : nullptr;
  full.wb[1] = wbv[1] ? &wbs[1] : nullptr;
  WarmStart ws;
  if (warm && pencil) {
    ws.kind = 3; ws.iters = opt.warm_start_iters; ws.SA[0] = SX; ws.SA[1] = SY; ws.sa_f32 = false; ws.s = s;
    ws.ws = scratch_base; ws.ws_bytes = scr;
  } else if (warm) {
    ws.kind = 1; ws.iters = opt.warm_start_iters; ws.Hxy = Hxy; ws.Rinv[0] = Rinv; ws.Rinv[1] = Rinv2;
    ws.ws = scratch_base; ws.ws_bytes = scr;
  }
  CommonArgs ca{k, tol, opt};
  double* outW[2] = {U, V};
  if (info) {
    memset(info, 0, sizeof(*info));
    info->ms_sketch = ms_sketch;
    info->ms_factor = ms_factor;
  }
  int rc = solve_tail(full, ws, B, ca, outW, sigma, info, tm, st);
  SRP_HIP(hipStreamSynchronize(st));
  finish_info(info, rc, sigma, k);
  if (rc == SRP_ENOCONV) set_error("max_iter reached before the gradient tolerance");
  return rc;
}

int lda_solve_csr_impl(const CsrView& X, const int32_t* labels, int c, int k, double lam, int s, double tol,
                       const srp_options* optp, hipStream_t st, double* Wout, double* rho, srp_info* info,
                       const SolveCtx* ctx) {
  clear_error();
  srp_options opt;
  srp_default_options(&opt);
  if (optp) opt = *optp;
  SRP_TRY(check_options(opt));
  SRP_TRY(csr_common_checks(opt));
  SRP_REQUIRE(labels && Wout && rho, "null pointer argument");
  const int64_t n = X.n;
  const int d = X.d;
  SRP_REQUIRE(n >= 2, "n out of range");
  SRP_REQUIRE(c >= 2 && c <= kLdaMaxClasses, "need 2 <= n_classes <= %d", kLdaMaxClasses);
  SRP_REQUIRE(k >= 1 && k <= std::min(c - 1, d) && k <= KMAX, "need 1 <= k <= min(c-1, d), k <= 32");
  SRP_REQUIRE(opt.method != SRP_RTR || k <= kRtrK, "the trust-region method needs k <= %d", kRtrK);
  SRP_REQUIRE(lam >= 0.0 && tol >= 0.0, "lambda and tol must be >= 0");
  const bool wbm = s < d;
  SRP_REQUIRE(s >= 1 && (!wbm || lam > 0.0), "sketch_size < d needs lambda > 0 (the Woodbury form of M^-1)");
  PhaseTimer tm(st);
  const size_t bytes = lda_csr_ws_bytes(X, c, k, s);
  const size_t scr = csr_scratch(&X, 1, s, k, c);
  Workspace Wk;
  void* wbase = nullptr;
  SRP_TRY(take_workspace(Wk, bytes, ctx, st, &wbase));
  Arena ar{(char*)wbase, bytes, 0};
  int* flag = ar.take<int>(4);
  SRP_TRY(csr_check(X, "X", flag, st));
  int* counts = ar.take<int>(c);
  SRP_TRY(fill_i32(flag + 1, 1, 0, st));
  SRP_TRY(label_counts_run(n, c, labels, counts, flag + 1, st));
  {
    int hc[kLdaMaxClasses];
    int hbad = 0;
    SRP_HIP(hipMemcpyAsync(&hbad, flag + 1, sizeof(int), hipMemcpyDeviceToHost, st));
    SRP_HIP(hipMemcpyAsync(hc, counts, sizeof(int) * c, hipMemcpyDeviceToHost, st));
    SRP_HIP(hipStreamSynchronize(st));
    SRP_REQUIRE(!hbad, "label out of range [0, %d)", c);
    for (int q = 0; q < c; ++q) SRP_REQUIRE(hc[q] > 0, "class %d is empty", q);
  }
  const int dd[2] = {d, 0};
  double* SXh = ar.take<double>((size_t)s * d);
  double* SE = ar.take<double>((size_t)s * c);
  double* R = ar.take<double>((size_t)d * d);
  double* Rinv = ar.take<double>((size_t)d * d);
  double* Minv = ar.take<double>((size_t)d * d);
  double* sums = ar.take<double>((size_t)c * d);
  double* means = ar.take<double>((size_t)c * d);
  double* Yhat = ar.take<double>((size_t)c * d);
  double* T = ar.take<double>((size_t)c * k);
  RcgBuffers B{};
  if (!T || rcg_buffers_take(B, ar, 1, k, std::max<int64_t>(n, s), dd, c) != SRP_OK) {
    set_error("workspace layout overflow");
    return SRP_ENOMEM;
  }
  SRP_TRY(setup_mu(opt, k, B.mu, st));
  if (ar.used + scr > ar.cap) { set_error("workspace layout overflow"); return SRP_ENOMEM; }
  Arena keep{ar.base + ar.used, ar.cap - ar.used - scr, 0};
  char* scratch_base = ar.base + ar.cap - scr;
  SparseData sd;
  sd.csr[0] = X;
  sd.labels = labels;
  sd.means = means;
  sd.T = T;
  {
    Arena t{scratch_base, scr, 0};
    SRP_TRY(csc_build(X, &sd.csc[0], keep, t, st));
    sd.partial[0] = (double*)keep.take<char>(csc_partial_bytes(X, k));
  }
  if (!sd.partial[0]) { set_error("workspace layout overflow"); return SRP_ENOMEM; }
  // class statistics; the sketch of Xhat = X - E C is S X - (S E) C
  SRP_TRY(fda_csr_stats_run(sd.csc[0], n, c, labels, counts, sums, means, Yhat, st));
  {
    Arena t{scratch_base, scr, 0};
    SRP_TRY(countsketch_csr_run(X, s, opt.seed, SXh, labels, c, SE, t, st));
  }
  {
    GemmArgs g{};
    g.m = s; g.n = d; g.kk = c; g.alpha = -1.0; g.beta = 1.0;
    g.A = SE; g.lda = c; g.ta = false; g.a_f32 = false;
    g.B = means; g.ldb = d; g.tb = false; g.b_f32 = false;
    g.C = SXh; g.ldc = d;
    SRP_TRY(gemm_f64(g, st));
  }
  const double ms_sketch = tm.lap_ms();
  SRP_TRY(fill_i32(flag, 1, 0, st));
  Woodbury wbs;
  {
    Arena t{scratch_base, scr, 0};
    if (wbm) {
      const size_t kb = woodbury_keep_bytes(s, d);
      Arena wk{keep.take<char>(kb), kb, 0};
      if (!wk.base) { set_error("workspace layout overflow"); return SRP_ENOMEM; }
      SRP_TRY(woodbury_factor(SXh, SRP_F64, s, d, lam, R, Minv, flag, t, wk, &wbs, st));
    } else {
      SRP_TRY(sketch_factor_run(SXh, SRP_F64, s, d, lam, R, Rinv, Minv, flag, t, st, nullptr, factor_aux(ctx, 0)));
    }
  }
  int hflag = 0;
  SRP_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  SRP_HIP(hipStreamSynchronize(st));
  if (hflag) {
    set_error("sketched Gram is not positive definite (lambda = 0 with rank-deficient data?)");
    if (info) info->status = SRP_ENOTSPD;
    return SRP_ENOTSPD;
  }
  const double ms_factor = tm.lap_ms();
  RcgProblem full;
  full.nb = 1; full.k = k; full.lda_cost = 1; full.dtype = SRP_F64; full.compute = SRP_F64;
  full.n = n; full.d[0] = d; full.lam[0] = lam; full.Minv[0] = Minv; full.Yhat = Yhat; full.c = c;
  full.sp = &sd;
  full.wb[0] = wbm ? &wbs : nullptr;
  WarmStart ws;
  if (opt.warm_start_iters > 0) {
    ws.kind = 2; ws.Yhat = Yhat; ws.c = c;
    ws.ws = scratch_base; ws.ws_bytes = scr;
  }
  CommonArgs ca{k, tol, opt};
  double* outW[2] = {Wout, nullptr};
  if (info) {
    memset(info, 0, sizeof(*info));
    info->ms_sketch = ms_sketch;
    info->ms_factor = ms_factor;
  }
  int rc = solve_tail(full, ws, B, ca, outW, rho, info, tm, st);
  SRP_HIP(hipStreamSynchronize(st));
  finish_info(info, rc, rho, k);
  if (rc == SRP_ENOCONV) set_error("max_iter reached before the gradient tolerance");
  return rc;
}

}  // namespace srp
