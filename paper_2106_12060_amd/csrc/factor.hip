// FP64 dense blocks for the preconditioner factor (Section 3): the Gram of
// the sketch SA^T SA (+ lambda I), its blocked Cholesky factor R (upper,
// positive diagonal, R^T R = M), R^-1, and the explicit M^-1 = R^-1 R^-T
// that the iteration applies.  All products run on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64) through one 64x64-tile GEMM kernel.
//
// Forming R from the Gram instead of a Householder QR of [SA; sqrt(lambda) I]
// gives the same R (both are the unique upper Cholesky factor of M) as long
// as kappa(M) * 2^-53 << 1, which holds for every workload here.
#include "common.hpp"
#include "kernels.hpp"

#include <type_traits>
#include <vector>

namespace srp {

__global__ void k_fill_f64(double* p, int64_t count, double v) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

int fill_f64(double* p, int64_t count, double v, hipStream_t st) {
  if (count <= 0) return SRP_OK;
  hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, p, count, v);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

__global__ void k_copy_f64(double* dst, const double* src, int64_t count) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < count) dst[i] = src[i];
}

int copy_f64(double* dst, const double* src, int64_t count, hipStream_t st) {
  if (count <= 0) return SRP_OK;
  hipLaunchKernelGGL(k_copy_f64, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, dst, src, count);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

// ------------------------------------------------------------- GEMM
// One workgroup = one 64x64 output tile; 4 waves, each a 32x32 quadrant of
// 2x2 MFMA tiles.  The k dimension is staged through LDS 32 at a time; the
// global loads of chunk i+1 are in flight in registers while the matrix
// cores work on chunk i.
constexpr int kGemmK = 32;

template <class AT, class BT, bool TA, bool TB>
__global__ void __launch_bounds__(256) k_gemm_f64(int m, int n, int kk, double alpha, const AT* __restrict__ A,
                                                  int64_t lda, const BT* __restrict__ B, int64_t ldb, double beta,
                                                  double* __restrict__ C, int64_t ldc, int upper_only, int kchunk,
                                                  int64_t c_split_stride) {
  const int tj = blockIdx.x, ti = blockIdx.y, z = blockIdx.z;
  if (upper_only && ti > tj) return;
  const int i0 = ti * 64, j0 = tj * 64;
  const int kbeg = z * kchunk;
  const int kend = min(kk, kbeg + kchunk);
  C += (int64_t)z * c_split_stride;
  __shared__ double As[kGemmK][65];
  __shared__ double Bs[kGemmK][65];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wi = (w >> 1) * 32, wj = (w & 1) * 32;
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  constexpr int PER = kGemmK * 64 / 256;
  double ra[PER], rb[PER];
  auto load = [&](int k0) __attribute__((always_inline)) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = t + q * 256;
      int kq, iq;
      if (TA) { kq = e >> 6; iq = e & 63; } else { iq = e >> 5; kq = e & 31; }
      const int gi = i0 + iq, gk = k0 + kq;
      ra[q] = (gi < m && gk < kend) ? (TA ? (double)A[(int64_t)gk * lda + gi] : (double)A[(int64_t)gi * lda + gk])
                                    : 0.0;
      int kb, jb;
      if (!TB) { kb = e >> 6; jb = e & 63; } else { jb = e >> 5; kb = e & 31; }
      const int gj = j0 + jb, gk2 = k0 + kb;
      rb[q] = (gj < n && gk2 < kend) ? (TB ? (double)B[(int64_t)gj * ldb + gk2] : (double)B[(int64_t)gk2 * ldb + gj])
                                     : 0.0;
    }
  };
  if (kbeg < kend) load(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += kGemmK) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = t + q * 256;
      if (TA) As[e >> 6][e & 63] = ra[q]; else As[e & 31][e >> 5] = ra[q];
      if (!TB) Bs[e >> 6][e & 63] = rb[q]; else Bs[e & 31][e >> 5] = rb[q];
    }
    __syncthreads();
    if (k0 + kGemmK < kend) load(k0 + kGemmK);
#pragma unroll
    for (int s = 0; s < kGemmK / 4; ++s) {
      const int kl = 4 * s + (lane >> 4);
      const double a0 = As[kl][wi + (lane & 15)], a1 = As[kl][wi + 16 + (lane & 15)];
      const double b0 = Bs[kl][wj + (lane & 15)], b1 = Bs[kl][wj + 16 + (lane & 15)];
      acc[0][0] = mfma16x16x4(a0, b0, acc[0][0]);
      acc[0][1] = mfma16x16x4(a0, b1, acc[0][1]);
      acc[1][0] = mfma16x16x4(a1, b0, acc[1][0]);
      acc[1][1] = mfma16x16x4(a1, b1, acc[1][1]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = i0 + wi + 16 * a + acc_row<double>(lane, r);
        const int col = j0 + wj + 16 * b + (lane & 15);
        if (row < m && col < n) {
          double v = alpha * acc[a][b][r];
          if (beta != 0.0) v += beta * C[(int64_t)row * ldc + col];
          C[(int64_t)row * ldc + col] = v;
        }
      }
}

// Large A^T B (the sketch Grams): one workgroup = one 128 x 128 output
// tile, each wave a 64 x 64 quadrant of 4 x 4 MFMA tiles (two products per
// LDS operand read); the contraction runs in stages of 16 through two LDS
// buffers, the global loads of the next two stages in flight during a
// stage's products.
constexpr int kGemmBigK = 16;
template <class AT, class BT>
__global__ void __launch_bounds__(256) k_gemm_f64_big(int m, int n, int kk, double alpha, const AT* __restrict__ A,
                                                      int64_t lda, const BT* __restrict__ B, int64_t ldb, double beta,
                                                      double* __restrict__ C, int64_t ldc, int upper_only, int kchunk,
                                                      int64_t c_split_stride) {
  constexpr int KS = kGemmBigK, P = 128 + 4, PER = KS * 128 / 256;
  const int tj = blockIdx.x, ti = blockIdx.y, z = blockIdx.z;
  if (upper_only && ti > tj) return;
  const int i0 = ti * 128, j0 = tj * 128;
  const int kbeg = z * kchunk;
  const int kend = min(kk, kbeg + kchunk);
  C += (int64_t)z * c_split_stride;
  __shared__ double As[2][KS][P];   // [buffer][k][row]
  __shared__ double Bs[2][KS][P];   // [buffer][k][col]
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wi = (w >> 1) * 64, wj = (w & 1) * 64;
  f64x4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  // Two register sets of staged operands: the loads of the stages two and
  // three ahead are in flight while a stage is multiplied (one stage of
  // products is shorter than a load's latency from HBM).
  AT ra0[PER], ra1[PER];
  BT rb0[PER], rb1[PER];
  auto load = [&](int k0, AT (&ra)[PER], BT (&rb)[PER]) __attribute__((always_inline)) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = t + q * 256;
      const int kq = e >> 7, iq = e & 127;
      const int gk = k0 + kq, gi = i0 + iq, gj = j0 + iq;
      ra[q] = (gi < m && gk < kend) ? A[(int64_t)gk * lda + gi] : AT(0);
      rb[q] = (gj < n && gk < kend) ? B[(int64_t)gk * ldb + gj] : BT(0);
    }
  };
  auto store = [&](int buf, const AT (&ra)[PER], const BT (&rb)[PER]) __attribute__((always_inline)) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = t + q * 256;
      As[buf][e >> 7][e & 127] = (double)ra[q];
      Bs[buf][e >> 7][e & 127] = (double)rb[q];
    }
  };
  auto compute = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int s = 0; s < KS / 4; ++s) {
      const int kl = 4 * s + (lane >> 4);
      double av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = As[buf][kl][wi + 16 * a + (lane & 15)];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = Bs[buf][kl][wj + 16 * b + (lane & 15)];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = mfma16x16x4(av[a], bv[b], acc[a][b]);
    }
  };
  if (kbeg < kend) {
    load(kbeg, ra0, rb0);
    store(0, ra0, rb0);
    if (kbeg + KS < kend) load(kbeg + KS, ra0, rb0);
    if (kbeg + 2 * KS < kend) load(kbeg + 2 * KS, ra1, rb1);
  }
  __syncthreads();
  // even stages in buffer 0, odd ones in buffer 1; set 0 carries the
  // stages 1, 3, ... ahead, set 1 the stages 2, 4, ...
  for (int k0 = kbeg; k0 < kend; k0 += 2 * KS) {
    compute(0);
    if (k0 + KS < kend) store(1, ra0, rb0);
    if (k0 + 3 * KS < kend) load(k0 + 3 * KS, ra0, rb0);
    __syncthreads();
    if (k0 + KS >= kend) break;
    compute(1);
    if (k0 + 2 * KS < kend) store(0, ra1, rb1);
    if (k0 + 4 * KS < kend) load(k0 + 4 * KS, ra1, rb1);
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = i0 + wi + 16 * a + acc_row<double>(lane, r);
        const int col = j0 + wj + 16 * b + (lane & 15);
        if (row < m && col < n) {
          double v = alpha * acc[a][b][r];
          if (beta != 0.0) v += beta * C[(int64_t)row * ldc + col];
          C[(int64_t)row * ldc + col] = v;
        }
      }
}

// FP32 operands (the sketch Grams of FP32 sketches): the tiles and wave
// quadrants of k_gemm_f64_big, with the operand stages moved HBM -> LDS by
// buffer loads with the LDS flag (no staging registers) into a ring of
// kGdStages stages, the next three in flight while one is multiplied.  A
// stage is 16 contraction rows of the tile's 128 columns of A and of B.
// One load instruction moves rows r and r + 8 of one operand (16 B per
// lane: lanes 0-31 row r, lanes 32-63 row r + 8) into slot r of 256 + 16
// floats, so the four rows one matrix step reads (4 s .. 4 s + 3: slots
// 16 floats apart) fall on distinct banks.  Each wave issues the same four
// instructions per stage (slots 2 w, 2 w + 1 of A and of B), so waiting for
// a stage leaves (stages issued after it) x 4 of its loads outstanding.
// The operands are converted to FP64 as they are read.
constexpr int kGdStages = 4;
constexpr int kGdSlot = 272;                  // floats per slot: two rows + pad
constexpr int kGdStage = 2 * 8 * kGdSlot;     // slots of A, then of B

__device__ __forceinline__ void gd_wait(int n) {   // at most n of this wave's loads outstanding
  if (n >= 8) __builtin_amdgcn_s_waitcnt(8 | (0x7 << 4) | (0xF << 8));
  else if (n >= 4) __builtin_amdgcn_s_waitcnt(4 | (0x7 << 4) | (0xF << 8));
  else __builtin_amdgcn_s_waitcnt(0 | (0x7 << 4) | (0xF << 8));
}

// One stage: issue the loads of stage `qi` (when issue) into nxt, then
// multiply the stage in cur (when mult).  The two regions arrive as
// separate restrict pointers, so the compiler sees the reads of cur as
// disjoint from the writes into nxt and waits on no load before them.
__device__ __forceinline__ void gd_step(const float* __restrict__ cur, float* __restrict__ nxt, bool issue, int k0,
                                        int kend, __amdgpu_buffer_rsrc_t ars, __amdgpu_buffer_rsrc_t brs, int lda,
                                        int ldb, int m, int n, int i0, int j0, int w, int lane, bool mult,
                                        f64x4 (&acc)[4][4], int wi, int wj) {
  if (issue) {
    const int half = lane >> 5, c4 = 4 * (lane & 31);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int slot = 2 * w + u;
      const int row = k0 + slot + 8 * half;
      const int ia = i0 + c4, jb = j0 + c4;
      const int oa = (row < kend && ia < m) ? (row * lda + ia) * 4 : kOob;
      const int ob = (row < kend && jb < n) ? (row * ldb + jb) * 4 : kOob;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(ars, (__attribute__((address_space(3))) void*)(nxt + slot * kGdSlot),
                                               16, oa, 0, 0, 0);
      __builtin_amdgcn_raw_ptr_buffer_load_lds(brs,
                                               (__attribute__((address_space(3))) void*)(nxt + (8 + slot) * kGdSlot),
                                               16, ob, 0, 0, 0);
    }
  }
  if (!mult) return;
  const int g = lane >> 4, l16 = lane & 15;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int kl = 4 * s + g;
    const int base = (kl & 7) * kGdSlot + (kl >> 3) * 128 + l16;
    double av[4], bv[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) av[a] = (double)cur[base + wi + 16 * a];
#pragma unroll
    for (int b = 0; b < 4; ++b) bv[b] = (double)cur[8 * kGdSlot + base + wj + 16 * b];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = mfma16x16x4(av[a], bv[b], acc[a][b]);
  }
}

__global__ void __launch_bounds__(256) k_gemm_f64_dma(int m, int n, int kk, double alpha, const float* __restrict__ A,
                                                      int64_t lda, const float* __restrict__ B, int64_t ldb,
                                                      double beta, double* __restrict__ C, int64_t ldc,
                                                      int upper_only, int kchunk, int64_t c_split_stride) {
  constexpr int NST = kGdStages, LOOK = NST - 1;
  const int tj = blockIdx.x, ti = blockIdx.y, z = blockIdx.z;
  if (upper_only && ti > tj) return;
  const int i0 = ti * 128, j0 = tj * 128;
  const int kbeg = z * kchunk;
  const int kend = min(kk, kbeg + kchunk);
  C += (int64_t)z * c_split_stride;
  extern __shared__ float gsm[];
  const int t = threadIdx.x, lane = t & 63;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int wi = (w >> 1) * 64, wj = (w & 1) * 64;
  const __amdgpu_buffer_rsrc_t ars = make_rsrc(A, (int64_t)kk * lda * 4);
  const __amdgpu_buffer_rsrc_t brs = make_rsrc(B, (int64_t)kk * ldb * 4);
  f64x4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  const int nstg = kbeg < kend ? (kend - kbeg + 15) / 16 : 0;
  // step q < 0 only issues stage q + LOOK; step q >= 0 waits for stage q
  // (this wave's loads, then every wave's), issues stage q + LOOK into the
  // slot stage q - 1 left and multiplies stage q
  for (int q = -LOOK; q < nstg; ++q) {
    if (q >= 0) {
      gd_wait(4 * min(LOOK - 1, nstg - 1 - q));
      asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
    }
    const int qi = q + LOOK;
    gd_step(gsm + ((q + NST) % NST) * kGdStage, gsm + (qi % NST) * kGdStage, qi < nstg, kbeg + 16 * qi, kend, ars,
            brs, (int)lda, (int)ldb, m, n, i0, j0, w, lane, q >= 0, acc, wi, wj);
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = i0 + wi + 16 * a + acc_row<double>(lane, r);
        const int col = j0 + wj + 16 * b + (lane & 15);
        if (row < m && col < n) {
          double v = alpha * acc[a][b][r];
          if (beta != 0.0) v += beta * C[(int64_t)row * ldc + col];
          C[(int64_t)row * ldc + col] = v;
        }
      }
}

// The big-tile kernel takes A^T B with both output sides and the
// contraction long enough to fill its tiles and stages.
static bool gemm_big(const GemmArgs& g) {
  return g.ta && !g.tb && g.m >= 256 && g.n >= 256 && g.kk >= 512;
}

template <class AT, class BT>
static int gemm_dispatch_t(const GemmArgs& g, hipStream_t st) {
  dim3 grid((g.n + 63) / 64, (g.m + 63) / 64, g.ksplit);
  int kchunk = g.kk;
  if (g.ksplit > 1) kchunk = (((g.kk + g.ksplit - 1) / g.ksplit) + kGemmK - 1) / kGemmK * kGemmK;
  const AT* A = (const AT*)g.A;
  const BT* B = (const BT*)g.B;
  if (gemm_big(g) && std::is_same<AT, float>::value && std::is_same<BT, float>::value && g.lda % 4 == 0 &&
      g.ldb % 4 == 0 && ((uintptr_t)g.A & 15) == 0 && ((uintptr_t)g.B & 15) == 0 &&
      (int64_t)g.kk * g.lda * 4 < kOob && (int64_t)g.kk * g.ldb * 4 < kOob) {
    const dim3 gb((g.n + 127) / 128, (g.m + 127) / 128, g.ksplit);
    const size_t lds = (size_t)kGdStages * kGdStage * sizeof(float);
    SRP_TRY(allow_dynamic_lds((const void*)k_gemm_f64_dma, lds));
    hipLaunchKernelGGL(k_gemm_f64_dma, gb, dim3(256), lds, st, g.m, g.n, g.kk, g.alpha, (const float*)g.A, g.lda,
                       (const float*)g.B, g.ldb, g.beta, g.C, g.ldc, (int)g.upper_only, kchunk, g.c_split_stride);
    SRP_LAUNCH_CHECK();
    return SRP_OK;
  }
  if (gemm_big(g)) {   // kchunk is a multiple of kGemmK, hence of kGemmBigK
    const dim3 gb((g.n + 127) / 128, (g.m + 127) / 128, g.ksplit);
    hipLaunchKernelGGL((k_gemm_f64_big<AT, BT>), gb, dim3(256), 0, st, g.m, g.n, g.kk, g.alpha, A, g.lda, B, g.ldb,
                       g.beta, g.C, g.ldc, (int)g.upper_only, kchunk, g.c_split_stride);
    SRP_LAUNCH_CHECK();
    return SRP_OK;
  }
#define SRP_GEMM_CASE(TA_, TB_)                                                                    \
  hipLaunchKernelGGL((k_gemm_f64<AT, BT, TA_, TB_>), grid, dim3(256), 0, st, g.m, g.n, g.kk, g.alpha, A, \
                     g.lda, B, g.ldb, g.beta, g.C, g.ldc, (int)g.upper_only, kchunk, g.c_split_stride)
  if (g.ta && !g.tb) SRP_GEMM_CASE(true, false);
  else if (!g.ta && !g.tb) SRP_GEMM_CASE(false, false);
  else if (!g.ta && g.tb) SRP_GEMM_CASE(false, true);
  else SRP_GEMM_CASE(true, true);
#undef SRP_GEMM_CASE
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

int gemm_f64(const GemmArgs& g, hipStream_t st) {
  if (g.m <= 0 || g.n <= 0) return SRP_OK;
  if (g.a_f32 && g.b_f32) return gemm_dispatch_t<float, float>(g, st);
  if (g.a_f32) return gemm_dispatch_t<float, double>(g, st);
  if (g.b_f32) return gemm_dispatch_t<double, float>(g, st);
  return gemm_dispatch_t<double, double>(g, st);
}

__global__ void k_sum_parts(const double* parts, int nparts, int64_t stride, int64_t count, double* out, int d,
                            double diag_add) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= count) return;
  double v = 0.0;
  for (int z = 0; z < nparts; ++z) v += parts[z * stride + i];
  if (d > 0 && (i / d) == (i % d)) v += diag_add;
  out[i] = v;
}

// The symmetric d x d Gram from upper-tile partials: entries with i <= j
// are summed in split order (diag_add on the diagonal); those below the
// diagonal, which no upper tile need cover and nothing reads, are set to
// zero without reading the partials (so the partials need no clearing).
__global__ void k_sum_upper(const double* parts, int nparts, int64_t stride, int d, double diag_add, double* out) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)d * d) return;
  const int i = (int)(e / d), j = (int)(e - (int64_t)i * d);
  double v = 0.0;
  if (i <= j) {
    for (int z = 0; z < nparts; ++z) v += parts[z * stride + e];
    if (i == j) v += diag_add;
  }
  out[e] = v;
}

int sum_parts_f64(const double* parts, int nparts, int64_t stride, int64_t count, double* out, int d,
                  double diag_add, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, parts, nparts, stride,
                     count, out, d, diag_add);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

// --------------------------------------------------------- skinny GEMM
// C (m x nc) = op(A) (m x kk) B (kk x nc), nc <= 64: the per-iteration
// products with M^-1, the sketch Gram products of the warm start, the FDA
// between-class factor and the two-read FP64 data products.  The
// contraction is split over blockIdx.y into slices (by default kSkSlice
// for a transposed A, kSkRowSlice otherwise; the caller may ask for longer
// ones); a workgroup writes the partial of its rows and slice, and a
// second kernel adds the partials in slice order (deterministic).  With a
// single slice the workgroups write C directly.
constexpr int kSkSlice = 64;
constexpr int kSkRowSlice = 128;

// Up to four independent problems per launch (blockIdx.z): both views, or
// the four blocks of a two-view Gram.
constexpr int kSkMaxProbs = 4;
struct SkinnyBatch {
  SkinnyProb p[kSkMaxProbs];
  double* part[kSkMaxProbs];
  int slice;          // contraction length per partial
  int direct;         // one slice covers every contraction: write C itself
};

// Output of a workgroup: its slice's partial, or C itself when one slice
// covers the contraction.
__device__ __forceinline__ double* sk_out(const SkinnyBatch& bt, const SkinnyProb& pr, int64_t* ld) {
  if (bt.direct) {
    *ld = pr.ldc;
    return pr.C;
  }
  *ld = pr.nc;
  return bt.part[blockIdx.z] + (int64_t)blockIdx.y * pr.m * pr.nc;
}

// Transposed A (op(A) = A^T, A kk x m row-major: the FDA between-class
// factor, X^T P of the two-read data products).  A workgroup owns 64
// output rows (64 columns of A) and a slice of the contraction; every wave
// covers all 64 rows (four 16-row tiles) and all columns of B, over the
// 4-row steps w, w + 4, ... of the slice, so the four waves read 16
// consecutive rows of A together.  Operands go straight from memory into
// the FP64 matrix-core registers (lane (i, kq) holds A[l][c0 + 16 t + i]
// and B[l][16 q + i] for its contraction row l), UG groups in flight at
// once; the four waves' sums are added in wave order through LDS.
template <class AT, int NCT>
__global__ void __launch_bounds__(256) k_gemm_skinny_t(SkinnyBatch bt) {
  constexpr int UG = 4;
  const SkinnyProb& pr = bt.p[blockIdx.z];
  const int m = pr.m, kk = pr.kk, nc = pr.nc;
  const int c0 = blockIdx.x * 64;
  const int zbeg = blockIdx.y * bt.slice;
  if (c0 >= m || zbeg >= kk) return;
  const int zend = min(kk, zbeg + bt.slice);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int i = lane & 15, kq = lane >> 4;
  const int lda = (int)pr.lda, ldb = (int)pr.ldb;
  const __amdgpu_buffer_rsrc_t arsrc = make_rsrc(pr.A, (int64_t)kk * pr.lda * (int64_t)sizeof(AT));
  const __amdgpu_buffer_rsrc_t brsrc = make_rsrc(pr.B, (int64_t)kk * pr.ldb * 8);
  f64x4 acc[4][NCT];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int q = 0; q < NCT; ++q) acc[t][q] = f64x4{0.0, 0.0, 0.0, 0.0};
  for (int g0 = zbeg; g0 < zend; g0 += 16 * UG) {
    AT a[UG][4];
    double b[UG][NCT];
#pragma unroll
    for (int u = 0; u < UG; ++u) {
      const int l = g0 + 16 * u + 4 * w + kq;   // this lane's contraction row
      const bool lv = l < zend;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int col = c0 + 16 * t + i;
        a[u][t] = buf_load<AT>(arsrc, (lv && col < m) ? (l * lda + col) * (int)sizeof(AT) : kOob, 0);
      }
#pragma unroll
      for (int q = 0; q < NCT; ++q) {
        const int j = 16 * q + i;
        b[u][q] = buf_load<double>(brsrc, (lv && j < nc) ? (l * ldb + j) * 8 : kOob, 0);
      }
    }
#pragma unroll
    for (int u = 0; u < UG; ++u)
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int q = 0; q < NCT; ++q) acc[t][q] = mfma16x16x4((double)a[u][t], b[u][q], acc[t][q]);
  }
  // wave 0 adds waves 1, 2, 3 in order
  __shared__ double red[4 * 4 * NCT][64];
#pragma unroll 1
  for (int src = 1; src < 4; ++src) {
    __syncthreads();
    if (w == src)
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int q = 0; q < NCT; ++q)
#pragma unroll
          for (int r = 0; r < 4; ++r) red[(t * NCT + q) * 4 + r][lane] = acc[t][q][r];
    __syncthreads();
    if (w == 0)
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int q = 0; q < NCT; ++q)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[t][q][r] += red[(t * NCT + q) * 4 + r][lane];
  }
  if (w != 0) return;
  int64_t ldo;
  double* out = sk_out(bt, pr, &ldo);
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int q = 0; q < NCT; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = c0 + 16 * t + acc_row<double>(lane, r);
        const int col = 16 * q + i;
        if (row < m && col < nc) out[(int64_t)row * ldo + col] = acc[t][q][r];
      }
}

// Row-major A (the M^-1 products, the sketch Gram products, X W of the
// two-read data products): a workgroup owns 64 rows (16 per wave) and a
// slice of the contraction, taken kSkRowSlice at a time.  A's rows go
// straight from HBM into registers as matrix-core operands, a whole
// sub-slice in flight at once (lane (i, kq) of the wave holds
// A[row i][16 c + 4 kq + s], s = 0..3, for chunk c: one 32-byte run per lane
// as two 16-byte loads when VEC, 16 bytes as one load for FP32 A); each
// sub-slice of B is staged once in LDS.  Step s of chunk c multiplies over
// the contraction indices 16 c + 4 kq + s (kq = 0..3, one per 16-lane row),
// so A and B agree on the order and every index is taken once.
// LOOP: slices longer than one sub-slice (else the single-pass body, whose
// accumulators need not stay live across a loop).
constexpr int sk_bpitch(int nct) { return (nct & 1) ? 16 * nct : 16 * nct + 16; }
template <class AT, int NCT, bool VEC, bool LOOP>
__global__ void __launch_bounds__(256) k_gemm_skinny_rows(SkinnyBatch bt) {
  constexpr int KS = kSkRowSlice, NCH = KS / 16, P = sk_bpitch(NCT), NBC = 16 * NCT;
  constexpr int NB = (KS * NBC + 255) / 256;
  const SkinnyProb& pr = bt.p[blockIdx.z];
  const int m = pr.m, kk = pr.kk, nc = pr.nc;
  const int r0 = blockIdx.x * 64;
  const int zbeg = blockIdx.y * bt.slice;
  if (r0 >= m || zbeg >= kk) return;
  const int zend = min(kk, zbeg + bt.slice);
  __shared__ double Bs[KS * P];   // [contraction][column], pitch P
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int i = lane & 15, kq = lane >> 4;
  const __amdgpu_buffer_rsrc_t arsrc = make_rsrc(pr.A, (int64_t)m * pr.lda * (int64_t)sizeof(AT));
  const __amdgpu_buffer_rsrc_t brsrc = make_rsrc(pr.B, (int64_t)kk * pr.ldb * 8);
  f64x4 acc[NCT];
#pragma unroll
  for (int q = 0; q < NCT; ++q) acc[q] = f64x4{0.0, 0.0, 0.0, 0.0};
  for (int lbeg = zbeg; lbeg < zend; lbeg += KS) {
  const int lend = LOOP ? min(zend, lbeg + KS) : zend;
  double rb[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int e = tid + 256 * q;
    const int bl = e / NBC, bj = e - bl * NBC, gl = lbeg + bl;
    rb[q] = buf_load<double>(brsrc, (e < KS * NBC && bj < nc && gl < lend) ? (gl * (int)pr.ldb + bj) * 8 : kOob, 0);
  }
  const int row = r0 + 16 * w + i;
  double av[NCH][4];
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const int col = lbeg + 16 * c + 4 * kq;
    if (VEC && sizeof(AT) == 8) {   // kk % 4 == 0, even lda, 16-byte aligned A: col < kk covers col + 3
      const int off = (row < m && col < lend) ? (row * (int)pr.lda + col) * 8 : kOob;
      const auto v0 = __builtin_amdgcn_raw_buffer_load_b128(arsrc, off, 0, 0);
      const auto v1 = __builtin_amdgcn_raw_buffer_load_b128(arsrc, off + 16, 0, 0);
      av[c][0] = __builtin_bit_cast(double, (uint64_t)v0[0] | ((uint64_t)v0[1] << 32));
      av[c][1] = __builtin_bit_cast(double, (uint64_t)v0[2] | ((uint64_t)v0[3] << 32));
      av[c][2] = __builtin_bit_cast(double, (uint64_t)v1[0] | ((uint64_t)v1[1] << 32));
      av[c][3] = __builtin_bit_cast(double, (uint64_t)v1[2] | ((uint64_t)v1[3] << 32));
    } else if (VEC) {               // FP32: kk % 4 == 0, lda % 4 == 0, 16-byte aligned A
      const int off = (row < m && col < lend) ? (row * (int)pr.lda + col) * 4 : kOob;
      const auto v0 = __builtin_amdgcn_raw_buffer_load_b128(arsrc, off, 0, 0);
      av[c][0] = (double)__builtin_bit_cast(float, (uint32_t)v0[0]);
      av[c][1] = (double)__builtin_bit_cast(float, (uint32_t)v0[1]);
      av[c][2] = (double)__builtin_bit_cast(float, (uint32_t)v0[2]);
      av[c][3] = (double)__builtin_bit_cast(float, (uint32_t)v0[3]);
    } else {
#pragma unroll
      for (int s = 0; s < 4; ++s)
        av[c][s] = (double)buf_load<AT>(arsrc, (row < m && col + s < lend)
                                                   ? (row * (int)pr.lda + col + s) * (int)sizeof(AT) : kOob, 0);
    }
  }
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int e = tid + 256 * q;
    if (e < KS * NBC) {
      const int bl = e / NBC, bj = e - bl * NBC;
      Bs[bl * P + bj] = rb[q];
    }
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < NCH; ++c)
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const double* bp = &Bs[(16 * c + 4 * kq + s) * P + i];
#pragma unroll
      for (int q = 0; q < NCT; ++q) acc[q] = mfma16x16x4(av[c][s], bp[16 * q], acc[q]);
    }
  if (!LOOP) break;
  __syncthreads();   // the next sub-slice overwrites Bs
  }
  int64_t ldo;
  double* out = sk_out(bt, pr, &ldo);
#pragma unroll
  for (int q = 0; q < NCT; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int orow = r0 + 16 * w + acc_row<double>(lane, r);
      const int col = 16 * q + i;
      if (orow < m && col < nc) out[(int64_t)orow * ldo + col] = acc[q][r];
    }
}

__global__ void __launch_bounds__(256) k_skinny_sum(SkinnyBatch bt) {
  const SkinnyProb& pr = bt.p[blockIdx.y];
  const int64_t e = blockIdx.x * 256ll + threadIdx.x;
  const int64_t cnt = (int64_t)pr.m * pr.nc;
  if (e >= cnt) return;
  const int nsl = (pr.kk + bt.slice - 1) / bt.slice;
  const double* part = bt.part[blockIdx.y];
  // even slices into s0, odd into s1, in slice order; the loads of 16
  // slices are in flight together
  double s0 = 0.0, s1 = 0.0;
  for (int z0 = 0; z0 < nsl; z0 += 16) {
    double t[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) t[u] = part[(int64_t)(z0 + u < nsl ? z0 + u : 0) * cnt + e];
#pragma unroll
    for (int u = 0; u < 16; u += 2) {
      if (z0 + u < nsl) s0 += t[u];
      if (z0 + u + 1 < nsl) s1 += t[u + 1];
    }
  }
  const int64_t row = e / pr.nc, col = e - row * pr.nc;
  pr.C[row * pr.ldc + col] = s0 + s1;
}

size_t skinny_ws_bytes(int m, int kk, int nc) {
  const size_t nsl = (size_t)(kk + kSkSlice - 1) / kSkSlice;
  return bytes_of<double>(nsl * (size_t)m * nc);
}

int gemm_skinny_batch(int nprob, const SkinnyProb* probs, double* ws, size_t ws_bytes, hipStream_t st,
                      int slice) {
  SkinnyBatch bt{};
  if (nprob < 1 || nprob > kSkMaxProbs) {
    set_error("gemm_skinny: %d problems (1 to %d per launch)", nprob, kSkMaxProbs);
    return SRP_EINVAL;
  }
  const bool rows = !probs[0].ta, f32 = probs[0].a_f32;
  const int64_t esz = f32 ? 4 : 8;
  bool vec = true;
  int nct = 1, gx = 1, kmax = 1, sx = 1;
  for (int q = 0; q < nprob; ++q) {
    const SkinnyProb& p = probs[q];
    if (p.ta != probs[0].ta || p.a_f32 != f32 || p.nc > 64 || p.nc < 1 || p.m < 1 || p.kk < 1 ||
        (int64_t)(p.ta ? p.kk : p.m) * p.lda * esz >= (int64_t(1) << 31) ||
        (int64_t)p.kk * p.ldb * 8 >= (int64_t(1) << 31)) {
      set_error("gemm_skinny: bad shape m=%d kk=%d nc=%d (one A type and layout per batch; operands under 2 GiB)",
                p.m, p.kk, p.nc);
      return SRP_EINVAL;
    }
    vec = vec && p.kk % 4 == 0 && p.lda % (f32 ? 4 : 2) == 0 && ((uintptr_t)p.A & 15) == 0;
    nct = std::max(nct, (p.nc + 15) / 16);
    gx = std::max(gx, (p.m + 63) / 64);
    kmax = std::max(kmax, p.kk);
    sx = std::max(sx, (int)(((int64_t)p.m * p.nc + 255) / 256));
  }
  // contraction per partial: whole sub-slices for the row kernel (the
  // default, kSkRowSlice, needs no more workspace than kSkSlice)
  int sl = slice > 0 ? slice : (rows ? kSkRowSlice : kSkSlice);
  if (rows) sl = (sl + kSkRowSlice - 1) / kSkRowSlice * kSkRowSlice;
  const int gy = (kmax + sl - 1) / sl;
  bt.slice = sl;
  bt.direct = gy == 1 ? 1 : 0;
  size_t used = 0;
  for (int q = 0; q < nprob; ++q) {
    bt.p[q] = probs[q];
    bt.part[q] = (double*)((char*)ws + used);
    if (!bt.direct) used += bytes_of<double>((size_t)((probs[q].kk + sl - 1) / sl) * probs[q].m * probs[q].nc);
  }
  if (used > 0 && (!ws || used > ws_bytes)) {
    set_error("gemm_skinny: workspace too small");
    return SRP_ENOMEM;
  }
  const dim3 grid(gx, gy, nprob);
  if (rows) {
#define SRP_SK_ROWS_T(AT, N, V)                                                                         \
      if (loop) hipLaunchKernelGGL((k_gemm_skinny_rows<AT, N, V, true>), grid, dim3(256), 0, st, bt);   \
      else hipLaunchKernelGGL((k_gemm_skinny_rows<AT, N, V, false>), grid, dim3(256), 0, st, bt);
#define SRP_SK_ROWS(N)                                                                                  \
    case N:                                                                                             \
      if (f32) {                                                                                        \
        if (vec) { SRP_SK_ROWS_T(float, N, true) } else { SRP_SK_ROWS_T(float, N, false) }              \
      } else {                                                                                          \
        if (vec) { SRP_SK_ROWS_T(double, N, true) } else { SRP_SK_ROWS_T(double, N, false) }            \
      }                                                                                                 \
      break;
    const bool loop = sl > kSkRowSlice;
    switch (nct) {
      SRP_SK_ROWS(1) SRP_SK_ROWS(2) SRP_SK_ROWS(3) SRP_SK_ROWS(4)
    }
#undef SRP_SK_ROWS
#undef SRP_SK_ROWS_T
  } else {
#define SRP_SK_T(N)                                                                              \
    case N:                                                                                      \
      if (f32) hipLaunchKernelGGL((k_gemm_skinny_t<float, N>), grid, dim3(256), 0, st, bt);      \
      else hipLaunchKernelGGL((k_gemm_skinny_t<double, N>), grid, dim3(256), 0, st, bt);         \
      break;
    switch (nct) {
      SRP_SK_T(1) SRP_SK_T(2) SRP_SK_T(3) SRP_SK_T(4)
    }
#undef SRP_SK_T
  }
  SRP_LAUNCH_CHECK();
  if (!bt.direct) {
    hipLaunchKernelGGL(k_skinny_sum, dim3(sx, nprob), dim3(256), 0, st, bt);
    SRP_LAUNCH_CHECK();
  }
  return SRP_OK;
}

int gemm_skinny_f64(int m, int kk, int nc, const double* A, int64_t lda, bool ta, const double* B, int64_t ldb,
                    double* C, int64_t ldc, double* ws, size_t ws_bytes, hipStream_t st) {
  SkinnyProb p{m, kk, nc, A, lda, ta, B, ldb, C, ldc};
  return gemm_skinny_batch(1, &p, ws, ws_bytes, st);
}

// --------------------------------------------------------- Cholesky
// Factor the nb x nb diagonal block at (k0, k0) of the symmetric matrix G
// (upper triangle read): R_kk upper with R_kk^T R_kk = G_kk, written into R;
// its inverse into Dinv (64 x 64, upper, identity-padded).  Sets *flag on a
// non-positive pivot.
//
// The block is loaded into LDS once and factored right-looking in four
// panels of 16 rows (details below); the inverse follows by 16 x 16
// blocks.
__device__ __forceinline__ void wave_fence_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// x from lane l (uniform l), as two 32-bit readlanes.
__device__ __forceinline__ double readlane_f64(double x, int l) {
  const uint64_t u = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__global__ void __launch_bounds__(256) k_potrf_block(const double* __restrict__ G, int64_t ld, int k0, int nb,
                                                     double* __restrict__ R, double* __restrict__ Dinv,
                                                     int* flag) {
  __shared__ double a[64][65];
  __shared__ double x[64][65];
  __shared__ double piv[64];
  __shared__ double row[2][65];   // unscaled row j of the trailing matrix, double-buffered by step parity
  __shared__ double rdiag[64];    // 1 / R[j][j]
  __shared__ double tsc[3][16][17];   // per-wave 16 x 16 scratch of the blocked inverse
  const int t = threadIdx.x;
  const int wv = t >> 6, ln = t & 63;
  // The upper triangle of the block in LDS (rows past nb: the identity).
  {
    // all sixteen loads of a thread in flight together (masked entries read
    // the block's first element and are replaced)
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = t + 256 * u, r = e >> 6, c = e & 63;
      const bool in = r <= c && r < nb && c < nb;
      v[u] = G[in ? (int64_t)(k0 + r) * ld + k0 + c : (int64_t)k0 * ld + k0];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = t + 256 * u, r = e >> 6, c = e & 63;
      const bool in = r <= c && r < nb && c < nb;
      a[r][c] = in ? v[u] : ((r == c) ? 1.0 : 0.0);
    }
  }
  __syncthreads();
  // Four panels of 16 rows, right-looking.  Wave 0 factors a panel alone
  // with lane c holding rows p0 .. p0+15 of column c in registers: step j
  // takes the pivot from lane p0+j, scales row j and subtracts its outer
  // product from the rows below, the row-j entries of the other columns
  // broadcast by readlane (no barrier inside the panel).  Then all waves
  // subtract the panel's rows' products from the trailing triangle on FP64
  // matrix cores.
  for (int p0 = 0; p0 < 64; p0 += 16) {
    if (wv == 0) {
      double pr[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) pr[i] = a[p0 + i][ln];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int pl = p0 + j;   // lane (column) of the pivot
        double p = readlane_f64(pr[j], pl);
        const bool bad = !(p > 0.0) || !isfinite(p);
        if (bad) p = 1.0;
        double rs = __builtin_amdgcn_rsq(p);
        rs = rs * fma(-0.5 * p * rs, rs, 1.5);
        rs = rs * fma(-0.5 * p * rs, rs, 1.5);   // 1 / sqrt(p), two Newton steps
        if (ln == 0) {
          if (bad) atomicOr(flag, 1);
          piv[pl] = p;
          rdiag[pl] = rs;
        }
        const double rj = pr[j] * rs;   // row j of R in column ln (ln >= pl)
#pragma unroll
        for (int i = j + 1; i < 16; ++i) {
          const double rji = readlane_f64(rj, p0 + i);   // R[j][p0 + i]
          pr[i] = fma(-rji, rj, pr[i]);
        }
        pr[j] = rj;
      }
      if (ln >= p0) {
#pragma unroll
        for (int i = 0; i < 16; ++i)
          if (p0 + i <= ln) a[p0 + i][ln] = pr[i];
      }
    }
    __syncthreads();
    const int q0 = p0 + 16;
    if (q0 < 64) {
      // a[r][c] -= sum_i R[p0+i][r] R[p0+i][c] for q0 <= r <= c < 64: the
      // upper 16 x 16 tiles of P^T P (P = the panel's rows, columns q0..63)
      // on FP64 matrix cores, tile (ti, tj) by wave (ti + tj) % 4 (entries
      // below the diagonal of a diagonal tile are updated too and never read)
      const int nt = (64 - q0) >> 4;
      const int m16 = ln & 15, kq = ln >> 4;
      for (int ti = 0; ti < nt; ++ti)
        for (int tj = ti; tj < nt; ++tj) {
          if (((ti + tj) & 3) != wv) continue;
          const int r0 = q0 + 16 * ti, c0 = q0 + 16 * tj;
          f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int kb = 0; kb < 4; ++kb)
            acc = mfma16x16x4(a[p0 + 4 * kb + kq][r0 + m16], a[p0 + 4 * kb + kq][c0 + m16], acc);
#pragma unroll
          for (int r = 0; r < 4; ++r) a[r0 + acc_row<double>(ln, r)][c0 + m16] -= acc[r];
        }
      __syncthreads();
    }
  }
  // x = a^-1 (upper) by 16 x 16 blocks: the four diagonal blocks by
  // back-substitution (wave w inverts block w; four lanes per column),
  // then the blocks at distance d = 1, 2, 3 from the diagonal as
  // X_ij = -X_ii sum_{i < l <= j} R_il X_lj on FP64 matrix cores (a level
  // needs only blocks closer to the diagonal).
  for (int e = t; e < 4096; e += 256) x[e >> 6][e & 63] = 0.0;
  __syncthreads();
  {
    const int c = ln >> 2, q = ln & 3, o = 16 * wv;
    for (int r = 15; r >= 0; --r) {
      double sum = 0.0;
#pragma unroll
      for (int m = 0; m < 4; ++m) {   // unconditional loads (clamped index), masked products
        const int l = r + 1 + q + 4 * m;
        const int lc = min(l, 15);
        const double prod = a[o + r][o + lc] * x[o + lc][o + c];
        sum += (l <= c) ? prod : 0.0;
      }
      sum += __shfl_xor(sum, 1, 64);
      sum += __shfl_xor(sum, 2, 64);
      if (q == 0 && r <= c) x[o + r][o + c] = ((r == c) ? 1.0 : -sum) * rdiag[o + r];
      wave_fence_sync();
    }
  }
  __syncthreads();
  {
    const int m16 = ln & 15, kq = ln >> 4;
    for (int d = 1; d <= 3; ++d) {
      if (wv < 4 - d) {
        const int i = wv, j = wv + d;
        f64x4 acc = {0.0, 0.0, 0.0, 0.0};
        for (int l = i + 1; l <= j; ++l) {
#pragma unroll
          for (int kb = 0; kb < 4; ++kb)
            acc = mfma16x16x4(a[16 * i + m16][16 * l + 4 * kb + kq], x[16 * l + 4 * kb + kq][16 * j + m16], acc);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) tsc[wv][acc_row<double>(ln, r)][m16] = acc[r];
        wave_fence_sync();
        f64x4 acc2 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
          acc2 = mfma16x16x4(x[16 * i + m16][16 * i + 4 * kb + kq], tsc[wv][4 * kb + kq][m16], acc2);
#pragma unroll
        for (int r = 0; r < 4; ++r) x[16 * i + acc_row<double>(ln, r)][16 * j + m16] = -acc2[r];
      }
      __syncthreads();
    }
  }
  for (int e = t; e < 4096; e += 256) {
    const int r = e >> 6, c = e & 63;
    Dinv[e] = x[r][c];
    if (r < nb && c < nb) R[(int64_t)(k0 + r) * ld + k0 + c] = (r <= c) ? a[r][c] : 0.0;
  }
}

// Copy 64x64 block inverses onto the diagonal of X (d x d).
__global__ void k_place_diag_blocks(const double* __restrict__ Dinv, int d, double* __restrict__ X, int kb0) {
  const int kb = kb0 + blockIdx.x;
  const int k0 = kb * 64;
  const int nb = min(64, d - k0);
  for (int e = threadIdx.x; e < 4096; e += blockDim.x) {
    const int r = e >> 6, c = e & 63;
    if (r < nb && c < nb) X[(int64_t)(k0 + r) * d + k0 + c] = Dinv[(int64_t)kb * 4096 + e];
  }
}

constexpr int kInvSplit = 8;   // split of the contraction in the R^-1 column blocks

// Split of the sketch Gram over the s rows: about 256 workgroups of the
// big-tile kernel over the upper 128 x 128 tiles (measured best: d = 1000,
// s = 4000 splits 8 ways, d = 2000, s = 8000 2 ways), each contraction at
// least 512 rows long.
static int gram_ksplit(int s, int d) {
  const int tiles = (d + 127) / 128;
  const int nupper = tiles * (tiles + 1) / 2;
  int ksplit = (256 + nupper - 1) / nupper;
  const int kmax = (s + 511) / 512;
  if (ksplit > kmax) ksplit = kmax;
  return ksplit < 1 ? 1 : ksplit;
}

size_t factor_ws_bytes(int s, int d) {
  const int tiles = (d + 63) / 64;
  const int ksplit = gram_ksplit(s, d);
  const size_t dd = (size_t)d * d;
  return bytes_of<double>(dd) * (ksplit + 1) + bytes_of<double>((size_t)tiles * 4096) +
         bytes_of<double>((size_t)64 * d) + bytes_of<double>(dd) + bytes_of<double>((size_t)kInvSplit * 64 * d);
}

// Full symmetric Gram from the upper-tile split partials: H[i][j] is the
// partials' sum at (min(i, j), max(i, j)), added in split order (the same
// sum as the factored Gram before lambda is added).
__global__ void k_gram_full(const double* __restrict__ parts, int nparts, int64_t stride, int d,
                            double* __restrict__ H) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)d * d) return;
  const int i = (int)(e / d), j = (int)(e - (int64_t)i * d);
  const int64_t src = i <= j ? e : (int64_t)j * d + i;
  double v = 0.0;
  for (int z = 0; z < nparts; ++z) v += parts[z * stride + src];
  H[e] = v;
}

template <class T>
__global__ void k_transpose_f64(const T* __restrict__ A, int rows, int cols, double* __restrict__ AT) {
  __shared__ double t[32][33];
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 256 threads: 8 rows of 32
  for (int r = ty; r < 32; r += 8)
    if (r0 + r < rows && c0 + tx < cols) t[r][tx] = to_f64(A[(int64_t)(r0 + r) * cols + c0 + tx]);
  __syncthreads();
  for (int c = ty; c < 32; c += 8)
    if (c0 + c < cols && r0 + tx < rows) AT[(int64_t)(c0 + c) * rows + r0 + tx] = t[tx][c];
}

int transpose_f64(const double* A, int rows, int cols, double* AT, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return SRP_OK;
  hipLaunchKernelGGL(k_transpose_f64<double>, dim3((cols + 31) / 32, (rows + 31) / 32), dim3(256), 0, st, A, rows,
                     cols, AT);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

int transpose_to_f64(const void* A, int dtype, int rows, int cols, double* AT, hipStream_t st) {
  if (dtype == SRP_F64) return transpose_f64((const double*)A, rows, cols, AT, st);
  if (rows <= 0 || cols <= 0) return SRP_OK;
  hipLaunchKernelGGL(k_transpose_f64<float>, dim3((cols + 31) / 32, (rows + 31) / 32), dim3(256), 0, st,
                     (const float*)A, rows, cols, AT);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

int gram_split(int s, int d0, int d1) {
  const int tiles = ((d0 + 127) / 128) * ((d1 + 127) / 128);
  int ks = (256 + tiles - 1) / tiles;
  const int kmax = (s + 511) / 512;
  if (ks > kmax) ks = kmax;
  return ks < 1 ? 1 : ks;
}

// Events of the calling thread on the current device, reused call after
// call (a wait takes the event's state when it is issued).  Never freed.
static int factor_events(int count, hipEvent_t** out) {
  thread_local std::vector<hipEvent_t>* pools[64] = {};
  int dev = 0;
  SRP_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) { set_error("factor: device %d out of range", dev); return SRP_EDEVICE; }
  if (!pools[dev]) pools[dev] = new std::vector<hipEvent_t>();
  std::vector<hipEvent_t>& pool = *pools[dev];
  while ((int)pool.size() < count) {
    hipEvent_t e = nullptr;
    SRP_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    pool.push_back(e);
  }
  *out = pool.data();
  return SRP_OK;
}

// Column block kb of X = R^-1 (left to right): X_kk = R_kk^-1 (from the
// diagonal block's factor) and X[0:k0, kb] = -X[0:k0, 0:k0] R[0:k0, kb] X_kk.
// It needs only R's columns up to kb and X's earlier column blocks, so it
// runs while the Cholesky works on the columns after kb.
static int rinv_column(int kb, int d, const double* R, const double* Dinv, double* X, double* Tmp, double* Tparts,
                       hipStream_t st) {
  const int k0 = kb * 64, nb = std::min(64, d - k0);
  hipLaunchKernelGGL(k_place_diag_blocks, dim3(1), dim3(256), 0, st, Dinv, d, X, kb);
  SRP_LAUNCH_CHECK();
  if (kb == 0) return SRP_OK;
  const int rows = k0;
  GemmArgs a{};
  a.m = rows; a.n = nb; a.kk = rows; a.alpha = 1.0; a.beta = 0.0;
  a.A = X; a.lda = d; a.ta = false;
  a.B = R + k0; a.ldb = d; a.tb = false;
  const int ks = std::min(kInvSplit, (rows + 127) / 128);
  if (ks > 1) {   // rows x nb outputs are few tiles: split the contraction
    a.C = Tparts; a.ldc = nb; a.ksplit = ks; a.c_split_stride = (int64_t)rows * nb;
    SRP_TRY(gemm_f64(a, st));
    SRP_TRY(sum_parts_f64(Tparts, ks, (int64_t)rows * nb, (int64_t)rows * nb, Tmp, 0, 0.0, st));
  } else {
    a.C = Tmp; a.ldc = nb;
    SRP_TRY(gemm_f64(a, st));
  }
  GemmArgs b{};
  b.m = rows; b.n = nb; b.kk = nb; b.alpha = -1.0; b.beta = 0.0;
  b.A = Tmp; b.lda = nb; b.ta = false;
  b.B = Dinv + (size_t)kb * 4096; b.ldb = 64; b.tb = false;
  b.C = X + k0; b.ldc = d;
  return gemm_f64(b, st);
}

int sketch_factor_run(const void* SA, int dtype, int s, int d, double lambda, double* R, double* Rinv,
                      double* Minv, int* flag_dev, Arena& ws, hipStream_t st, double* Hfull, hipStream_t aux) {
  const int tiles = (d + 63) / 64;
  const int ksplit = gram_ksplit(s, d);
  const int64_t dd = (int64_t)d * d;
  double* G = ws.take<double>(dd);
  const bool use_parts = ksplit > 1 || Hfull;
  double* parts = use_parts ? ws.take<double>(dd * ksplit) : nullptr;
  double* Dinv = ws.take<double>((size_t)tiles * 4096);
  double* Tmp = ws.take<double>((size_t)64 * d);
  double* X = Rinv ? Rinv : ws.take<double>(dd);
  double* Tparts = ws.take<double>((size_t)kInvSplit * 64 * d);
  if (!G || !Dinv || !Tmp || !X || !Tparts || (use_parts && !parts)) {
    set_error("sketch_factor: workspace too small");
    return SRP_ENOMEM;
  }
  const bool f32 = (dtype != SRP_F64);
  // Gram of the sketch (upper tiles), split over the s rows.
  GemmArgs g{};
  g.m = d; g.n = d; g.kk = s; g.alpha = 1.0; g.beta = 0.0;
  g.A = SA; g.lda = d; g.ta = true; g.a_f32 = f32;
  g.B = SA; g.ldb = d; g.tb = false; g.b_f32 = f32;
  g.upper_only = true;
  // every upper-tile entry of every split is written by the GEMM, and only
  // those (i <= j) are read: no clearing of the partials
  if (use_parts) {
    g.C = parts; g.ldc = d; g.ksplit = ksplit; g.c_split_stride = dd;
    SRP_TRY(gemm_f64(g, st));
    hipLaunchKernelGGL(k_sum_upper, dim3((unsigned)((dd + 255) / 256)), dim3(256), 0, st, parts, ksplit, dd, d,
                       lambda, G);
    SRP_LAUNCH_CHECK();
    if (Hfull) {
      hipLaunchKernelGGL(k_gram_full, dim3((unsigned)((dd + 255) / 256)), dim3(256), 0, st, parts, ksplit, dd, d,
                         Hfull);
      SRP_LAUNCH_CHECK();
    }
  } else {
    g.C = G; g.ldc = d;
    SRP_TRY(gemm_f64(g, st));
    hipLaunchKernelGGL(k_sum_upper, dim3((unsigned)((dd + 255) / 256)), dim3(256), 0, st, G, 1, dd, d, lambda, G);
    SRP_LAUNCH_CHECK();
  }
  // Right-looking blocked Cholesky, 64-wide panels; column block kb of
  // X = R^-1 follows diagonal block kb, on the second stream when there is
  // one (the same arithmetic either way, so the result does not depend on
  // it).
  const bool overlap = aux != nullptr && aux != st && tiles > 1;
  hipEvent_t* ev = nullptr;
  if (overlap) SRP_TRY(factor_events(tiles + 1, &ev));
  // joins the second stream into st on every return (an error return too,
  // so the caller's stream-ordered release of the workspace follows it)
  struct Join {
    hipStream_t st, aux;
    hipEvent_t e;
    ~Join() {
      if (aux) {
        (void)hipEventRecord(e, aux);
        (void)hipStreamWaitEvent(st, e, 0);
      }
    }
  } join{st, overlap ? aux : nullptr, overlap ? ev[tiles] : nullptr};
  SRP_TRY(fill_f64(R, dd, 0.0, st));
  SRP_TRY(fill_f64(X, dd, 0.0, st));
  for (int kb = 0; kb < tiles; ++kb) {
    const int k0 = kb * 64, nb = min(64, d - k0);
    hipLaunchKernelGGL(k_potrf_block, dim3(1), dim3(256), 0, st, G, (int64_t)d, k0, nb, R,
                       Dinv + (size_t)kb * 4096, flag_dev);
    SRP_LAUNCH_CHECK();
    if (overlap) {
      SRP_HIP(hipEventRecord(ev[kb], st));
      SRP_HIP(hipStreamWaitEvent(aux, ev[kb], 0));
    }
    SRP_TRY(rinv_column(kb, d, R, Dinv, X, Tmp, Tparts, overlap ? aux : st));
    const int rest = d - k0 - nb;
    if (rest <= 0) continue;
    GemmArgs t{};
    t.m = nb; t.n = rest; t.kk = nb; t.alpha = 1.0; t.beta = 0.0;
    t.A = Dinv + (size_t)kb * 4096; t.lda = 64; t.ta = true;
    t.B = G + (int64_t)k0 * d + k0 + nb; t.ldb = d; t.tb = false;
    t.C = R + (int64_t)k0 * d + k0 + nb; t.ldc = d;
    SRP_TRY(gemm_f64(t, st));
    GemmArgs u{};
    u.m = rest; u.n = rest; u.kk = nb; u.alpha = -1.0; u.beta = 1.0;
    u.A = R + (int64_t)k0 * d + k0 + nb; u.lda = d; u.ta = true;
    u.B = R + (int64_t)k0 * d + k0 + nb; u.ldb = d; u.tb = false;
    u.C = G + (int64_t)(k0 + nb) * d + k0 + nb; u.ldc = d;
    u.upper_only = true;
    SRP_TRY(gemm_f64(u, st));
  }
  if (overlap) {   // R^-1 done on the second stream: join it
    join.aux = nullptr;
    SRP_HIP(hipEventRecord(ev[tiles], aux));
    SRP_HIP(hipStreamWaitEvent(st, ev[tiles], 0));
  }
  if (Minv) {
    GemmArgs mm{};
    mm.m = d; mm.n = d; mm.kk = d; mm.alpha = 1.0; mm.beta = 0.0;
    mm.A = X; mm.lda = d; mm.ta = false;
    mm.B = X; mm.ldb = d; mm.tb = true;
    mm.C = Minv; mm.ldc = d;
    SRP_TRY(gemm_f64(mm, st));
  }
  return SRP_OK;
}

}  // namespace srp
