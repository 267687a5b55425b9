// Reduced-precision staging of the tall data: the BF16 and FP8 E4M3 copies
// that the low-precision forms of the sketch and of the data passes read.
//
//  * BF16: round to nearest even on the 16 discarded bits of the FP32 value;
//    a NaN stays a quiet NaN with its sign and upper payload.
//  * FP8 E4M3 (OCP; bias 7, 3 mantissa bits, no infinities, 448 largest):
//    each column j is scaled by the smallest power of two 2^e_j with
//    max_i |x_ij| <= 448 2^e_j (exact comparisons), then every entry is
//    rounded to the nearest E4M3 value, ties to the even mantissa,
//    saturating at +-448.  Undoing a power-of-two scale is exact, so a
//    sketch of the codes times the column scales equals the sketch of the
//    staged matrix.
#include "common.hpp"
#include "kernels.hpp"

#include <cmath>

namespace srp {

__global__ void k_stage_bf16(const float* __restrict__ X, int64_t count, uint16_t* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= count) return;
  out[i] = bf16_rne_bits(X[i]);
}

// Column maxima of |x|: non-negative floats order like their bit patterns,
// so an integer atomic max gives the exact (order-independent) maximum.
template <class T>
__global__ void __launch_bounds__(256) k_col_amax(const T* __restrict__ X, int64_t n, int d, int rows_per_block,
                                                  uint32_t* __restrict__ amax_bits) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= d) return;
  const int64_t r0 = (int64_t)blockIdx.y * rows_per_block;
  const int64_t r1 = min<int64_t>(n, r0 + rows_per_block);
  float m = 0.f;
  for (int64_t r = r0; r < r1; ++r) m = fmaxf(m, fabsf(load_as<float>(X + r * d + c)));
  atomicMax(&amax_bits[c], __float_as_uint(m));
}

__global__ void k_fp8_scales(const uint32_t* __restrict__ amax_bits, int d, double* __restrict__ scales,
                             float* __restrict__ inv_scales) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= d) return;
  const double a = (double)__uint_as_float(amax_bits[c]);
  int e = 0;
  if (a > 0.0) {
    e = (int)ceil(log2(a / 448.0));
    while (a > 448.0 * ldexp(1.0, e)) ++e;
    while (a <= 448.0 * ldexp(1.0, e - 1)) --e;
  }
  scales[c] = ldexp(1.0, e);
  inv_scales[c] = ldexpf(1.0f, -e);
}

// Nearest E4M3 code of v (ties to even mantissa, saturating at +-448).
__device__ __forceinline__ uint8_t fp8_e4m3_encode(float v) {
  const uint32_t u = __float_as_uint(v);
  const uint8_t sign = (uint8_t)((u >> 24) & 0x80u);
  const float a = fabsf(v);
  if (!(a < 448.0f)) return sign | 0x7E;   // 448 = (1 + 6/8) 2^8
  if (a < 0.015625f) {                     // below 2^-6: subnormal grid of 2^-9
    const int m = (int)rintf(a * 512.0f);  // exact scaling, ties to even
    if (m == 0) return 0;
    return sign | (uint8_t)(m >= 8 ? 0x08 : m);
  }
  int E = (int)((u >> 23) & 0xFF) - 127;   // -6 .. 8
  const uint32_t m23 = u & 0x7FFFFFu;
  uint32_t r = m23 >> 20;
  const uint32_t rem = m23 & 0xFFFFFu;
  if (rem > 0x80000u || (rem == 0x80000u && (r & 1u))) ++r;
  if (r == 8) { r = 0; ++E; }
  if (E > 8 || (E == 8 && r == 7)) return sign | 0x7E;
  return sign | (uint8_t)(((E + 7) << 3) | r);
}

template <class T>
__global__ void __launch_bounds__(256) k_stage_fp8(const T* __restrict__ X, int64_t n, int d, int rows_per_block,
                                                   const float* __restrict__ inv_scales, uint8_t* __restrict__ out) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= d) return;
  const float is = inv_scales[c];
  const int64_t r0 = (int64_t)blockIdx.y * rows_per_block;
  const int64_t r1 = min<int64_t>(n, r0 + rows_per_block);
  for (int64_t r = r0; r < r1; ++r) out[r * d + c] = fp8_e4m3_encode(load_as<float>(X + r * d + c) * is);
}

__global__ void k_scale_cols(float* __restrict__ A, int64_t rows, int d, const double* __restrict__ scales) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= d) return;
  const float sc = (float)scales[c];   // a power of two: the product is exact
  for (int64_t r = blockIdx.y; r < rows; r += gridDim.y) A[r * d + c] *= sc;
}

int stage_bf16_run(const float* X, int64_t n, int d, uint16_t* out, hipStream_t st) {
  const int64_t count = n * (int64_t)d;
  if (count <= 0) return SRP_OK;
  hipLaunchKernelGGL(k_stage_bf16, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, X, count, out);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

size_t stage_fp8_ws_bytes(int d) { return bytes_of<uint32_t>(d) + bytes_of<float>(d); }

template <class T>
static int stage_fp8_t(const T* X, int64_t n, int d, uint8_t* out, double* scales, Arena& ws, hipStream_t st) {
  uint32_t* amax = ws.take<uint32_t>(d);
  float* inv = ws.take<float>(d);
  if (!amax || !inv) { set_error("stage_fp8: workspace too small"); return SRP_ENOMEM; }
  SRP_TRY(fill_i32((int*)amax, d, 0, st));
  const int rpb = 2048;
  dim3 g1((d + 255) / 256, (unsigned)((n + rpb - 1) / rpb));
  hipLaunchKernelGGL((k_col_amax<T>), g1, dim3(256), 0, st, X, n, d, rpb, amax);
  SRP_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_fp8_scales, dim3((d + 255) / 256), dim3(256), 0, st, amax, d, scales, inv);
  SRP_LAUNCH_CHECK();
  const int rq = 256;
  dim3 g2((d + 255) / 256, (unsigned)((n + rq - 1) / rq));
  hipLaunchKernelGGL((k_stage_fp8<T>), g2, dim3(256), 0, st, X, n, d, rq, inv, out);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

int stage_fp8_run(const void* X, int dtype, int64_t n, int d, uint8_t* out, double* scales, Arena& ws,
                  hipStream_t st) {
  if (dtype == SRP_F32) return stage_fp8_t((const float*)X, n, d, out, scales, ws, st);
  if (dtype == SRP_BF16) return stage_fp8_t((const bf16*)X, n, d, out, scales, ws, st);
  set_error("stage_fp8: data must be F32 or BF16");
  return SRP_EINVAL;
}

int scale_cols_run(float* A, int64_t rows, int d, const double* scales, hipStream_t st) {
  if (rows <= 0 || d <= 0) return SRP_OK;
  const unsigned gy = (unsigned)std::min<int64_t>(rows, 1024);
  hipLaunchKernelGGL(k_scale_cols, dim3((d + 255) / 256, gy), dim3(256), 0, st, A, rows, d, scales);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

}  // namespace srp
