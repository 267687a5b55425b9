// Internal helpers shared by the HIP sources of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/srp.h"

namespace srp {

// ----------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
void clear_error();

struct Status {
  int code = SRP_OK;
  bool ok() const { return code == SRP_OK; }
};

#define SRP_HIP(expr)                                                      \
  do {                                                                     \
    hipError_t e_ = (expr);                                                \
    if (e_ != hipSuccess) {                                                \
      ::srp::set_error("%s failed: %s (%s:%d)", #expr,                     \
                       hipGetErrorString(e_), __FILE__, __LINE__);         \
      return (e_ == hipErrorOutOfMemory) ? SRP_ENOMEM : SRP_EDEVICE;       \
    }                                                                      \
  } while (0)

#define SRP_TRY(expr)                                                      \
  do {                                                                     \
    int rc_ = (expr);                                                      \
    if (rc_ != SRP_OK) return rc_;                                         \
  } while (0)

#define SRP_REQUIRE(cond, ...)                                             \
  do {                                                                     \
    if (!(cond)) {                                                         \
      ::srp::set_error(__VA_ARGS__);                                       \
      return SRP_EINVAL;                                                   \
    }                                                                      \
  } while (0)

// Launch check: picks up configuration errors right after a launch.
#define SRP_LAUNCH_CHECK() SRP_HIP(hipGetLastError())

// ------------------------------------------------------------ element io
using bf16 = __hip_bfloat16;

template <class T> __device__ __forceinline__ double to_f64(T v);
template <> __device__ __forceinline__ double to_f64<double>(double v) { return v; }
template <> __device__ __forceinline__ double to_f64<float>(float v) { return (double)v; }
template <> __device__ __forceinline__ double to_f64<bf16>(bf16 v) {
  return (double)__bfloat162float(v);
}
template <class T> __device__ __forceinline__ float to_f32(T v);
template <> __device__ __forceinline__ float to_f32<double>(double v) { return (float)v; }
template <> __device__ __forceinline__ float to_f32<float>(float v) { return v; }
template <> __device__ __forceinline__ float to_f32<bf16>(bf16 v) { return __bfloat162float(v); }

template <class CT, class T> __device__ __forceinline__ CT load_as(const T* p);
template <> __device__ __forceinline__ double load_as<double, double>(const double* p) { return *p; }
template <> __device__ __forceinline__ double load_as<double, float>(const float* p) { return (double)*p; }
template <> __device__ __forceinline__ double load_as<double, bf16>(const bf16* p) { return to_f64(*p); }
template <> __device__ __forceinline__ float load_as<float, float>(const float* p) { return *p; }
template <> __device__ __forceinline__ float load_as<float, bf16>(const bf16* p) { return to_f32(*p); }
template <> __device__ __forceinline__ float load_as<float, double>(const double* p) { return (float)*p; }

// BF16 bits of v: round to nearest, ties to even, on the 16 discarded bits
// (adding 0x7FFF plus the kept lowest bit carries into the kept bits exactly
// when the discarded part is above half, or at half with an odd kept part;
// a carry out of the largest finite value gives the infinity pattern).  A
// NaN keeps its sign and upper payload with the quiet bit set.
__device__ __forceinline__ uint16_t bf16_rne_bits(float v) {
  const uint32_t u = __float_as_uint(v);
  if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((u >> 16) | 0x40u);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// FP8 E4M3 code (OCP: bias 7, 3 mantissa bits, no infinities).
struct fp8e4m3 {
  uint8_t v;
};
__device__ __forceinline__ float fp8_to_f32(fp8e4m3 c) {
  const int e = (c.v >> 3) & 15, m = c.v & 7;
  const float mag = e ? ldexpf(1.0f + 0.125f * (float)m, e - 7) : 0.001953125f * (float)m;
  return (c.v & 0x80) ? -mag : mag;
}
template <> __device__ __forceinline__ float load_as<float, fp8e4m3>(const fp8e4m3* p) { return fp8_to_f32(*p); }
template <> __device__ __forceinline__ double load_as<double, fp8e4m3>(const fp8e4m3* p) {
  return (double)fp8_to_f32(*p);
}

inline size_t dtype_size(int dtype) {
  return dtype == SRP_F64 ? 8 : dtype == SRP_F32 ? 4 : dtype == SRP_BF16 ? 2 : 1;
}

// ------------------------------------------------- counter-based hashing
// i-th output (0-based) of SplitMix64 seeded with `seed` (Steele, Lea and
// Flood 2014): state advanced by the golden gamma, then the mix.
__host__ __device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
constexpr uint64_t kSrhtSignSalt = 0x5352485444494147ull;
constexpr uint64_t kSrhtRowSalt = 0x535248545357524Full;

__host__ __device__ __forceinline__ int cs_bucket(uint64_t w, int s) {
  return (int)(((w >> 32) * (uint64_t)s) >> 32);
}
__host__ __device__ __forceinline__ float cs_sign(uint64_t w) {
  return (w & 1ull) ? -1.0f : 1.0f;
}

// --------------------------------------------------------- MFMA helpers
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// 16x16x4 products; operand lane layout (both precisions):
//   A[m][k]: m = lane % 16, k = lane / 16;  B[k][n]: n = lane % 16, k = lane / 16.
// Result row index of accumulator element r (column n = lane % 16):
//   f32: m = 4 * (lane / 16) + r;   f64: m = lane / 16 + 4 * r.
__device__ __forceinline__ f32x4 mfma16x16x4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma16x16x4(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
template <class CT> struct Acc4;
template <> struct Acc4<float> { using type = f32x4; };
template <> struct Acc4<double> { using type = f64x4; };

template <class CT> __device__ __forceinline__ int acc_row(int lane, int r);
template <> __device__ __forceinline__ int acc_row<float>(int lane, int r) { return 4 * (lane >> 4) + r; }
template <> __device__ __forceinline__ int acc_row<double>(int lane, int r) { return (lane >> 4) + 4 * r; }

// Buffer loads: a scalar base (the row block) plus a 32-bit lane offset;
// offsets at or past num_records read as zero, which pads the last row
// block and masked lanes without branches.
constexpr uint32_t kBufDword3 = 0x00020000u;   // raw buffer, gfx9 family
constexpr int kOob = 0x40000000;                 // lane offset that always reads zero

template <class T> __device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, int voff, int soff);
template <> __device__ __forceinline__ float buf_load<float>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <> __device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <> __device__ __forceinline__ bf16 buf_load<bf16>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(bf16, __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0));
}
// An element of type T at byte offset off of a buffer, converted to Acc
// (offsets past the resource read as zero).
template <class Acc, class T> __device__ __forceinline__ Acc buf_load_as(__amdgpu_buffer_rsrc_t r, int off);
template <> __device__ __forceinline__ float buf_load_as<float, float>(__amdgpu_buffer_rsrc_t r, int off) {
  return buf_load<float>(r, off, 0);
}
template <> __device__ __forceinline__ double buf_load_as<double, double>(__amdgpu_buffer_rsrc_t r, int off) {
  return buf_load<double>(r, off, 0);
}
template <> __device__ __forceinline__ double buf_load_as<double, float>(__amdgpu_buffer_rsrc_t r, int off) {
  return (double)buf_load<float>(r, off, 0);
}
template <> __device__ __forceinline__ float buf_load_as<float, bf16>(__amdgpu_buffer_rsrc_t r, int off) {
  return to_f32(buf_load<bf16>(r, off, 0));
}
template <> __device__ __forceinline__ double buf_load_as<double, bf16>(__amdgpu_buffer_rsrc_t r, int off) {
  return to_f64(buf_load<bf16>(r, off, 0));
}
template <> __device__ __forceinline__ float buf_load_as<float, fp8e4m3>(__amdgpu_buffer_rsrc_t r, int off) {
  return fp8_to_f32(fp8e4m3{(uint8_t)__builtin_amdgcn_raw_buffer_load_b8(r, off, 0, 0)});
}
template <> __device__ __forceinline__ double buf_load_as<double, fp8e4m3>(__amdgpu_buffer_rsrc_t r, int off) {
  return (double)buf_load_as<float, fp8e4m3>(r, off);
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, int64_t bytes) {
  const int nrec = (int)(bytes < 0x7ffff000ll ? bytes : 0x7ffff000ll);
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, nrec, (int)kBufDword3);
}

// ------------------------------------------------------------ workspace
// Bump allocator over one stream-ordered allocation.
struct Arena {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  template <class T> T* take(size_t count) {
    size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
    if (used + bytes > cap) return nullptr;
    T* p = reinterpret_cast<T*>(base + used);
    used += bytes;
    return p;
  }
};

// Sizes in bytes with 256-byte rounding (mirrors Arena::take).
template <class T> inline size_t bytes_of(size_t count) {
  return (count * sizeof(T) + 255) & ~size_t(255);
}

int device_alloc(void** p, size_t bytes, hipStream_t s);
int device_free(void* p, hipStream_t s);
int num_cus();
// Raises the dynamic-LDS limit of kernel `fn` on the current device to at
// least `bytes`.  Thread-safe; the limit only grows, so launches made by
// other threads with smaller requests stay valid.
int allow_dynamic_lds(const void* fn, size_t bytes);

}  // namespace srp
