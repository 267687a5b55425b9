// FDA centring (Section 5.1 problem statement and Algorithm LDAopt, step
// "compute S_B and Xhat"): class counts n_k, FP64 class sums, class means
// m_k, the data mean m, Yhat with rows sqrt(n_k)(m_k - m) (so that
// S_B = Yhat^T Yhat), and the materialised within-class data
// Xhat = X - m_{y_i}, each entry formed in FP64 and rounded once to the data
// type.  Class sums are accumulated per column in fixed row order inside
// fixed row chunks and then summed over chunks in order (deterministic).
#include "common.hpp"
#include "kernels.hpp"

namespace srp {

constexpr int kCenterRows = 1024;
constexpr int kCenterMaxC = kLdaMaxClasses;

// Class counts: a histogram per workgroup in LDS, then one atomic add per
// class and workgroup (integer sums: the order does not matter).
__global__ void __launch_bounds__(256) k_lda_counts(const int32_t* __restrict__ y, int64_t n, int c, int* counts,
                                                    int* bad) {
  __shared__ int hist[kCenterMaxC];
  for (int q = threadIdx.x; q < c; q += 256) hist[q] = 0;
  __syncthreads();
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) {
    const int l = y[i];
    if (l < 0 || l >= c) atomicOr(bad, 1);
    else atomicAdd(&hist[l], 1);
  }
  __syncthreads();
  for (int q = threadIdx.x; q < c; q += 256)
    if (hist[q]) atomicAdd(&counts[q], hist[q]);
}

// partial[chunk][class][col] = sum of X[i][col] over rows of the chunk with label class.
template <class T>
__global__ void __launch_bounds__(256) k_lda_chunk_sums(const T* __restrict__ X, const int32_t* __restrict__ y,
                                                        int64_t n, int d, int c, double* __restrict__ partial) {
  extern __shared__ double acc_raw[];   // c x 256: sized to the classes present
  double (*acc)[256] = reinterpret_cast<double (*)[256]>(acc_raw);
  const int chunk = blockIdx.x;
  const int col = blockIdx.y * 256 + threadIdx.x;
  for (int q = 0; q < c; ++q) acc[q][threadIdx.x] = 0.0;
  const int64_t r0 = (int64_t)chunk * kCenterRows;
  const int64_t r1 = min(n, r0 + kCenterRows);
  if (col < d) {
    // 16 rows' labels and values loaded together, then added in row order
    int64_t i = r0;
    for (; i + 16 <= r1; i += 16) {
      int l[16];
      double x[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        l[u] = y[i + u];
        x[u] = to_f64(X[(i + u) * d + col]);
      }
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (l[u] >= 0 && l[u] < c) acc[l[u]][threadIdx.x] += x[u];
    }
    for (; i < r1; ++i) {
      const int l = y[i];
      if (l >= 0 && l < c) acc[l][threadIdx.x] += to_f64(X[i * d + col]);
    }
    for (int q = 0; q < c; ++q) partial[((int64_t)chunk * c + q) * d + col] = acc[q][threadIdx.x];
  }
}

// Class sums over the chunks, in chunk order (16 chunks' loads in flight),
// and class means; one thread per (class, column).  The sums go to Yhat,
// which k_lda_yhat then overwrites.
__global__ void __launch_bounds__(256) k_lda_class_sums(const double* __restrict__ partial, int nchunks,
                                                        const int* __restrict__ counts, int d, int c,
                                                        double* __restrict__ means, double* __restrict__ sums) {
  const int64_t e = blockIdx.x * 256ll + threadIdx.x;
  if (e >= (int64_t)c * d) return;
  const int q = (int)(e / d);
  double s = 0.0;
  for (int z0 = 0; z0 < nchunks; z0 += 16) {
    double t[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) t[u] = partial[(int64_t)(z0 + u < nchunks ? z0 + u : 0) * c * d + e];
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (z0 + u < nchunks) s += t[u];
  }
  sums[e] = s;
  means[e] = counts[q] > 0 ? s / counts[q] : 0.0;
}

// Data mean (class sums added in class order) and Yhat; one thread per column.
__global__ void k_lda_yhat(const int* __restrict__ counts, int64_t n, int d, int c, const double* __restrict__ means,
                           double* __restrict__ Yhat) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= d) return;
  double total = 0.0;
  for (int q = 0; q < c; ++q) total += Yhat[(int64_t)q * d + col];
  const double m = total / (double)n;
  for (int q = 0; q < c; ++q)
    Yhat[(int64_t)q * d + col] = sqrt((double)counts[q]) * (means[(int64_t)q * d + col] - m);
}

template <class T> __device__ __forceinline__ T from_f64(double v);
template <> __device__ __forceinline__ double from_f64<double>(double v) { return v; }
template <> __device__ __forceinline__ float from_f64<float>(double v) { return (float)v; }
template <> __device__ __forceinline__ bf16 from_f64<bf16>(double v) { return __float2bfloat16((float)v); }

// One workgroup per row: the row's label is read once, its class mean row
// (in L2) is subtracted column by column.  A label out of range (already
// flagged by k_lda_counts, which fails the solve) reads class 0's row.
template <class T>
__global__ void __launch_bounds__(256) k_lda_center(const T* __restrict__ X, const int32_t* __restrict__ y,
                                                    int64_t n, int d, int c, const double* __restrict__ means,
                                                    T* __restrict__ Xhat) {
  const int64_t i = blockIdx.x;
  if (i >= n) return;
  const int l = y[i];
  const double* __restrict__ mrow = means + (int64_t)((l >= 0 && l < c) ? l : 0) * d;
  const T* __restrict__ xr = X + i * d;
  T* __restrict__ hr = Xhat + i * d;
  for (int col = threadIdx.x; col < d; col += 256) hr[col] = from_f64<T>(to_f64(xr[col]) - mrow[col]);
}

size_t lda_center_ws_bytes(int64_t n, int d, int c) {
  const int64_t nchunks = (n + kCenterRows - 1) / kCenterRows;
  return bytes_of<double>((size_t)nchunks * c * d) + bytes_of<double>((size_t)c * d);
}

template <class T>
static int lda_center_t(const T* X, const int32_t* y, int64_t n, int d, int c, T* Xhat, double* Yhat,
                        int* counts, int* bad, Arena& ws, hipStream_t st) {
  if (n > 0x7fffffffll) {
    set_error("lda: at most 2^31 - 1 rows");
    return SRP_EINVAL;
  }
  const int nchunks = (int)((n + kCenterRows - 1) / kCenterRows);
  double* partial = ws.take<double>((size_t)nchunks * c * d);
  double* means = ws.take<double>((size_t)c * d);
  if (!means) { set_error("lda: workspace too small"); return SRP_ENOMEM; }
  SRP_TRY(fill_i32(counts, c, 0, st));
  SRP_TRY(fill_i32(bad, 1, 0, st));
  hipLaunchKernelGGL(k_lda_counts, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, y, n, c, counts, bad);
  SRP_LAUNCH_CHECK();
  const size_t lds = (size_t)c * 256 * sizeof(double);
  SRP_TRY(allow_dynamic_lds((const void*)k_lda_chunk_sums<T>, lds));
  hipLaunchKernelGGL((k_lda_chunk_sums<T>), dim3(nchunks, (d + 255) / 256), dim3(256), lds, st, X, y, n, d, c, partial);
  SRP_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_lda_class_sums, dim3((unsigned)(((int64_t)c * d + 255) / 256)), dim3(256), 0, st, partial,
                     nchunks, counts, d, c, means, Yhat);
  SRP_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_lda_yhat, dim3((d + 255) / 256), dim3(256), 0, st, counts, n, d, c, means, Yhat);
  SRP_LAUNCH_CHECK();
  hipLaunchKernelGGL((k_lda_center<T>), dim3((unsigned)n), dim3(256), 0, st, X, y, n, d, c, means, Xhat);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

int lda_center_run(const void* X, const int32_t* labels, int dtype, int64_t n, int d, int c, void* Xhat,
                   double* Yhat, int* counts, int* bad, Arena& ws, hipStream_t st) {
  if (c > kCenterMaxC) {
    set_error("lda: at most %d classes supported", kCenterMaxC);
    return SRP_EINVAL;
  }
  switch (dtype) {
    case SRP_F64: return lda_center_t((const double*)X, labels, n, d, c, (double*)Xhat, Yhat, counts, bad, ws, st);
    case SRP_F32: return lda_center_t((const float*)X, labels, n, d, c, (float*)Xhat, Yhat, counts, bad, ws, st);
    case SRP_BF16: return lda_center_t((const bf16*)X, labels, n, d, c, (bf16*)Xhat, Yhat, counts, bad, ws, st);
  }
  set_error("lda: bad dtype %d", dtype);
  return SRP_EINVAL;
}

}  // namespace srp
