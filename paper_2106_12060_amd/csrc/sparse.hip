// Sparse (CSR) data: the O(nnz) CountSketch of Section 3 and the
// per-iteration products of Algorithms CCAopt / LDAopt as sparse-times-
// skinny products, whose cost the paper states in terms of nnz(X) and
// nnz(Y) (Section 3, Table costs; Section 4.5 and 5.5 cost remarks).
//
// Input: row-major CSR (row pointers int64, column indices int32 strictly
// increasing within a row, values F32 or F64).  The products A W read the
// rows.  The products A^T P read the columns: a CSC copy is built once per
// solve by a stable counting sort (column histograms per chunk of rows, a
// scan per column over the chunks, placement row by row inside a chunk),
// so every column lists its rows in ascending order.  Every output is then
// a sum in a fixed order (the kernels are bitwise reproducible), and with
// the zero entries left out it is the same sum, in the same order, as over
// the dense matrix.  All arithmetic is FP64.
#include "common.hpp"
#include "kernels.hpp"

#include <cmath>

namespace srp {

constexpr int kCscChunkMax = 4096;   // largest chunk of rows in the CSC build
// Entries per segment of a column in the products A^T P.
constexpr int kCscSeg = 256;

// ------------------------------------------------------- validation
// Every row: 0 <= ptr[i] <= ptr[i+1] <= nnz, ptr[0] = 0, ptr[n] = nnz,
// columns in [0, d) and strictly increasing.  Entries are only read inside
// [0, nnz), whatever the pointers hold.
__global__ void k_csr_check(int64_t n, int d, int64_t nnz, const int64_t* __restrict__ ptr,
                            const int32_t* __restrict__ idx, int* bad) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t p0 = ptr[i], p1 = ptr[i + 1];
  bool ok = p0 >= 0 && p0 <= p1 && p1 <= nnz && (i != 0 || p0 == 0) && (i != n - 1 || p1 == nnz);
  if (ok) {
    int prev = -1;
    for (int64_t e = p0; e < p1; ++e) {
      const int j = idx[e];
      if (j <= prev || j >= d) { ok = false; break; }
      prev = j;
    }
  }
  if (!ok) atomicOr(bad, 1);
}

int csr_validate(const CsrView& A, int* bad, hipStream_t st) {
  const unsigned blocks = (unsigned)((A.n + 255) / 256);
  hipLaunchKernelGGL(k_csr_check, dim3(blocks), dim3(256), 0, st, A.n, A.d, A.nnz, A.ptr, A.idx, bad);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

// ------------------------------------------------------- CSC build
__global__ void __launch_bounds__(256) k_csc_chunk_count(int64_t n, int d, int chunk_rows,
                                                         const int64_t* __restrict__ ptr,
                                                         const int32_t* __restrict__ idx, int* chunk_cnt) {
  extern __shared__ int cnt[];
  const int ch = blockIdx.x;
  for (int j = threadIdx.x; j < d; j += blockDim.x) cnt[j] = 0;
  __syncthreads();
  const int64_t r0 = (int64_t)ch * chunk_rows, r1 = min(n, r0 + chunk_rows);
  const int64_t e0 = ptr[r0], e1 = ptr[r1];
  for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) atomicAdd(&cnt[idx[e]], 1);
  __syncthreads();
  for (int j = threadIdx.x; j < d; j += blockDim.x) chunk_cnt[(int64_t)ch * d + j] = cnt[j];
}

// Per column: the chunk counts become offsets inside the column (exclusive
// scan over the chunks, in chunk order); total[j] = entries of column j.
// Three levels over groups of kCscScanGroup chunks: the groups' sums (one
// thread per group and column), their scan per column, then each group's
// chunks from its offset; every level keeps sixteen loads in flight.
constexpr int kCscScanGroup = 64;

__global__ void k_csc_group_sums(int nchunks, int d, const int* __restrict__ chunk_cnt, int* __restrict__ gsum) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int ngroups = (nchunks + kCscScanGroup - 1) / kCscScanGroup;
  if (t >= (int64_t)ngroups * d) return;
  const int g = (int)(t / d), j = (int)(t - (int64_t)g * d);
  const int c0 = g * kCscScanGroup, c1 = min(nchunks, c0 + kCscScanGroup);
  int sum = 0;
  for (int ch0 = c0; ch0 < c1; ch0 += 16) {
    int v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = ch0 + u < c1 ? chunk_cnt[(int64_t)(ch0 + u) * d + j] : 0;
#pragma unroll
    for (int u = 0; u < 16; ++u) sum += v[u];
  }
  gsum[t] = sum;
}

__global__ void k_csc_group_scan(int ngroups, int d, int* __restrict__ gsum, int* __restrict__ total) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= d) return;
  int run = 0;
  for (int g0 = 0; g0 < ngroups; g0 += 16) {
    int v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = g0 + u < ngroups ? gsum[(int64_t)(g0 + u) * d + j] : 0;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      if (g0 + u < ngroups) gsum[(int64_t)(g0 + u) * d + j] = run;
      run += v[u];
    }
  }
  total[j] = run;
}

__global__ void k_csc_chunk_offsets(int nchunks, int d, const int* __restrict__ gsum, int* __restrict__ chunk_cnt) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int ngroups = (nchunks + kCscScanGroup - 1) / kCscScanGroup;
  if (t >= (int64_t)ngroups * d) return;
  const int g = (int)(t / d), j = (int)(t - (int64_t)g * d);
  const int c0 = g * kCscScanGroup, c1 = min(nchunks, c0 + kCscScanGroup);
  int run = gsum[t];
  for (int ch0 = c0; ch0 < c1; ch0 += 16) {
    int v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = ch0 + u < c1 ? chunk_cnt[(int64_t)(ch0 + u) * d + j] : 0;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      if (ch0 + u < c1) chunk_cnt[(int64_t)(ch0 + u) * d + j] = run;
      run += v[u];
    }
  }
}

// One wave per chunk of rows, in row order: the entries of one row have
// distinct columns, so its lanes bump distinct counters; the barrier after
// each row orders the rows.  The chunk's row pointers are staged in LDS
// first, so a row waits only for its own entries.
template <class T>
__global__ void __launch_bounds__(64) k_csc_place(int64_t n, int d, int chunk_rows, const int64_t* __restrict__ ptr,
                                                  const int32_t* __restrict__ idx, const T* __restrict__ val,
                                                  const int* __restrict__ colptr, const int* __restrict__ chunk_off,
                                                  int32_t* __restrict__ rows_out, T* __restrict__ val_out) {
  extern __shared__ int off[];
  int64_t* rp = reinterpret_cast<int64_t*>(off + ((d + 1) & ~1));   // chunk_rows + 1 row pointers
  const int ch = blockIdx.x;
  const int64_t r0 = (int64_t)ch * chunk_rows, r1 = min(n, r0 + chunk_rows);
  for (int j = threadIdx.x; j < d; j += 64) off[j] = colptr[j] + chunk_off[(int64_t)ch * d + j];
  for (int64_t r = r0 + threadIdx.x; r <= r1; r += 64) rp[r - r0] = ptr[r];
  __syncthreads();
  int64_t e0 = rp[0];
  for (int64_t r = r0; r < r1; ++r) {
    const int64_t e1 = rp[r + 1 - r0];
    for (int64_t e = e0 + threadIdx.x; e < e1; e += 64) {
      const int j = idx[e];
      const int pos = off[j];
      off[j] = pos + 1;
      rows_out[pos] = (int32_t)r;
      val_out[pos] = val[e];
    }
    e0 = e1;
    __syncthreads();
  }
}

// Rows per chunk of the CSC build: 128, doubled while the per-chunk column
// counters (chunks x d) would outnumber twice the entries.
static int csc_chunk_rows(int64_t n, int d, int64_t nnz) {
  int rows = 128;
  while (rows < kCscChunkMax && ((n + rows - 1) / rows) * (int64_t)d > 2 * std::max<int64_t>(nnz, 1)) rows *= 2;
  return rows;
}
static int csc_nchunks(const CsrView& A) {
  const int rows = csc_chunk_rows(A.n, A.d, A.nnz);
  return (int)((A.n + rows - 1) / rows);
}

// Segments of kCscSeg entries per column (a column of m entries has
// ceil(m / kCscSeg) of them): at most nnz / kCscSeg + d in all.
int64_t csc_max_segments(const CsrView& A) { return A.nnz / kCscSeg + A.d + 1; }

__global__ void k_csc_seg_count(int d, const int* __restrict__ colptr, int* __restrict__ nseg) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < d) nseg[j] = (colptr[j + 1] - colptr[j] + kCscSeg - 1) / kCscSeg;
}

__global__ void k_csc_seg_fill(int d, const int* __restrict__ segptr, int* __restrict__ segcol) {
  const int j = blockIdx.x;
  for (int q = segptr[j] + threadIdx.x; q < segptr[j + 1]; q += blockDim.x) segcol[q] = j;
}

size_t csc_bytes(const CsrView& A) {
  return 2 * bytes_of<int>((size_t)A.d + 1) + bytes_of<int32_t>((size_t)A.nnz) +
         ((size_t)A.nnz * dtype_size(A.dtype) + 255) / 256 * 256 + bytes_of<int>((size_t)csc_max_segments(A));
}

size_t csc_scratch_bytes(const CsrView& A) {
  const int ngroups = (csc_nchunks(A) + kCscScanGroup - 1) / kCscScanGroup;
  return bytes_of<int>((size_t)csc_nchunks(A) * A.d) + bytes_of<int>((size_t)ngroups * A.d) +
         bytes_of<int>((size_t)A.d + 1);
}

int csc_build(const CsrView& A, CscView* out, Arena& keep, Arena& scratch, hipStream_t st) {
  out->d = A.d;
  out->nnz = A.nnz;
  out->dtype = A.dtype;
  out->ptr = keep.take<int>((size_t)A.d + 1);
  out->idx = keep.take<int32_t>((size_t)A.nnz);
  out->val = keep.take<char>((size_t)A.nnz * dtype_size(A.dtype));
  out->segptr = keep.take<int>((size_t)A.d + 1);
  out->segcol = keep.take<int>((size_t)csc_max_segments(A));
  const int crows = csc_chunk_rows(A.n, A.d, A.nnz);
  const int nch = csc_nchunks(A);
  const int ngroups = (nch + kCscScanGroup - 1) / kCscScanGroup;
  int* chunk = scratch.take<int>((size_t)nch * A.d);
  int* gsum = scratch.take<int>((size_t)ngroups * A.d);
  int* total = scratch.take<int>((size_t)A.d + 1);
  if (!out->segcol || !total) { set_error("CSC copy: workspace too small"); return SRP_ENOMEM; }
  const size_t lds = sizeof(int) * (size_t)A.d;
  const size_t lds_place = sizeof(int) * (size_t)((A.d + 1) & ~1) + sizeof(int64_t) * ((size_t)crows + 1);
  SRP_TRY(allow_dynamic_lds((const void*)k_csc_chunk_count, lds));
  hipLaunchKernelGGL(k_csc_chunk_count, dim3(nch), dim3(256), lds, st, A.n, A.d, crows, A.ptr, A.idx, chunk);
  SRP_LAUNCH_CHECK();
  const unsigned gthreads = (unsigned)(((int64_t)ngroups * A.d + 255) / 256);
  hipLaunchKernelGGL(k_csc_group_sums, dim3(gthreads), dim3(256), 0, st, nch, A.d, chunk, gsum);
  SRP_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_csc_group_scan, dim3((A.d + 255) / 256), dim3(256), 0, st, ngroups, A.d, gsum, total);
  SRP_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_csc_chunk_offsets, dim3(gthreads), dim3(256), 0, st, nch, A.d, gsum, chunk);
  SRP_LAUNCH_CHECK();
  SRP_TRY(scan_excl_i32(total, A.d, out->ptr, st));
  if (A.dtype == SRP_F64) {
    SRP_TRY(allow_dynamic_lds((const void*)k_csc_place<double>, lds_place));
    hipLaunchKernelGGL(k_csc_place<double>, dim3(nch), dim3(64), lds_place, st, A.n, A.d, crows, A.ptr, A.idx,
                       (const double*)A.val, out->ptr, chunk, out->idx, (double*)out->val);
  } else {
    SRP_TRY(allow_dynamic_lds((const void*)k_csc_place<float>, lds_place));
    hipLaunchKernelGGL(k_csc_place<float>, dim3(nch), dim3(64), lds_place, st, A.n, A.d, crows, A.ptr, A.idx,
                       (const float*)A.val, out->ptr, chunk, out->idx, (float*)out->val);
  }
  SRP_LAUNCH_CHECK();
  // segment tables; the segment count is read back once (it sizes the
  // product launches)
  hipLaunchKernelGGL(k_csc_seg_count, dim3((A.d + 255) / 256), dim3(256), 0, st, A.d, out->ptr, total);
  SRP_LAUNCH_CHECK();
  SRP_TRY(scan_excl_i32(total, A.d, out->segptr, st));
  hipLaunchKernelGGL(k_csc_seg_fill, dim3(A.d), dim3(64), 0, st, A.d, out->segptr, out->segcol);
  SRP_LAUNCH_CHECK();
  int nseg = 0;
  SRP_HIP(hipMemcpyAsync(&nseg, out->segptr + A.d, sizeof(int), hipMemcpyDeviceToHost, st));
  SRP_HIP(hipStreamSynchronize(st));
  out->nseg = nseg;
  return SRP_OK;
}

// ------------------------------------------- sparse rows times dense
// Sum of val[e] * D[idx[e]][c] over the entries e0 <= e < e1 (in stored
// order) for lane c of a group of G lanes: the group loads G entries at a
// time (coalesced), broadcasts them by shuffle, and issues the G gathers
// of D before the G multiply-adds, so the gathers are in flight together.
template <class T, int G>
__device__ __forceinline__ double seg_dot(int64_t e0, int64_t e1, const int32_t* __restrict__ idx,
                                          const T* __restrict__ val, const double* __restrict__ D, int ldd, int w,
                                          int c) {
  double acc = 0.0;
  for (int64_t b = e0; b < e1; b += G) {
    const int64_t e = b + c;
    int j = 0;
    double v = 0.0;
    if (e < e1) {
      j = idx[e];
      v = to_f64(val[e]);
    }
    const int m = (int)min<int64_t>(G, e1 - b);
    double dv[G];
#pragma unroll
    for (int t = 0; t < G; ++t) {
      const int jt = __shfl(j, t, G);
      dv[t] = (t < m && c < w) ? D[(int64_t)jt * ldd + c] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < G; ++t) {
      const double vt = __shfl(v, t, G);
      if (t < m) acc += vt * dv[t];
    }
  }
  return acc;
}

// CSR rows: out[r][c] = sum over row r's entries of val[e] * D[idx[e]][c]
// (c < w), minus sub[labels[r]][c] when labels is set.  A group of G lanes
// owns one row.
template <class T, int G>
__global__ void __launch_bounds__(256) k_spmm_rows(int64_t rows, const int64_t* __restrict__ ptr,
                                                   const int32_t* __restrict__ idx, const T* __restrict__ val,
                                                   const double* __restrict__ D, int ldd, int w,
                                                   double* __restrict__ out, int ldo, const double* __restrict__ sub,
                                                   const int32_t* __restrict__ labels, const int* __restrict__ done) {
  if (done && *done) return;
  const int lane = threadIdx.x & 63, g = lane / G, c = lane % G;
  const int64_t r = ((int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64) * (64 / G) + g;
  if (r >= rows) return;   // uniform over the group: shuffles stay inside active groups
  double acc = seg_dot<T, G>(ptr[r], ptr[r + 1], idx, val, D, ldd, w, c);
  if (c < w) {
    if (labels) acc -= sub[(int64_t)labels[r] * w + c];
    out[r * ldo + c] = acc;
  }
}

// CSC columns, stage 1: segment q (kCscSeg entries of column segcol[q] at
// most) gives partial[q][c].
template <class T, int G>
__global__ void __launch_bounds__(256) k_spmm_segs(int nseg, const int* __restrict__ colptr,
                                                   const int* __restrict__ segptr, const int* __restrict__ segcol,
                                                   const int32_t* __restrict__ idx, const T* __restrict__ val,
                                                   const double* __restrict__ D, int ldd, int w,
                                                   double* __restrict__ partial, const int* __restrict__ done) {
  if (done && *done) return;
  const int lane = threadIdx.x & 63, g = lane / G, c = lane % G;
  const int64_t q = ((int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64) * (64 / G) + g;
  if (q >= nseg) return;
  const int j = segcol[q];
  const int64_t e0 = colptr[j] + (int64_t)(q - segptr[j]) * kCscSeg;
  const int64_t e1 = min<int64_t>(colptr[j + 1], e0 + kCscSeg);
  const double acc = seg_dot<T, G>(e0, e1, idx, val, D, ldd, w, c);
  if (c < w) partial[q * w + c] = acc;
}

// Stage 2: out[j][c] = sum of column j's segment partials.  One workgroup
// per column: W lanes per slice (W >= w), 256 / W slices; slice l adds
// segments l, l + 256/W, ... in order, then slice 0 adds the slices'
// sums in slice order (a fixed order: bitwise reproducible).
template <int W>
__global__ void __launch_bounds__(256) k_spmm_seg_sum(int w, const int* __restrict__ segptr,
                                                      const double* __restrict__ partial, double* __restrict__ out,
                                                      int ldo, const int* __restrict__ done) {
  if (done && *done) return;
  constexpr int SL = 256 / W;
  __shared__ double red[SL][W];
  const int j = blockIdx.x, c = threadIdx.x % W, l = threadIdx.x / W;
  double acc = 0.0;
  if (c < w)
    for (int q = segptr[j] + l; q < segptr[j + 1]; q += SL) acc += partial[(int64_t)q * w + c];
  red[l][c] = acc;
  __syncthreads();
  if (l == 0 && c < w) {
    double s = 0.0;
    for (int t = 0; t < SL; ++t) s += red[t][c];
    out[(int64_t)j * ldo + c] = s;
  }
}

template <class T>
static int spmm_rows_launch(int64_t rows, const int64_t* ptr, const int32_t* idx, const T* val, const double* D,
                            int ldd, int w, double* out, int ldo, const double* sub, const int32_t* labels,
                            const int* done, hipStream_t st) {
  auto grid = [&](int G) { return dim3((unsigned)((rows + (4 * (64 / G)) - 1) / (4 * (64 / G)))); };
  if (w <= 8) hipLaunchKernelGGL((k_spmm_rows<T, 8>), grid(8), dim3(256), 0, st, rows, ptr, idx, val, D, ldd, w,
                                 out, ldo, sub, labels, done);
  else if (w <= 16) hipLaunchKernelGGL((k_spmm_rows<T, 16>), grid(16), dim3(256), 0, st, rows, ptr, idx, val, D,
                                       ldd, w, out, ldo, sub, labels, done);
  else if (w <= 32) hipLaunchKernelGGL((k_spmm_rows<T, 32>), grid(32), dim3(256), 0, st, rows, ptr, idx, val, D,
                                       ldd, w, out, ldo, sub, labels, done);
  else hipLaunchKernelGGL((k_spmm_rows<T, 64>), grid(64), dim3(256), 0, st, rows, ptr, idx, val, D, ldd, w, out,
                          ldo, sub, labels, done);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

template <class T>
static int spmm_segs_launch(const CscView& A, const T* val, const double* D, int ldd, int w, double* partial,
                            const int* done, hipStream_t st) {
  const int64_t n = A.nseg;
  auto grid = [&](int G) { return dim3((unsigned)((n + (4 * (64 / G)) - 1) / (4 * (64 / G)))); };
  if (w <= 8) hipLaunchKernelGGL((k_spmm_segs<T, 8>), grid(8), dim3(256), 0, st, A.nseg, A.ptr, A.segptr, A.segcol,
                                 A.idx, val, D, ldd, w, partial, done);
  else if (w <= 16) hipLaunchKernelGGL((k_spmm_segs<T, 16>), grid(16), dim3(256), 0, st, A.nseg, A.ptr, A.segptr,
                                       A.segcol, A.idx, val, D, ldd, w, partial, done);
  else if (w <= 32) hipLaunchKernelGGL((k_spmm_segs<T, 32>), grid(32), dim3(256), 0, st, A.nseg, A.ptr, A.segptr,
                                       A.segcol, A.idx, val, D, ldd, w, partial, done);
  else hipLaunchKernelGGL((k_spmm_segs<T, 64>), grid(64), dim3(256), 0, st, A.nseg, A.ptr, A.segptr, A.segcol,
                          A.idx, val, D, ldd, w, partial, done);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

int csr_times_dense(const CsrView& A, const double* D, int ldd, int w, double* out, int ldo, const double* sub,
                    const int32_t* labels, const int* done, hipStream_t st) {
  SRP_REQUIRE(w >= 1 && w <= 64, "sparse product width %d outside 1..64", w);
  if (A.n <= 0) return SRP_OK;
  if (A.dtype == SRP_F64)
    return spmm_rows_launch(A.n, A.ptr, A.idx, (const double*)A.val, D, ldd, w, out, ldo, sub, labels, done, st);
  return spmm_rows_launch(A.n, A.ptr, A.idx, (const float*)A.val, D, ldd, w, out, ldo, sub, labels, done, st);
}

size_t csc_partial_bytes(const CsrView& A, int w) {
  return bytes_of<double>((size_t)csc_max_segments(A) * w);
}

int csc_times_dense(const CscView& A, const double* D, int ldd, int w, double* out, int ldo, double* partial,
                    const int* done, hipStream_t st) {
  SRP_REQUIRE(w >= 1 && w <= 64, "sparse product width %d outside 1..64", w);
  if (A.d <= 0) return SRP_OK;
  if (A.nseg > 0) {
    if (A.dtype == SRP_F64) SRP_TRY(spmm_segs_launch(A, (const double*)A.val, D, ldd, w, partial, done, st));
    else SRP_TRY(spmm_segs_launch(A, (const float*)A.val, D, ldd, w, partial, done, st));
  }
  if (w <= 8) hipLaunchKernelGGL(k_spmm_seg_sum<8>, dim3(A.d), dim3(256), 0, st, w, A.segptr, partial, out, ldo, done);
  else if (w <= 16) hipLaunchKernelGGL(k_spmm_seg_sum<16>, dim3(A.d), dim3(256), 0, st, w, A.segptr, partial, out, ldo,
                                       done);
  else if (w <= 32) hipLaunchKernelGGL(k_spmm_seg_sum<32>, dim3(A.d), dim3(256), 0, st, w, A.segptr, partial, out, ldo,
                                       done);
  else hipLaunchKernelGGL(k_spmm_seg_sum<64>, dim3(A.d), dim3(256), 0, st, w, A.segptr, partial, out, ldo, done);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

// ------------------------------------------------- CSR CountSketch
// One workgroup per bucket; its rows (ascending) are added into an LDS row
// of d doubles, one row at a time (a row's columns are distinct, so its
// threads write distinct words; the barrier orders the rows).  With labels,
// the bucket's signed class counts (S E for the one-hot E) ride along.
template <class T>
__global__ void __launch_bounds__(256) k_cs_csr(int d, uint64_t seed, const int* __restrict__ offsets,
                                                const int* __restrict__ sorted, const int64_t* __restrict__ ptr,
                                                const int32_t* __restrict__ idx, const T* __restrict__ val,
                                                double* __restrict__ out, const int32_t* __restrict__ labels, int c,
                                                double* __restrict__ se) {
  extern __shared__ double acc[];
  const int b = blockIdx.x;
  const int w = d + (labels ? c : 0);
  for (int j = threadIdx.x; j < w; j += blockDim.x) acc[j] = 0.0;
  __syncthreads();
  const int beg = offsets[b], cnt = offsets[b + 1] - beg;
  for (int q = 0; q < cnt; ++q) {
    const int row = sorted[beg + q];
    const double g = (double)cs_sign(splitmix64(seed, (uint64_t)row));
    const int64_t e0 = ptr[row], e1 = ptr[row + 1];
    for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) acc[idx[e]] += g * to_f64(val[e]);
    if (labels && threadIdx.x == 0) acc[d + labels[row]] += g;
    __syncthreads();
  }
  for (int j = threadIdx.x; j < d; j += blockDim.x) out[(int64_t)b * d + j] = acc[j];
  if (labels)
    for (int j = threadIdx.x; j < c; j += blockDim.x) se[(int64_t)b * c + j] = acc[d + j];
}

size_t countsketch_csr_ws_bytes(int64_t n, int s) { return countsketch_ws_bytes(n, s); }

int countsketch_csr_run(const CsrView& A, int s, uint64_t seed, double* out, const int32_t* labels, int c,
                        double* se, Arena& ws, hipStream_t st) {
  SRP_REQUIRE(A.d <= kCsrMaxCols, "CSR input wider than %d columns", kCsrMaxCols);
  const int* offsets = nullptr;
  const int* sorted = nullptr;
  SRP_TRY(countsketch_buckets(A.n, s, seed, ws, &offsets, &sorted, st));
  const size_t lds = sizeof(double) * (size_t)(A.d + (labels ? c : 0));
  if (A.dtype == SRP_F64) {
    SRP_TRY(allow_dynamic_lds((const void*)k_cs_csr<double>, lds));
    hipLaunchKernelGGL(k_cs_csr<double>, dim3(s), dim3(256), lds, st, A.d, seed, offsets, sorted, A.ptr, A.idx,
                       (const double*)A.val, out, labels, c, se);
  } else {
    SRP_TRY(allow_dynamic_lds((const void*)k_cs_csr<float>, lds));
    hipLaunchKernelGGL(k_cs_csr<float>, dim3(s), dim3(256), lds, st, A.d, seed, offsets, sorted, A.ptr, A.idx,
                       (const float*)A.val, out, labels, c, se);
  }
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

// ------------------------------------------------- FDA class statistics
__global__ void __launch_bounds__(256) k_label_counts(int64_t n, int c, const int32_t* __restrict__ labels,
                                                      int* counts, int* bad) {
  __shared__ int h[kLdaMaxClasses];
  for (int q = threadIdx.x; q < c; q += blockDim.x) h[q] = 0;
  __syncthreads();
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) {
    const int y = labels[i];
    if (y < 0 || y >= c) atomicOr(bad, 1);
    else atomicAdd(&h[y], 1);
  }
  __syncthreads();
  for (int q = threadIdx.x; q < c; q += blockDim.x)
    if (h[q]) atomicAdd(&counts[q], h[q]);
}

int label_counts_run(int64_t n, int c, const int32_t* labels, int* counts, int* bad, hipStream_t st) {
  SRP_TRY(fill_i32(counts, c, 0, st));
  hipLaunchKernelGGL(k_label_counts, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, c, labels, counts, bad);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

// Class sums of column j: one wave per column, lane l adds the column's
// entries l, l + 64, ... into its own LDS slot per class, then the slots
// are summed in lane order.  Labels must already be known to be in range.
template <class T>
__global__ void __launch_bounds__(64) k_csc_class_sums(int d, int c, const int* __restrict__ colptr,
                                                       const int32_t* __restrict__ rows, const T* __restrict__ val,
                                                       const int32_t* __restrict__ labels, double* __restrict__ sums) {
  __shared__ double acc[kLdaMaxClasses * 64];
  const int j = blockIdx.x, lane = threadIdx.x;
  for (int q = 0; q < c; ++q) acc[q * 64 + lane] = 0.0;
  const int e0 = colptr[j], e1 = colptr[j + 1];
  for (int e = e0 + lane; e < e1; e += 64) acc[labels[rows[e]] * 64 + lane] += to_f64(val[e]);
  __syncthreads();
  for (int q = lane; q < c; q += 64) {
    double s = 0.0;
    for (int l = 0; l < 64; ++l) s += acc[q * 64 + l];
    sums[(int64_t)q * d + j] = s;
  }
}

// Per column j: m_q = sums_q / n_q, m = sum_q sums_q / n,
// Yhat_q = sqrt(n_q) (m_q - m).
__global__ void k_fda_class_factors(int64_t n, int d, int c, const int* __restrict__ counts,
                                    const double* __restrict__ sums, double* __restrict__ means,
                                    double* __restrict__ Yhat) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= d) return;
  double tot = 0.0;
  for (int q = 0; q < c; ++q) tot += sums[(int64_t)q * d + j];
  const double m = tot / (double)n;
  for (int q = 0; q < c; ++q) {
    const double mq = sums[(int64_t)q * d + j] / (double)counts[q];
    means[(int64_t)q * d + j] = mq;
    Yhat[(int64_t)q * d + j] = sqrt((double)counts[q]) * (mq - m);
  }
}

int fda_csr_stats_run(const CscView& A, int64_t n, int c, const int32_t* labels, const int* counts, double* sums,
                      double* means, double* Yhat, hipStream_t st) {
  if (A.dtype == SRP_F64)
    hipLaunchKernelGGL(k_csc_class_sums<double>, dim3(A.d), dim3(64), 0, st, A.d, c, A.ptr, A.idx,
                       (const double*)A.val, labels, sums);
  else
    hipLaunchKernelGGL(k_csc_class_sums<float>, dim3(A.d), dim3(64), 0, st, A.d, c, A.ptr, A.idx,
                       (const float*)A.val, labels, sums);
  SRP_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_fda_class_factors, dim3((A.d + 255) / 256), dim3(256), 0, st, n, A.d, c, counts, sums, means,
                     Yhat);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

}  // namespace srp

namespace srp {

int csr_check(const CsrView& A, const char* name, int* bad, hipStream_t st) {
  SRP_REQUIRE(A.n >= 1 && A.n < (int64_t(1) << 31), "%s: rows out of range", name);
  SRP_REQUIRE(A.d >= 1 && A.d <= kCsrMaxCols, "%s: need 1 <= columns <= %d", name, kCsrMaxCols);
  SRP_REQUIRE(A.nnz >= 0 && A.nnz < (int64_t(1) << 31), "%s: nnz out of range", name);
  SRP_REQUIRE(A.dtype == SRP_F32 || A.dtype == SRP_F64, "%s: values must be SRP_F32 or SRP_F64", name);
  SRP_REQUIRE(A.ptr && (A.nnz == 0 || (A.idx && A.val)), "%s: null pointer", name);
  SRP_TRY(fill_i32(bad, 1, 0, st));
  SRP_TRY(csr_validate(A, bad, st));
  int h = 0;
  SRP_HIP(hipMemcpyAsync(&h, bad, sizeof(int), hipMemcpyDeviceToHost, st));
  SRP_HIP(hipStreamSynchronize(st));
  SRP_REQUIRE(!h, "%s is not a well-formed CSR matrix (row pointers, or columns in range and strictly increasing)",
              name);
  return SRP_OK;
}

}  // namespace srp
