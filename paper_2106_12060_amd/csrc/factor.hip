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
// 2x2 MFMA tiles; the k dimension is staged through LDS 16 at a time.
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
  __shared__ double As[16][65];
  __shared__ double Bs[16][65];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wi = (w >> 1) * 32, wj = (w & 1) * 32;
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = kbeg; k0 < kend; k0 += 16) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = t + q * 256;
      int kq, iq;
      if (TA) { kq = e >> 6; iq = e & 63; } else { iq = e >> 4; kq = e & 15; }
      const int gi = i0 + iq, gk = k0 + kq;
      double v = 0.0;
      if (gi < m && gk < kend) v = TA ? (double)A[(int64_t)gk * lda + gi] : (double)A[(int64_t)gi * lda + gk];
      As[kq][iq] = v;
      int kb, jb;
      if (!TB) { kb = e >> 6; jb = e & 63; } else { jb = e >> 4; kb = e & 15; }
      const int gj = j0 + jb, gk2 = k0 + kb;
      double u = 0.0;
      if (gj < n && gk2 < kend) u = TB ? (double)B[(int64_t)gj * ldb + gk2] : (double)B[(int64_t)gk2 * ldb + gj];
      Bs[kb][jb] = u;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 4; ++s) {
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

template <class AT, class BT>
static int gemm_dispatch_t(const GemmArgs& g, hipStream_t st) {
  dim3 grid((g.n + 63) / 64, (g.m + 63) / 64, g.ksplit);
  int kchunk = g.kk;
  if (g.ksplit > 1) kchunk = (((g.kk + g.ksplit - 1) / g.ksplit) + 15) / 16 * 16;
  const AT* A = (const AT*)g.A;
  const BT* B = (const BT*)g.B;
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

int sum_parts_f64(const double* parts, int nparts, int64_t stride, int64_t count, double* out, int d,
                  double diag_add, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, parts, nparts, stride,
                     count, out, d, diag_add);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

// --------------------------------------------------------- skinny GEMM
// C (m x nc) = op(A) (m x kk) B (kk x nc), nc <= 64: the per-iteration
// products with M^-1 and the FDA between-class factor.  The contraction is
// split over blockIdx.y into slices of kSkSlice; a workgroup owns 16 rows of
// op(A) in its slice and streams them once through LDS together with the
// matching rows of B, and writes a partial; a second kernel adds the
// partials in slice order (deterministic).  Thread (r, jg) keeps the
// columns jg, jg + 16, ... of row r.
constexpr int kSkRows = 16;
constexpr int kSkChunk = 64;
constexpr int kSkSlice = 128;

__global__ void __launch_bounds__(256) k_gemm_skinny(int m, int kk, int nc, const double* __restrict__ A,
                                                     int64_t lda, int ta, const double* __restrict__ B,
                                                     int64_t ldb, double* __restrict__ part) {
  __shared__ double As[kSkRows][kSkChunk + 1];
  __shared__ double Bs[kSkChunk][64];
  const int r0 = blockIdx.x * kSkRows;
  const int lbeg = blockIdx.y * kSkSlice, lend = min(kk, lbeg + kSkSlice);
  const int tid = threadIdx.x;
  const int r = tid >> 4, jg = tid & 15;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int l0 = lbeg; l0 < lend; l0 += kSkChunk) {
    if (ta) {
      for (int e = tid; e < kSkRows * kSkChunk; e += 256) {
        const int ll = e / kSkRows, rr = e % kSkRows;
        const int gr = r0 + rr, gl = l0 + ll;
        As[rr][ll] = (gr < m && gl < lend) ? A[(int64_t)gl * lda + gr] : 0.0;
      }
    } else {
      for (int e = tid; e < kSkRows * kSkChunk; e += 256) {
        const int rr = e / kSkChunk, ll = e % kSkChunk;
        const int gr = r0 + rr, gl = l0 + ll;
        As[rr][ll] = (gr < m && gl < lend) ? A[(int64_t)gr * lda + gl] : 0.0;
      }
    }
    for (int e = tid; e < kSkChunk * nc; e += 256) {
      const int ll = e / nc, j = e % nc;
      const int gl = l0 + ll;
      Bs[ll][j] = (gl < lend) ? B[(int64_t)gl * ldb + j] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int ll = 0; ll < kSkChunk; ++ll) {
      const double a = As[r][ll];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = jg + 16 * q;
        if (j < nc) acc[q] += a * Bs[ll][j];
      }
    }
    __syncthreads();
  }
  const int gr = r0 + r;
  if (gr < m) {
    double* out = part + ((int64_t)blockIdx.y * m + gr) * nc;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = jg + 16 * q;
      if (j < nc) out[j] = acc[q];
    }
  }
}

__global__ void __launch_bounds__(256) k_skinny_sum(int m, int nc, int nsl, const double* __restrict__ part,
                                                    double* __restrict__ C, int64_t ldc) {
  const int64_t e = blockIdx.x * 256ll + threadIdx.x;
  const int64_t cnt = (int64_t)m * nc;
  if (e >= cnt) return;
  double s0 = 0.0, s1 = 0.0;
  int z = 0;
  for (; z + 2 <= nsl; z += 2) {
    s0 += part[(int64_t)z * cnt + e];
    s1 += part[(int64_t)(z + 1) * cnt + e];
  }
  if (z < nsl) s0 += part[(int64_t)z * cnt + e];
  const int64_t row = e / nc, col = e % nc;
  C[row * ldc + col] = s0 + s1;
}

size_t skinny_ws_bytes(int m, int kk, int nc) {
  const size_t nsl = (size_t)(kk + kSkSlice - 1) / kSkSlice;
  return bytes_of<double>(nsl * (size_t)m * nc);
}

int gemm_skinny_f64(int m, int kk, int nc, const double* A, int64_t lda, bool ta, const double* B, int64_t ldb,
                    double* C, int64_t ldc, double* ws, size_t ws_bytes, hipStream_t st) {
  if (nc > 64 || nc < 1 || m < 1 || kk < 1) {
    set_error("gemm_skinny: bad shape m=%d kk=%d nc=%d", m, kk, nc);
    return SRP_EINVAL;
  }
  const int nsl = (kk + kSkSlice - 1) / kSkSlice;
  if (!ws || skinny_ws_bytes(m, kk, nc) > ws_bytes) {
    set_error("gemm_skinny: workspace too small");
    return SRP_ENOMEM;
  }
  hipLaunchKernelGGL(k_gemm_skinny, dim3((m + kSkRows - 1) / kSkRows, nsl), dim3(256), 0, st, m, kk, nc, A, lda,
                     ta ? 1 : 0, B, ldb, ws);
  SRP_LAUNCH_CHECK();
  const int64_t cnt = (int64_t)m * nc;
  hipLaunchKernelGGL(k_skinny_sum, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, m, nc, nsl, ws, C, ldc);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

// --------------------------------------------------------- Cholesky
// Factor the nb x nb diagonal block at (k0, k0) of the symmetric matrix G
// (upper triangle read): R_kk upper with R_kk^T R_kk = G_kk, written into R;
// its inverse into Dinv (64 x 64, upper, identity-padded).  Sets *flag on a
// non-positive pivot.
__global__ void __launch_bounds__(256) k_potrf_block(const double* __restrict__ G, int64_t ld, int k0, int nb,
                                                     double* __restrict__ R, double* __restrict__ Dinv,
                                                     int* flag) {
  __shared__ double a[64][65];
  __shared__ double x[64][65];
  const int t = threadIdx.x;
  for (int e = t; e < 4096; e += 256) {
    const int r = e >> 6, c = e & 63;
    double v;
    if (r < nb && c < nb) {
      const int lo = min(r, c), hi = max(r, c);
      v = G[(int64_t)(k0 + lo) * ld + k0 + hi];
    } else {
      v = (r == c) ? 1.0 : 0.0;
    }
    a[r][c] = v;
  }
  __syncthreads();
  for (int j = 0; j < 64; ++j) {
    if (t == 0) {
      double p = a[j][j];
      if (!(p > 0.0)) {
        atomicOr(flag, 1);
        p = 1.0;
      }
      a[j][j] = sqrt(p);
    }
    __syncthreads();
    const double djj = a[j][j];
    for (int c = j + 1 + t; c < 64; c += 256) a[j][c] /= djj;
    __syncthreads();
    const int w = 63 - j;  // trailing size
    for (int e = t; e < w * w; e += 256) {
      const int r = j + 1 + e / w, c = j + 1 + e % w;
      if (r <= c) a[r][c] -= a[j][r] * a[j][c];
    }
    __syncthreads();
  }
  // inverse of the upper factor, one column per thread
  if (t < 64) {
    const int c = t;
    for (int r = 0; r < 64; ++r) x[r][c] = 0.0;
    x[c][c] = 1.0 / a[c][c];
    for (int r = c - 1; r >= 0; --r) {
      double s = 0.0;
      for (int l = r + 1; l <= c; ++l) s += a[r][l] * x[l][c];
      x[r][c] = -s / a[r][r];
    }
  }
  __syncthreads();
  for (int e = t; e < 4096; e += 256) {
    const int r = e >> 6, c = e & 63;
    Dinv[e] = x[r][c];
    if (r < nb && c < nb) R[(int64_t)(k0 + r) * ld + k0 + c] = (r <= c) ? a[r][c] : 0.0;
  }
}

// Copy 64x64 block inverses onto the diagonal of X (d x d).
__global__ void k_place_diag_blocks(const double* __restrict__ Dinv, int d, double* __restrict__ X) {
  const int kb = blockIdx.x;
  const int k0 = kb * 64;
  const int nb = min(64, d - k0);
  for (int e = threadIdx.x; e < 4096; e += blockDim.x) {
    const int r = e >> 6, c = e & 63;
    if (r < nb && c < nb) X[(int64_t)(k0 + r) * d + k0 + c] = Dinv[(int64_t)kb * 4096 + e];
  }
}

size_t factor_ws_bytes(int s, int d) {
  const int tiles = (d + 63) / 64;
  const int nupper = tiles * (tiles + 1) / 2;
  int ksplit = (512 + nupper - 1) / nupper;
  const int kmax = (s + 63) / 64;
  if (ksplit > kmax) ksplit = kmax;
  if (ksplit < 1) ksplit = 1;
  const size_t dd = (size_t)d * d;
  return bytes_of<double>(dd) * (ksplit > 1 ? ksplit + 1 : 1) + bytes_of<double>((size_t)tiles * 4096) +
         bytes_of<double>((size_t)64 * d) + bytes_of<double>(dd);
}

int sketch_factor_run(const void* SA, int dtype, int s, int d, double lambda, double* R, double* Rinv,
                      double* Minv, int* flag_dev, Arena& ws, hipStream_t st) {
  const int tiles = (d + 63) / 64;
  const int nupper = tiles * (tiles + 1) / 2;
  int ksplit = (512 + nupper - 1) / nupper;
  const int kmax = (s + 63) / 64;
  if (ksplit > kmax) ksplit = kmax;
  if (ksplit < 1) ksplit = 1;
  const int64_t dd = (int64_t)d * d;
  double* G = ws.take<double>(dd);
  double* parts = ksplit > 1 ? ws.take<double>(dd * ksplit) : nullptr;
  double* Dinv = ws.take<double>((size_t)tiles * 4096);
  double* Tmp = ws.take<double>((size_t)64 * d);
  double* X = Rinv ? Rinv : ws.take<double>(dd);
  if (!G || !Dinv || !Tmp || !X || (ksplit > 1 && !parts)) {
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
  if (ksplit > 1) {
    g.C = parts; g.ldc = d; g.ksplit = ksplit; g.c_split_stride = dd;
    SRP_TRY(fill_f64(parts, dd * ksplit, 0.0, st));
    SRP_TRY(gemm_f64(g, st));
    SRP_TRY(sum_parts_f64(parts, ksplit, dd, dd, G, d, lambda, st));
  } else {
    g.C = G; g.ldc = d;
    SRP_TRY(fill_f64(G, dd, 0.0, st));
    SRP_TRY(gemm_f64(g, st));
    SRP_TRY(sum_parts_f64(G, 1, dd, dd, G, d, lambda, st));
  }
  // Right-looking blocked Cholesky, 64-wide panels.
  SRP_TRY(fill_f64(R, dd, 0.0, st));
  for (int kb = 0; kb < tiles; ++kb) {
    const int k0 = kb * 64, nb = min(64, d - k0);
    hipLaunchKernelGGL(k_potrf_block, dim3(1), dim3(256), 0, st, G, (int64_t)d, k0, nb, R,
                       Dinv + (size_t)kb * 4096, flag_dev);
    SRP_LAUNCH_CHECK();
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
  // X = R^-1, block rows bottom-up: X_ij = -R_ii^-1 sum_{l>i} R_il X_lj.
  SRP_TRY(fill_f64(X, dd, 0.0, st));
  hipLaunchKernelGGL(k_place_diag_blocks, dim3(tiles), dim3(256), 0, st, Dinv, d, X);
  SRP_LAUNCH_CHECK();
  for (int ib = tiles - 2; ib >= 0; --ib) {
    const int i0 = ib * 64, c1 = i0 + 64, rest = d - c1;
    GemmArgs a{};
    a.m = 64; a.n = rest; a.kk = rest; a.alpha = 1.0; a.beta = 0.0;
    a.A = R + (int64_t)i0 * d + c1; a.lda = d; a.ta = false;
    a.B = X + (int64_t)c1 * d + c1; a.ldb = d; a.tb = false;
    a.C = Tmp; a.ldc = rest;
    SRP_TRY(gemm_f64(a, st));
    GemmArgs b{};
    b.m = 64; b.n = rest; b.kk = 64; b.alpha = -1.0; b.beta = 0.0;
    b.A = Dinv + (size_t)ib * 4096; b.lda = 64; b.ta = false;
    b.B = Tmp; b.ldb = rest; b.tb = false;
    b.C = X + (int64_t)i0 * d + c1; b.ldc = d;
    SRP_TRY(gemm_f64(b, st));
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
