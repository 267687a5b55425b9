// Small kernels of the Riemannian trust-region solver (Section 2.2 lists
// the trust-region method among the Riemannian algorithms the components
// of Table 1 serve): linear combinations of d x k blocks, the traces that
// give the metric's inner products, the Sylvester solve of the projection
// from a stored eigendecomposition, and the trial step's k x k algebra
// (Cholesky of the retraction Gram, cost at the trial point).  The
// product manifold's two blocks (CCA) run as blockIdx.y.
#include "common.hpp"
#include "solver.hpp"
#include "rtr.hpp"

namespace srp {

// out_b = a A_b + c C_b K_b  (K_b k x k row-major; null = identity; A and
// C may be column blocks of wider row-major arrays, rows lda / ldc apart).
__global__ void __launch_bounds__(256) k_rtr_lin(RtrLinArgs args) {
  const RtrLinSide& sd = args.side[blockIdx.y];
  const int k = args.k;
  const int64_t cnt = (int64_t)sd.d * k;
  const int64_t e = blockIdx.x * 256ll + threadIdx.x;
  if (e >= cnt || !sd.out) return;
  const int64_t i = e / k;
  const int j = (int)(e - i * k);
  const int64_t lda = sd.lda ? sd.lda : k, ldc = sd.ldc ? sd.ldc : k;
  double v = sd.A ? sd.a * sd.A[i * lda + j] : 0.0;
  if (sd.C) {
    if (sd.K) {
      double s = 0.0;
      for (int l = 0; l < k; ++l) s += sd.C[i * ldc + l] * sd.K[l * k + j];
      v += sd.c * s;
    } else {
      v += sd.c * sd.C[i * ldc + j];
    }
  }
  sd.out[e] = v;
}

int rtr_lin(const RtrLinArgs& a, int nb, hipStream_t st) {
  int64_t cnt = 0;
  for (int b = 0; b < nb; ++b) cnt = std::max<int64_t>(cnt, (int64_t)a.side[b].d * a.k);
  hipLaunchKernelGGL(k_rtr_lin, dim3((unsigned)((cnt + 255) / 256), nb), dim3(256), 0, st, a);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

// out[p] = sum over blocks of tr(X_p^T Y_p): one workgroup, fixed order.
__global__ void __launch_bounds__(256) k_rtr_dots(RtrDotArgs args) {
  __shared__ double red[4][kRtrMaxDots];
  const int tid = threadIdx.x;
  double acc[kRtrMaxDots];
#pragma unroll
  for (int p = 0; p < kRtrMaxDots; ++p) acc[p] = 0.0;
  for (int b = 0; b < args.nb; ++b) {
    const int64_t cnt = (int64_t)args.d[b] * args.k;
    for (int p = 0; p < args.np; ++p) {
      const double* X = args.X[p][b];
      const double* Y = args.Y[p][b];
      double s = 0.0;
      for (int64_t e = tid; e < cnt; e += 256) s += X[e] * Y[e];
      acc[p] += s;
    }
  }
  for (int p = 0; p < args.np; ++p) {
    double v = acc[p];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((tid & 63) == 0) red[tid >> 6][p] = v;
  }
  __syncthreads();
  if (tid < args.np) args.out[tid] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
}

int rtr_dots(const RtrDotArgs& a, hipStream_t st) {
  if (a.np < 1 || a.np > kRtrMaxDots) {
    set_error("rtr: %d inner products per launch (1 to %d)", a.np, kRtrMaxDots);
    return SRP_EINVAL;
  }
  hipLaunchKernelGGL(k_rtr_dots, dim3(1), dim3(256), 0, st, a);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

// Sylvester solve of the projection, P S + S P = C + C^T, from the
// eigendecomposition P = Q diag(lam) Q^T: S = Q [(Q^T (C + C^T) Q)_ij /
// (lam_i + lam_j)] Q^T.  One wave per block.
__global__ void __launch_bounds__(64) k_rtr_sylv(RtrSylvArgs args) {
  __shared__ double T1[kRtrK * kRtrK], T2[kRtrK * kRtrK];
  const int b = blockIdx.x, k = args.k, lane = threadIdx.x, kk = k * k;
  const double* Q = args.Q[b];
  const double* lam = args.lam[b];
  const double* C = args.C[b];
  // T1 = (C + C^T) Q
  for (int e = lane; e < kk; e += 64) {
    const int i = e / k, j = e - i * k;
    double s = 0.0;
    for (int l = 0; l < k; ++l) s += (C[i * k + l] + C[l * k + i]) * Q[l * k + j];
    T1[e] = s;
  }
  __syncthreads();
  // T2 = Q^T T1, scaled by 1 / (lam_i + lam_j)
  for (int e = lane; e < kk; e += 64) {
    const int i = e / k, j = e - i * k;
    double s = 0.0;
    for (int l = 0; l < k; ++l) s += Q[l * k + i] * T1[l * k + j];
    T2[e] = s / (lam[i] + lam[j]);
  }
  __syncthreads();
  // T1 = T2 Q^T, S = Q T1
  for (int e = lane; e < kk; e += 64) {
    const int i = e / k, j = e - i * k;
    double s = 0.0;
    for (int l = 0; l < k; ++l) s += T2[i * k + l] * Q[j * k + l];
    T1[e] = s;
  }
  __syncthreads();
  double* S = args.S[b];
  for (int e = lane; e < kk; e += 64) {
    const int i = e / k, j = e - i * k;
    double s = 0.0;
    for (int l = 0; l < k; ++l) s += Q[i * k + l] * T1[l * k + j];
    S[e] = s;
  }
}

int rtr_sylv(const RtrSylvArgs& a, int nb, hipStream_t st) {
  hipLaunchKernelGGL(k_rtr_sylv, dim3(nb), dim3(64), 0, st, a);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

// Lower Cholesky in place (k x k) by one wave; false on a non-positive pivot.
__device__ static bool rtr_chol(double* A, int k, int lane) {
  for (int j = 0; j < k; ++j) {
    __syncthreads();
    const double piv = A[j * k + j];
    if (!(piv > 0.0) || !isfinite(piv)) return false;
    const double dj = sqrt(piv);
    __syncthreads();
    if (lane == 0) A[j * k + j] = dj;
    for (int i = j + 1 + lane; i < k; i += 64) A[i * k + j] /= dj;
    __syncthreads();
    for (int e = lane; e < k * k; e += 64) {
      const int r = e / k, c = e - r * k;
      if (r > j && c > j && c <= r) A[r * k + c] -= A[r * k + j] * A[c * k + j];
    }
  }
  __syncthreads();
  return true;
}

// Trial step of the trust region.  Per block, the retraction Gram
// G = (Z + eta)^T B (Z + eta) = I + E + E^T + F (E = Z^T B eta, F = eta^T
// B eta) and its Cholesky L; Lit = L^-T.  The cost at R_Z(eta) from the
// cross Gram X0 = (Z_0 + eta_0)^T K (Z_1 + eta_1) (CCA: K = Sxy; FDA:
// S_B with Z_1 = Z_0), given as its four parts Z^T K Z, Z^T K eta,
// eta^T K Z, eta^T K eta: f+ = -c tr(L_0^-1 X0 L_1^-T N), c = 1 (CCA) or
// 1/2 (FDA).  out[0] = f+, out[1] = 1 on a Cholesky breakdown.  One wave.
__global__ void __launch_bounds__(64) k_rtr_trial(RtrTrialArgs args) {
  __shared__ double G[2][kRtrK * kRtrK], Li[2][kRtrK * kRtrK], X0[kRtrK * kRtrK], T[kRtrK * kRtrK];
  const int k = args.k, nb = args.nb, lane = threadIdx.x, kk = k * k;
  for (int b = 0; b < nb; ++b) {
    for (int e = lane; e < kk; e += 64) {
      const int i = e / k, j = e - i * k;
      G[b][e] = args.E[b][e] + args.E[b][j * k + i] + 0.5 * (args.F[b][e] + args.F[b][j * k + i]);
    }
  }
  for (int e = lane; e < kk; e += 64) X0[e] = args.X0[0][e] + args.X0[1][e] + args.X0[2][e] + args.X0[3][e];
  __syncthreads();
  bool ok = true;
  for (int b = 0; b < nb; ++b) ok = ok && rtr_chol(G[b], k, lane);
  if (!ok) {
    if (lane == 0) { args.out[0] = 0.0; args.out[1] = 1.0; }
    return;
  }
  // Li = L^-1 (lower), column per lane
  for (int b = 0; b < nb; ++b) {
    for (int c = lane; c < k; c += 64) {
      for (int r = 0; r < c; ++r) Li[b][r * k + c] = 0.0;
      Li[b][c * k + c] = 1.0 / G[b][c * k + c];
      for (int r = c + 1; r < k; ++r) {
        double s = 0.0;
        for (int l = c; l < r; ++l) s += G[b][r * k + l] * Li[b][l * k + c];
        Li[b][r * k + c] = -s / G[b][r * k + r];
      }
    }
  }
  __syncthreads();
  const int o = nb == 2 ? 1 : 0;
  // T = Li_0 X0 ; cost = -c sum_i mu_i (T Li_o^T)_ii
  for (int e = lane; e < kk; e += 64) {
    const int i = e / k, j = e - i * k;
    double s = 0.0;
    for (int l = 0; l <= i; ++l) s += Li[0][i * k + l] * X0[l * k + j];
    T[e] = s;
  }
  __syncthreads();
  if (lane == 0) {
    double f = 0.0;
    for (int i = 0; i < k; ++i) {
      double s = 0.0;
      for (int l = 0; l <= i; ++l) s += T[i * k + l] * Li[o][i * k + l];
      f += args.mu[i] * s;
    }
    args.out[0] = -args.cost_scale * f;
    args.out[1] = 0.0;
  }
  for (int b = 0; b < nb; ++b)
    for (int e = lane; e < kk; e += 64) {
      const int i = e / k, j = e - i * k;
      args.Lit[b][e] = Li[b][j * k + i];   // L^-T
    }
}

int rtr_trial(const RtrTrialArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_rtr_trial, dim3(1), dim3(64), 0, st, a);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

}  // namespace srp
