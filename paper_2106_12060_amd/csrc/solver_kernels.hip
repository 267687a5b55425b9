// Step kernels of the preconditioned Riemannian CG (Table 1 components on
// St_B(k, d) with the fixed sketched metric M; the CCA problem is the
// product of two such manifolds, Section 4.2).
//
// The iterate never leaves the device and every data product comes from
// one fused pass per iteration (pass.hip).  With Ks = A^T A U,
// Kc = cost products (CCA: A_b^T A_o U_o; FDA: S_B W) maintained across
// iterations and J = A^T A xi (and cross terms) from the pass along the
// direction xi, everything below is algebra on d x k and k x k blocks:
//
//  * Retraction curve R(U + t xi) = (U + t xi) L(t)^-T with
//    L L^T = (U + t xi)^T B (U + t xi) = G0 + t G1 + t^2 G2 (QR retraction
//    of Table 1 written as a Cholesky of the small Gram), and the cost on
//    it (Eq. costriemannianccaBrockett / Eq. lda_riemannian) follows from
//    k x k products only, so the line search costs no data pass.
//  * At the accepted point U+ = (U + t xi) L^-T the products update as
//    Ks+ = (Ks + t J) L^-T, Kc+ = (Kc + t Jc) L_o^-T.
//  * Gradient (Table 1 / Eq. gradCCA): with E = -Kc N (Euclidean gradient)
//    and BU = Ks + lam U, grad = M^-1 E - M^-1 BU S where S solves the
//    Sylvester equation P S + S P = BU^T M^-1 E + (.)^T, P = BU^T M^-1 BU.
//    M grad = E - BU S, so metric inner products need no extra M product.
//  * Transport by projection (Table 1) of the previous direction and
//    gradient, Polak-Ribiere+ coefficient, restart on non-descent.
// The k x k work runs in single-workgroup "controller" kernels in FP64;
// the Sylvester equations use a parallel cyclic Jacobi eigensolver.
#include "solver.hpp"
#include "kernels.hpp"

#include <cmath>

namespace srp {

// e / d for 0 <= e < 2^19 and 1 <= d <= 4096 without an integer division:
// (e + 0.5) / d lies at least 0.5 / d from an integer, far more than the
// error of the single-precision reciprocal and product.
__device__ __forceinline__ int sdiv(int e, int d) {
  return (int)(((float)e + 0.5f) * __builtin_amdgcn_rcpf((float)d));
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__host__ __device__ __forceinline__ double* kkslot(const ProbView& p, int side, int slot) {
  return p.kk + ((size_t)side * KK_NSLOTS + slot) * KK_STRIDE;
}

// ------------------------------------------------------------ partials
// out[z][a*k+i][b*k+j] = sum over rows r in slice z of L_a[r][i] * R_b[r][j]
// (PartialArgs in solver.hpp).

constexpr int kPartRows = 16;
constexpr int kMaxSlices = 64;   // row-slice partials per side (summed by k_part_reduce)

// One row slice of a side: the (nl k) x (nr k) products L^T R over the
// slice's rows on FP64 matrix cores (16x16 output tiles, 4 rows per step).
// Rows are staged 16 at a time by buffer loads, one operand block (a d x k
// array) per step: a masked element takes an offset past the resource and
// reads zero, so the loads issue unconditionally and a stage's loads are in
// flight together; the next stage's loads overlap this stage's products.
__device__ __forceinline__ void partials_body(const PartialArgs& a, int z, int y) {
  if (a.ctrl && a.ctrl->done) return;
  const PartialSide& ps = a.side[y];
  const int k = a.k;
  const int NL = ps.nl * k, NR = ps.nr * k;
  const int MT = (NL + 15) >> 4, NT = (NR + 15) >> 4;
  __shared__ double ls[kPartRows][2 * KMAX];
  __shared__ double rs[kPartRows][6 * KMAX];
  constexpr int EL = (kPartRows * KMAX + 255) / 256;   // elements of one operand block per thread
  constexpr int MAXT = ((2 * KMAX / 16) * (6 * KMAX / 16) + 3) / 4;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int ntiles = MT * NT;
  // the staged columns past NL / NR are read by the edge tiles: zero them
  for (int e = tid; e < kPartRows * 2 * KMAX; e += 256) (&ls[0][0])[e] = 0.0;
  for (int e = tid; e < kPartRows * 6 * KMAX; e += 256) (&rs[0][0])[e] = 0.0;
  f64x4 acc[MAXT];
#pragma unroll
  for (int q = 0; q < MAXT; ++q) acc[q] = f64x4{0.0, 0.0, 0.0, 0.0};
  // element q of a block for this thread: row rr[q], column jj[q] (-1: none)
  int rr[EL], jj[EL];
#pragma unroll
  for (int q = 0; q < EL; ++q) {
    const int e = tid + 256 * q;
    const int r = sdiv(e, k);
    rr[q] = r;
    jj[q] = (e < kPartRows * k) ? e - r * k : -1;
  }
  double vl[2][EL], vr[6][EL];
  auto fetch = [&](int r0) __attribute__((always_inline)) {
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      if (b < ps.nl) {
        const __amdgpu_buffer_rsrc_t rs_b = make_rsrc(ps.lp[b], (int64_t)ps.d * ps.lld[b] * 8);
#pragma unroll
        for (int q = 0; q < EL; ++q) {
          const int r = r0 + rr[q];
          vl[b][q] = buf_load<double>(rs_b, (jj[q] >= 0 && r < ps.d) ? (r * ps.lld[b] + jj[q]) * 8 : kOob, 0);
        }
      }
    }
#pragma unroll
    for (int b = 0; b < 6; ++b) {
      if (b < ps.nr) {
        const __amdgpu_buffer_rsrc_t rs_b = make_rsrc(ps.rp[b], (int64_t)ps.d * ps.rld[b] * 8);
#pragma unroll
        for (int q = 0; q < EL; ++q) {
          const int r = r0 + rr[q];
          vr[b][q] = buf_load<double>(rs_b, (jj[q] >= 0 && r < ps.d) ? (r * ps.rld[b] + jj[q]) * 8 : kOob, 0);
        }
      }
    }
  };
  const int step = a.slices * kPartRows;
  int r0 = z * kPartRows;
  if (r0 < ps.d) fetch(r0);
  __syncthreads();   // zeroed staging visible before the first stores
  for (; r0 < ps.d; r0 += step) {
#pragma unroll
    for (int q = 0; q < EL; ++q) {
      if (jj[q] >= 0) {
#pragma unroll
        for (int b = 0; b < 2; ++b)
          if (b < ps.nl) ls[rr[q]][b * k + jj[q]] = vl[b][q];
#pragma unroll
        for (int b = 0; b < 6; ++b)
          if (b < ps.nr) rs[rr[q]][b * k + jj[q]] = vr[b][q];
      }
    }
    __syncthreads();
    if (r0 + step < ps.d) fetch(r0 + step);
#pragma unroll
    for (int q = 0; q < MAXT; ++q) {
      const int tt = w + 4 * q;
      if (tt < ntiles) {
        const int mt = sdiv(tt, NT), nt = tt - mt * NT;
#pragma unroll
        for (int s4 = 0; s4 < kPartRows / 4; ++s4) {
          const int row = 4 * s4 + (lane >> 4);
          acc[q] = mfma16x16x4(ls[row][16 * mt + (lane & 15)], rs[row][16 * nt + (lane & 15)], acc[q]);
        }
      }
    }
    __syncthreads();
  }
  double* out = a.out + y * a.side_stride + (int64_t)z * NL * NR;
#pragma unroll
  for (int q = 0; q < MAXT; ++q) {
    const int tt = w + 4 * q;
    if (tt < ntiles) {
      const int mt = sdiv(tt, NT), nt = tt - mt * NT;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * mt + acc_row<double>(lane, r), j = 16 * nt + (lane & 15);
        if (i < NL && j < NR) out[(int64_t)i * NR + j] = acc[q][r];
      }
    }
  }
}

__global__ void __launch_bounds__(256) k_partials(PartialArgs a) { partials_body(a, blockIdx.x, blockIdx.y); }

// Grouped: blockIdx.z picks the solve (sel.idx), each with its own slices
// and sides.
__global__ void __launch_bounds__(256) k_partials_g(const PartialArgs* __restrict__ ga, GroupSel sel) {
  const PartialArgs& a = ga[sel.idx[blockIdx.z]];
  if ((int)blockIdx.x >= a.slices || (int)blockIdx.y >= a.nb) return;
  partials_body(a, blockIdx.x, blockIdx.y);
}

int partial_slices(int dmax) {
  int s = (dmax + kPartRows - 1) / kPartRows;
  return s < kMaxSlices ? (s < 1 ? 1 : s) : kMaxSlices;
}

size_t partial_bytes(int k, int dmax) {
  return bytes_of<double>((size_t)2 * partial_slices(dmax) * (4 * k) * (6 * k));
}

// Sum of the row-slice partials in slice order, in place into slice 0 (one
// thread per entry): the single-workgroup controllers then read one slice
// instead of pulling every slice through one compute unit.
__device__ __forceinline__ void part_reduce_body(double* __restrict__ part, int slices, int64_t side_stride,
                                                 int64_t nlnr, const SolverCtrl* __restrict__ ctrl, int64_t e,
                                                 int y) {
  if (ctrl && ctrl->done) return;
  if (e >= nlnr) return;
  double* base = part + y * side_stride + e;
  // the loads of all slices (at most kMaxSlices) in flight together, added
  // in slice order; one batch of 16 when there are no more
  double s = 0.0;
  if (slices > 16) {
    double t[kMaxSlices];
#pragma unroll
    for (int u = 0; u < kMaxSlices; ++u) t[u] = base[(u < slices ? u : 0) * nlnr];
#pragma unroll
    for (int u = 0; u < kMaxSlices; ++u) s += (u < slices) ? t[u] : 0.0;
  } else {
    double t[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) t[u] = base[(u < slices ? u : 0) * nlnr];
#pragma unroll
    for (int u = 0; u < 16; ++u) s += (u < slices) ? t[u] : 0.0;
  }
  base[0] = s;
}

__global__ void __launch_bounds__(256) k_part_reduce(double* __restrict__ part, int slices, int64_t side_stride,
                                                     int64_t nlnr, const SolverCtrl* __restrict__ ctrl) {
  part_reduce_body(part, slices, side_stride, nlnr, ctrl, blockIdx.x * 256ll + threadIdx.x, blockIdx.y);
}

__global__ void __launch_bounds__(256) k_part_reduce_g(const PartialArgs* __restrict__ ga, GroupSel sel) {
  const PartialArgs& a = ga[sel.idx[blockIdx.z]];
  if (a.slices <= 1 || (int)blockIdx.y >= a.nb) return;
  const int64_t nlnr = (int64_t)a.side[0].nl * a.k * a.side[0].nr * a.k;
  part_reduce_body(a.out, a.slices, a.side_stride, nlnr, a.ctrl, blockIdx.x * 256ll + threadIdx.x, blockIdx.y);
}

static int run_partials(PartialArgs& a, int nb, hipStream_t st) {
  a.side_stride = (int64_t)a.slices * (4 * a.k) * (6 * a.k);
  a.nb = nb;
  hipLaunchKernelGGL(k_partials, dim3(a.slices, nb), dim3(256), 0, st, a);
  SRP_LAUNCH_CHECK();
  if (a.slices > 1) {
    const int64_t nlnr = (int64_t)a.side[0].nl * a.k * a.side[0].nr * a.k;
    hipLaunchKernelGGL(k_part_reduce, dim3((unsigned)((nlnr + 255) / 256), nb), dim3(256), 0, st, a.out, a.slices,
                       a.side_stride, nlnr, a.ctrl);
    SRP_LAUNCH_CHECK();
  }
  return SRP_OK;
}

// Sum of block (a, b) of the partials: k x k into dst (ld k), scaled.
__device__ void sum_block(const double* part, int slices, int nl, int nr, int k, int a, int b, double scale,
                          double* dst, int tid, int nthreads, bool accumulate) {
  const int NR = nr * k;
  const int64_t zs = (int64_t)(nl * k) * NR;
  for (int e = tid; e < k * k; e += nthreads) {
    const int i = sdiv(e, k), j = e - i * k;
    double s = 0.0;
    for (int z = 0; z < slices; ++z) s += part[z * zs + (int64_t)(a * k + i) * NR + b * k + j];
    dst[e] = accumulate ? dst[e] + scale * s : scale * s;
  }
}

void fill_partial_args(const ProbView& p, int kind, PartialArgs* out) {
  PartialArgs& a = *out;
  a = PartialArgs{};
  a.k = p.k; a.slices = p.part_slices; a.out = p.part; a.ctrl = kind == 2 ? nullptr : p.ctrl;
  a.nb = p.nb;
  a.side_stride = (int64_t)a.slices * (4 * a.k) * (6 * a.k);
  const int k = p.k;
  for (int b = 0; b < p.nb; ++b) {
    const SideView& s = p.s[b];
    PartialSide& q = a.side[b];
    q.d = s.d;
    if (kind == 0) {   // line search: [U | xi]^T [Ks | Js | U | xi | Kc | Jc]
      q.nl = 2; q.nr = 6;
      q.lp[0] = s.U; q.lld[0] = k;
      q.lp[1] = s.xi; q.lld[1] = k;
      q.rp[0] = s.Ks; q.rld[0] = k;
      q.rp[1] = s.J + s.js_off; q.rld[1] = s.jld;
      q.rp[2] = s.U; q.rld[2] = k;
      q.rp[3] = s.xi; q.rld[3] = k;
      q.rp[4] = s.Kc; q.rld[4] = k;
      if (s.Jc_sep) { q.rp[5] = s.Jc_sep; q.rld[5] = k; }
      else { q.rp[5] = s.J + s.jc_off; q.rld[5] = s.jld; }
    } else if (kind == 1) {   // direction: [B U | E]^T [M^-1 B U | M^-1 E | xi | gold]
      q.nl = 2; q.nr = 4;
      q.lp[0] = s.Z + k; q.lld[0] = 2 * k;
      q.lp[1] = s.Z; q.lld[1] = 2 * k;
      q.rp[0] = s.Wz + k; q.rld[0] = 2 * k;
      q.rp[1] = s.Wz; q.rld[1] = 2 * k;
      q.rp[2] = s.xi; q.rld[2] = k;
      q.rp[3] = s.gold; q.rld[3] = k;
    } else {   // finish: U^T [Ks | U | Kc]
      q.nl = 1; q.nr = 3;
      q.lp[0] = s.U; q.lld[0] = k;
      q.rp[0] = s.Ks; q.rld[0] = k;
      q.rp[1] = s.U; q.rld[1] = k;
      q.rp[2] = s.Kc; q.rld[2] = k;
    }
  }
}

int launch_ls_partials(const ProbView& p, hipStream_t st) {
  PartialArgs a;
  fill_partial_args(p, 0, &a);
  return run_partials(a, p.nb, st);
}

int launch_dir_partials(const ProbView& p, hipStream_t st) {
  PartialArgs a;
  fill_partial_args(p, 1, &a);
  return run_partials(a, p.nb, st);
}

int launch_final_partials(const ProbView& p, hipStream_t st) {
  PartialArgs a;
  fill_partial_args(p, 2, &a);
  return run_partials(a, p.nb, st);
}

int launch_partials_g(const PartialArgs* ga, const GroupSel& sel, int max_slices, int64_t max_nlnr,
                      hipStream_t st) {
  if (sel.n <= 0) return SRP_OK;
  hipLaunchKernelGGL(k_partials_g, dim3(max_slices, 2, sel.n), dim3(256), 0, st, ga, sel);
  SRP_LAUNCH_CHECK();
  if (max_slices > 1) {
    hipLaunchKernelGGL(k_part_reduce_g, dim3((unsigned)((max_nlnr + 255) / 256), 2, sel.n), dim3(256), 0, st, ga,
                       sel);
    SRP_LAUNCH_CHECK();
  }
  return SRP_OK;
}

// ------------------------------------------------- small dense helpers
// Sum over the row-slice partials of up to four entries with weights:
// sum_z sum_q w_q part[z * zs + i_q] (q < nq, z < slices <= MAXZ).  The
// partials were written by workgroups on other XCDs, so each load is a
// trip beyond this XCD's L2: all of them are issued before the first is
// used (unrolled to MAXZ), and the sum runs in a fixed order
// (deterministic).  The controllers read the slice sums k_part_reduce
// leaves in slice 0 (MAXZ = 1).
template <int MAXZ = 1>
__device__ __forceinline__ double slice_sum(const double* __restrict__ part, int slices, int64_t zs, int nq,
                                            int64_t i0, int64_t i1, int64_t i2, int64_t i3, double w0,
                                            double w1, double w2, double w3) {
  // unused entries point at i0 with weight 0; unused slices at slice 0 with
  // weight 0: every load is unconditional, so they all issue together
  const int64_t j1 = nq > 1 ? i1 : i0, j2 = nq > 2 ? i2 : i0, j3 = nq > 3 ? i3 : i0;
  const double u1 = nq > 1 ? w1 : 0.0, u2 = nq > 2 ? w2 : 0.0, u3 = nq > 3 ? w3 : 0.0;
  double s = 0.0;
#pragma unroll
  for (int z = 0; z < MAXZ; ++z) {
    const bool on = z < slices;
    const double* pz = part + (int64_t)(on ? z : 0) * zs;
    const double t = (w0 * pz[i0] + u1 * pz[j1]) + (u2 * pz[j2] + u3 * pz[j3]);
    s += on ? t : 0.0;
  }
  return s;
}

// Lower Cholesky in place (ld = k) by one wave; false if not SPD.
__device__ bool wave_chol(double* A, int k, int lane) {
  for (int j = 0; j < k; ++j) {
    wave_sync();
    const double piv = A[j * k + j];
    if (!(piv > 0.0) || !isfinite(piv)) return false;
    const double dj = sqrt(piv);
    wave_sync();
    if (lane == 0) A[j * k + j] = dj;
    for (int i = j + 1 + lane; i < k; i += 64) A[i * k + j] /= dj;
    wave_sync();
    const int w = k - j - 1;
    for (int e = lane; e < w * w; e += 64) {
      const int q = sdiv(e, w), r = j + 1 + q, c = j + 1 + (e - q * w);
      if (c <= r) A[r * k + c] -= A[r * k + j] * A[c * k + j];
    }
  }
  wave_sync();
  return true;
}

// X = L^-1 for lower L (both ld k), column per lane.
__device__ void wave_lower_inv(const double* L, double* X, int k, int lane) {
  for (int c = lane; c < k; c += 64) {
    for (int r = 0; r < c; ++r) X[r * k + c] = 0.0;
    X[c * k + c] = 1.0 / L[c * k + c];
    for (int r = c + 1; r < k; ++r) {
      double s = 0.0;
      for (int l = c; l < r; ++l) s += L[r * k + l] * X[l * k + c];
      X[r * k + c] = -s / L[r * k + r];
    }
  }
  wave_sync();
}

// 1 / x and 1 / sqrt(x) for positive normal x: the hardware estimates
// refined by two Newton steps (within an ulp of the correctly rounded
// values; the divide sequence's scaling for denormal and infinite operands
// is not needed for the pivots these serve).
__device__ __forceinline__ double fast_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}
__device__ __forceinline__ double fast_rsq(double x) {
  double r = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  r = r * fma(-h * r, r, 1.5);
  r = r * fma(-h * r, r, 1.5);
  return r;
}

// The trial evaluations run out of line (their register use stays apart
// from the line search's); their operands are LDS arrays, typed as such so
// that the accesses compile to LDS instructions rather than generic ones.
typedef __attribute__((address_space(3))) double lds_f64;

// Lower Cholesky in place (ld k) by a group of gsize lanes (gl = lane in
// the group); all lanes of the wave run the same loop, so two groups of 32
// factor two matrices side by side.  A non-positive pivot is replaced by 1
// to keep the loop uniform and reported through the return value.
//
// Right-looking and unscaled: step j subtracts A[r][j] A[c][j] / A[j][j]
// from the trailing lower triangle (r >= c > j), whose entries the lanes
// own in NS fixed slots (no index arithmetic per step, one barrier per
// step); column j is final after step j, and all columns are scaled by
// 1 / sqrt(pivot) at the end.  The diagonal of the result holds
// 1 / L[i][i] (the only use of the factor is its inverse below).
template <int NS>
__device__ bool chol_slots(lds_f64* A, int k, int gl, int gsize) {
  const int ntri = k * (k + 1) / 2;
  int sr[NS], sc[NS];
  bool sv[NS];
#pragma unroll
  for (int m = 0; m < NS; ++m) {
    const int e = gl + gsize * m;
    int r = 0;
    while ((r + 1) * (r + 2) / 2 <= e) ++r;   // row of element e of the row-major lower triangle
    sv[m] = e < ntri;
    sr[m] = sv[m] ? r : 0;
    sc[m] = sv[m] ? e - r * (r + 1) / 2 : 0;
  }
  bool ok = true;
  for (int j = 0; j < k; ++j) {
    wave_sync();
    double piv = A[j * k + j];
    if (!(piv > 0.0) || !isfinite(piv)) {
      ok = false;
      piv = 1.0;
    }
    const double rp = fast_rcp(piv);
    // Every slot loads and stores each step (a slot not updated at this
    // step writes back the value it read; each entry of the triangle has
    // one owner, and the clamped slots past the triangle all rewrite entry
    // (0, 0), which no step changes), so no load sits under a branch.
    double nv[NS];
#pragma unroll
    for (int m = 0; m < NS; ++m) {
      const int r = sr[m], c = sc[m];
      const double old = A[r * k + c];
      const double upd = old - A[r * k + j] * A[c * k + j] * rp;
      nv[m] = (sc[m] > j) ? upd : old;
    }
#pragma unroll
    for (int m = 0; m < NS; ++m) A[sr[m] * k + sc[m]] = nv[m];
  }
  wave_sync();
  // Final scaling: the diagonal entries become 1 / sqrt(pivot) (the lower
  // inverse multiplies by them), then L[r][c] = A[r][c] / sqrt(A[c][c]) for
  // r > c as a product with that reciprocal.
  if (gl < k) {
    const double pc = A[gl * k + gl];
    A[gl * k + gl] = fast_rsq((pc > 0.0 && isfinite(pc)) ? pc : 1.0);
  }
  wave_sync();
  double lv[NS];
#pragma unroll
  for (int m = 0; m < NS; ++m) {
    const int r = sr[m], c = sc[m];
    const double x = A[r * k + c];
    lv[m] = (r > c) ? x * A[c * k + c] : x;
  }
  wave_sync();
#pragma unroll
  for (int m = 0; m < NS; ++m)
    if (sv[m] && sr[m] > sc[m]) A[sr[m] * k + sc[m]] = lv[m];
  wave_sync();
  return ok;
}

// Picks the slot count ceil(k (k + 1) / 2 / gsize) (uniform over the wave),
// so a small k in a large instance loads no more than it needs.
template <int NS, int MAXS>
__device__ __forceinline__ bool chol_dispatch(int ns, lds_f64* A, int k, int gl, int gsize) {
  if constexpr (NS >= MAXS) {
    return chol_slots<MAXS>(A, k, gl, gsize);
  } else {
    if (ns <= NS) return chol_slots<NS>(A, k, gl, gsize);
    return chol_dispatch<NS + 1, MAXS>(ns, A, k, gl, gsize);
  }
}

template <int KC>
__device__ bool group_chol(lds_f64* A, int k, int gl, int gsize) {
  constexpr int MAXS = (KC * (KC + 1) / 2 + 31) / 32;
  const int ns = (k * (k + 1) / 2 + gsize - 1) / gsize;
  return chol_dispatch<1, MAXS>(ns, A, k, gl, gsize);
}

// X = L^-1 for lower L (ld k) whose diagonal holds 1 / L[i][i] (as
// group_chol leaves it): lane c of the group forward-substitutes column c
// of X in registers (no cross-lane dependence, no LDS round trip inside the
// chain).  Row r of L arrives as broadcast loads, so a step of the chain is
// the dot product of the row with the finished entries and one multiply.  An empty
// asm statement with a memory clobber keeps each row's loads in its own
// step (hoisting all of them ahead of the chain would exhaust registers).
template <int KC>
__device__ void group_lower_inv(const lds_f64* L, lds_f64* X, int k, int gl) {
  if (gl < k) {
    const int c = gl;
    double x[KC];
#pragma unroll
    for (int r = 0; r < KC; ++r) {
      double v = 0.0;
      if (r < k) {
        asm volatile("" ::: "memory");
        const double rinv = L[r * k + r];   // the factor's diagonal holds 1 / L[r][r]
        double acc4[4] = {0.0, 0.0, 0.0, 0.0};   // four short chains instead of one long one
#pragma unroll
        for (int l = 0; l < r; ++l) acc4[l & 3] += L[r * k + l] * x[l];   // x[l] = 0 for l < c
        const double s = ((r == c) ? 1.0 : 0.0) - ((acc4[0] + acc4[1]) + (acc4[2] + acc4[3]));
        v = (r >= c) ? s * rinv : 0.0;
      }
      x[r] = v;
    }
#pragma unroll
    for (int r = 0; r < KC; ++r)
      if (r < k) X[r * k + c] = x[r];
  }
  wave_sync();
}

// sum_i mu_i (Lx^-1 C Ly^-T)_ii with Xx = Lx^-1, Xy = Ly^-1 (lower, ld k),
// by one wave: M = C Xy^T on FP64 matrix cores (16x16 tiles), then each
// lane weighs the entries M[a][i] it holds by mu_i Xx[i][a]; reduced over
// the wave.
template <int KC>
__device__ double trial_cost(const lds_f64* C, const lds_f64* Xx, const lds_f64* Xy, const lds_f64* mu, int k,
                             int lane) {
  constexpr int T = (KC + 15) / 16;
  const int m16 = lane & 15, q = lane >> 4;
  double part = 0.0;
#pragma unroll
  for (int ta = 0; ta < T; ++ta)
#pragma unroll
    for (int ti = 0; ti < T; ++ti) {
      if (16 * ta >= k || 16 * ti >= k) continue;   // uniform: tiles past k are zero
      f64x4 acc = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kb = 0; kb < (KC + 3) / 4; ++kb) {
        if (4 * kb >= k) break;   // uniform: blocks past k contribute nothing
        const int a = 16 * ta + m16, b = 4 * kb + q, i = 16 * ti + m16;
        const int ac = a < k ? a : k - 1, bc = b < k ? b : k - 1, ic = i < k ? i : k - 1;
        const double cv = C[ac * k + bc], yv = Xy[ic * k + bc];
        acc = mfma16x16x4((a < k && b < k) ? cv : 0.0, (b < k && i < k) ? yv : 0.0, acc);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = 16 * ta + acc_row<double>(lane, r), i = 16 * ti + m16;
        const int ac = a < k ? a : 0, ic = i < k ? i : 0;
        const double w = mu[ic] * Xx[ic * k + ac];
        part += (a < k && i < k) ? w * acc[r] : 0.0;
      }
    }
  for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
  return part;
}

// Line-search polynomial coefficients, k x k each, in LDS:
// [side b][G0, G1, G2] then [C0, C1, C2] (CCA cross or FDA S_B).
__device__ __forceinline__ const double* coefp(const double* base, int k, int idx) {
  return base + (size_t)idx * k * k;
}
__device__ __forceinline__ const lds_f64* coefp(const lds_f64* base, int k, int idx) {
  return base + idx * k * k;
}

// Cost along the curve at step t, evaluated by one wave.  CCA factors the
// two Grams in the two half-waves; Lm holds nb k x k factors, Li their
// inverses; C(t) is staged into Lm once the factors have been inverted.
template <int KC>
__device__ __attribute__((noinline)) double eval_trial(const ProbView& p, const lds_f64* coef, const lds_f64* mu, double t,
                                                      lds_f64* Lm, lds_f64* Li, int lane, bool* ok) {
  const int k = p.k, nb = p.nb, kk2 = k * k;
  const int gsize = nb == 2 ? 32 : 64;
  const int grp = nb == 2 ? (lane >> 5) : 0;
  const int gl = nb == 2 ? (lane & 31) : lane;
  const double t2 = t * t;
  {
    lds_f64* L = Lm + grp * kk2;
    const lds_f64* G0 = coefp(coef, k, 3 * grp + 0);
    const lds_f64* G1 = coefp(coef, k, 3 * grp + 1);
    const lds_f64* G2 = coefp(coef, k, 3 * grp + 2);
    for (int e = gl; e < kk2; e += gsize) L[e] = G0[e] + t * G1[e] + t2 * G2[e];
    const bool good = group_chol<KC>(L, k, gl, gsize);
    *ok = __all(good ? 1 : 0) != 0;
    group_lower_inv<KC>(L, Li + grp * kk2, k, gl);
  }
  if (!*ok) return INFINITY;
  const lds_f64* C0 = coefp(coef, k, 3 * nb + 0);
  const lds_f64* C1 = coefp(coef, k, 3 * nb + 1);
  const lds_f64* C2 = coefp(coef, k, 3 * nb + 2);
  lds_f64* Ct = Lm;
  for (int e = lane; e < kk2; e += 64) Ct[e] = C0[e] + t * C1[e] + t2 * C2[e];
  wave_sync();
  const double s = trial_cost<KC>(Ct, Li, Li + (nb == 2 ? kk2 : 0), mu, k, lane);
  const double f = p.lda_cost ? -0.5 * s : -s;
  return isfinite(f) ? f : INFINITY;
}

// -------------------------------------------------------- line search
// One workgroup.  All threads first reduce the row-slice partials into the
// polynomial coefficients (LDS); then each round evaluates ntr trial steps
// on a geometric grid in parallel (one wave each), keeps the best and
// narrows the grid around it.  The winning wave's factor inverses are
// stored directly when the best step comes from the last round.
constexpr int kLsThreads = 512;   // 8 trial steps per round

template <int KC>
__device__ __forceinline__ void ctrl_ls_body(const ProbView& p, int ntr) {
  SolverCtrl* c = p.ctrl;
  if (c->done) return;
  extern __shared__ double sm[];
  __shared__ double fbest[64];
  __shared__ double tbest[64];
  __shared__ int okflag[64];
  __shared__ double mu[KC];
  const int k = p.k, nb = p.nb, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int kk2 = k * k;
  const int slices = 1;   // k_part_reduce left the slice sums in slice 0
  const int NR = 6 * k;
  const int64_t zs = (int64_t)(2 * k) * NR;
  const int64_t side_stride = (int64_t)p.part_slices * (4 * k) * (6 * k);   // as laid out by run_partials
  double* coef = sm;                                 // (3 nb + 3) k x k
  const int ncoef = 3 * nb + 3;
  // coefficients (ls partial layout: left [U, xi], right [Ks, Js, U, xi, Kc, Jc])
  for (int e = tid; e < ncoef * kk2; e += kLsThreads) {
    const int m = sdiv(e, kk2), q = e - m * kk2, i = sdiv(q, k), j = q - i * k;
    const int64_t r0 = (int64_t)i * NR + j, r1 = (int64_t)(k + i) * NR + j;   // rows of U and xi
    double v;
    if (m < 3 * nb) {
      const int b = m / 3, which = m - 3 * b;
      const double lam = p.s[b].lam;
      const double* part = p.part + b * side_stride;
      if (which == 0)        // G0 = U^T Ks + lam U^T U
        v = slice_sum(part, slices, zs, 2, r0, r0 + 2 * k, 0, 0, 1.0, lam, 0.0, 0.0);
      else if (which == 1)   // G1 = xi^T Ks + U^T Js + lam (xi^T U + U^T xi)
        v = slice_sum(part, slices, zs, 4, r1, r0 + k, r1 + 2 * k, r0 + 3 * k, 1.0, 1.0, lam, lam);
      else                   // G2 = xi^T Js + lam xi^T xi
        v = slice_sum(part, slices, zs, 2, r1 + k, r1 + 3 * k, 0, 0, 1.0, lam, 0.0, 0.0);
    } else {
      const int which = m - 3 * nb;   // side 0 carries the cost products
      if (which == 0)        // C0 = U^T Kc
        v = slice_sum(p.part, slices, zs, 1, r0 + 4 * k, 0, 0, 0, 1.0, 0.0, 0.0, 0.0);
      else if (which == 1)   // C1 = xi^T Kc + U^T Jc
        v = slice_sum(p.part, slices, zs, 2, r1 + 4 * k, r0 + 5 * k, 0, 0, 1.0, 1.0, 0.0, 0.0);
      else                   // C2 = xi^T Jc
        v = slice_sum(p.part, slices, zs, 1, r1 + 5 * k, 0, 0, 0, 1.0, 0.0, 0.0, 0.0);
    }
    coef[e] = v;
  }
  for (int e = tid; e < k; e += kLsThreads) mu[e] = p.mu[e];
  __syncthreads();
  // symmetrise the Gram coefficients (and the FDA cost coefficients)
  const int nsym = 3 * nb + (p.lda_cost ? 3 : 0);
  for (int e = tid; e < nsym * kk2; e += kLsThreads) {
    const int m = sdiv(e, kk2), q = e - m * kk2, i = sdiv(q, k), j = q - i * k;
    if (i < j) {
      double* M = coef + (size_t)m * kk2;
      const double v = 0.5 * (M[i * k + j] + M[j * k + i]);
      M[i * k + j] = v;
      M[j * k + i] = v;
    }
  }
  __syncthreads();

  const int per_wave = 2 * nb * kk2;
  double* Lm = sm + (size_t)ncoef * kk2 + (size_t)w * per_wave;
  double* Li = Lm + nb * kk2;
  const double f0 = c->f;
  const double df0 = c->df0;
  double t_acc = 0.0;
  double t_seen = 0.0;   // best step of the search, accepted or not
  bool accepted = false;
  int winner = -1;       // wave holding the factors of the best step
  if (c->fixed_step) {
    t_acc = 1.0;
    accepted = true;
  } else {
    // First step: the inverse of the cost's curvature scale, about
    // 1 / (2 mu_1 |f| / sum mu); afterwards the last accepted step.
    double centre = c->t_guess;
    if (!(centre > 0.0)) {
      double smu = 0.0;
      for (int i = 0; i < k; ++i) smu += mu[i];
      centre = (fabs(f0) > 0.0) ? smu / (2.0 * mu[0] * fabs(f0)) : 1.0;
    }
    double H = 3.0;  // half span in octaves (the grid moves when the best step is on its edge)
    double tb = centre, fb = INFINITY;
    int expand = 0;
    for (int round = 0; round < 16 && H > 0.25; ++round) {
      if (w < ntr) {
        const double x = (ntr > 1) ? (2.0 * w / (ntr - 1) - 1.0) : 0.0;
        const double t = centre * exp2(H * x);
        bool ok;
        const double f = eval_trial<KC>(p, (const lds_f64*)coef, (const lds_f64*)mu, t, (lds_f64*)Lm, (lds_f64*)Li, lane, &ok);
        if (lane == 0) { fbest[w] = f; tbest[w] = t; }
      }
      __syncthreads();
      if (tid == 0) {
        int best = -1;
        for (int j = 0; j < ntr; ++j)
          if (fbest[j] < INFINITY && (best < 0 || fbest[j] < fbest[best])) best = j;
        int win = -1;
        if (best >= 0 && fbest[best] < fb) {
          fb = fbest[best];
          tb = tbest[best];
          win = best;
        }
        okflag[2] = win;
        // minimum on the edge of the grid: move the grid there, same span
        okflag[1] = (best == 0 || best == ntr - 1) && expand < 6 ? 1 : 0;
        fbest[63] = fb;
        tbest[63] = tb;
      }
      __syncthreads();
      fb = fbest[63];
      tb = tbest[63];
      centre = tb;
      winner = okflag[2] >= 0 ? okflag[2] : -1;
      if (okflag[1]) {
        ++expand;
      } else {
        H = (ntr > 1) ? 2.0 * H / (ntr - 1) : 0.5 * H;
      }
      __syncthreads();
    }
    t_seen = tb;
    // Armijo sufficient decrease
    if (fb < INFINITY && df0 < 0.0 && fb <= f0 + 1e-4 * tb * df0) {
      t_acc = tb;
      accepted = true;
    } else if (fb < INFINITY && fb < f0 && df0 < 0.0) {
      t_acc = tb;  // decrease without the Armijo margin: still progress
      accepted = true;
    }
    if (accepted && winner >= 0 && tbest[winner] != t_acc) winner = -1;
    if (!accepted) winner = -1;
  }
  // factors at the accepted step: from the winning wave, else recomputed
  // by wave 0 (t = 0 re-orthonormalises on failure)
  const int src = winner >= 0 ? winner : 0;
  if (w == src) {
    double f;
    bool ok = true;
    if (winner >= 0) f = fbest[63];
    else f = eval_trial<KC>(p, (const lds_f64*)coef, (const lds_f64*)mu, t_acc, (lds_f64*)Lm, (lds_f64*)Li, lane, &ok);
    if (lane == 0) { fbest[62] = f; okflag[0] = ok ? 1 : 0; }
    wave_sync();
    for (int b = 0; b < nb; ++b) {
      double* LT = kkslot(p, b, KK_LINVT);
      const double* X = Li + b * kk2;
      for (int e = lane; e < kk2; e += 64) {
        const int i = sdiv(e, k), j = e - i * k;
        LT[i * k + j] = X[j * k + i];
      }
    }
  }
  __syncthreads();
  if (tid == 0) {
    if (!okflag[0]) {
      c->done = 1;
      c->status = SRP_ENOTSPD;
      c->t = 0.0;
    } else if (accepted) {
      c->t = t_acc;
      c->f = fbest[62];
      c->t_guess = t_acc;
      c->ls_fail = 0;
    } else {
      c->t = 0.0;
      c->f = fbest[62];
      c->restart = 1;
      c->ls_fail += 1;
      c->t_guess = (t_seen > 0.0 ? t_seen : 1.0) / 16.0;
      if (c->ls_fail >= 3) c->done = 1;  // no further decrease at working precision
    }
    c->fixed_step = 0;
  }
}

template <int KC>
__global__ void __launch_bounds__(kLsThreads) k_ctrl_ls(ProbView p, int ntr) { ctrl_ls_body<KC>(p, ntr); }

// Grouped: one workgroup per solve, sel.aux holds each solve's trial count.
template <int KC>
__global__ void __launch_bounds__(kLsThreads) k_ctrl_ls_g(const ProbView* __restrict__ v, GroupSel sel) {
  ctrl_ls_body<KC>(v[sel.idx[blockIdx.x]], sel.aux[blockIdx.x]);
}

int ctrl_ls_shape(int k, int nb, size_t* lds) {
  const size_t coef_bytes = (size_t)(3 * nb + 3) * k * k * sizeof(double);
  const size_t per_wave = (size_t)2 * nb * k * k * sizeof(double);
  const size_t budget = 156 * 1024;
  int ntr = (int)((budget - coef_bytes) / per_wave);
  if (ntr > kLsThreads / 64) ntr = kLsThreads / 64;
  *lds = coef_bytes + (size_t)(ntr > 0 ? ntr : 0) * per_wave;
  return ntr;
}

template <int KC>
static int launch_ctrl_ls_t(const ProbView& p, hipStream_t st) {
  const int k = p.k;
  size_t lds = 0;
  const int ntr = ctrl_ls_shape(k, p.nb, &lds);
  if (ntr < 1) {
    set_error("line search: k = %d too large for the LDS budget", k);
    return SRP_EINVAL;
  }
  SRP_TRY(allow_dynamic_lds((const void*)k_ctrl_ls<KC>, lds));
  hipLaunchKernelGGL(k_ctrl_ls<KC>, dim3(1), dim3(kLsThreads), lds, st, p, ntr);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

int launch_ctrl_ls(const ProbView& p, hipStream_t st) {
  if (p.k <= 16) return launch_ctrl_ls_t<16>(p, st);
  return launch_ctrl_ls_t<32>(p, st);
}

int launch_ctrl_ls_g(const ProbView* v, const GroupSel& sel, size_t lds, int kc, hipStream_t st) {
  if (sel.n <= 0) return SRP_OK;
  if (kc == 16) {
    SRP_TRY(allow_dynamic_lds((const void*)k_ctrl_ls_g<16>, lds));
    hipLaunchKernelGGL(k_ctrl_ls_g<16>, dim3(sel.n), dim3(kLsThreads), lds, st, v, sel);
  } else {
    SRP_TRY(allow_dynamic_lds((const void*)k_ctrl_ls_g<32>, lds));
    hipLaunchKernelGGL(k_ctrl_ls_g<32>, dim3(sel.n), dim3(kLsThreads), lds, st, v, sel);
  }
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

// ------------------------------------------------------------- update
// Per row: U+ = (U + t xi) Linv^T, Ks+ = (Ks + t Js) Linv^T,
// Kc+ = (Kc + t Jc) Linv_o^T; then Z = [-Kc+ N | Ks+ + lam U+].
// refresh = 1: Ks = Js, Kc = Jc at the current U (exact products);
// refresh = 2: the same, also after the stop flag is set.
// A workgroup stages 16 rows in LDS, then one thread per (row, column).
constexpr int kUpdRows = 16;

template <int KC>
__device__ __forceinline__ void update_body(const ProbView& p, int refresh, int bx, int b) {
  const SolverCtrl* c = p.ctrl;
  if (c->done && refresh != 2) return;   // 2 = forced refresh after the loop
  const SideView& s = p.s[b];
  const int o = (p.nb == 2) ? 1 - b : b;
  const int k = p.k;
  const int r0 = bx * kUpdRows;
  if (r0 >= s.d) return;
  const int nr = min(kUpdRows, s.d - r0);
  __shared__ double LT[KMAX * KMAX], LTo[KMAX * KMAX], mu[KMAX];
  __shared__ double u[kUpdRows][KMAX], ks[kUpdRows][KMAX], kc[kUpdRows][KMAX];
  const double t = c->t;
  const int tid = threadIdx.x;
  if (!refresh) {
    const double* gLT = kkslot(p, b, KK_LINVT);
    const double* gLTo = kkslot(p, o, KK_LINVT);
    for (int e = tid; e < k * k; e += 256) { LT[e] = gLT[e]; LTo[e] = gLTo[e]; }
  }
  for (int e = tid; e < k; e += 256) mu[e] = p.mu[e];
  for (int e = tid; e < nr * k; e += 256) {
    const int rr = sdiv(e, k), j = e - rr * k;
    const int64_t i = r0 + rr;
    const double* Jrow = s.J + i * s.jld;
    const double js = Jrow[s.js_off + j];
    const double jc = s.Jc_sep ? s.Jc_sep[i * k + j] : Jrow[s.jc_off + j];
    if (refresh) {
      u[rr][j] = s.U[i * k + j];
      ks[rr][j] = js;
      kc[rr][j] = jc;
    } else {
      u[rr][j] = s.U[i * k + j] + t * s.xi[i * k + j];
      ks[rr][j] = s.Ks[i * k + j] + t * js;
      kc[rr][j] = s.Kc[i * k + j] + t * jc;
    }
  }
  __syncthreads();
  for (int e = tid; e < nr * k; e += 256) {
    const int rr = sdiv(e, k), j = e - rr * k;
    const int64_t i = r0 + rr;
    double un, ksn, kcn;
    if (refresh) {
      un = u[rr][j]; ksn = ks[rr][j]; kcn = kc[rr][j];
    } else {
      double u2[2] = {0.0, 0.0}, k2[2] = {0.0, 0.0}, c2[2] = {0.0, 0.0};
#pragma unroll
      for (int l = 0; l < KC; ++l) {   // unconditional LDS loads, masked terms
        const int lc = l < k ? l : 0;
        const double lt = LT[lc * k + j], lto = LTo[lc * k + j];
        const double a1 = u[rr][lc] * lt, a2 = ks[rr][lc] * lt, a3 = kc[rr][lc] * lto;
        u2[l & 1] += (l < k) ? a1 : 0.0;
        k2[l & 1] += (l < k) ? a2 : 0.0;
        c2[l & 1] += (l < k) ? a3 : 0.0;
      }
      un = u2[0] + u2[1]; ksn = k2[0] + k2[1]; kcn = c2[0] + c2[1];
      s.U[i * k + j] = un;
      s.Ks[i * k + j] = ksn;
    }
    s.Kc[i * k + j] = kcn;
    if (refresh) s.Ks[i * k + j] = ksn;
    double* Zi = s.Z + i * 2 * k;
    Zi[j] = -kcn * mu[j];
    Zi[k + j] = ksn + s.lam * un;
  }
}

template <int KC>
__global__ void __launch_bounds__(256) k_update(ProbView p, int refresh) {
  update_body<KC>(p, refresh, blockIdx.x, blockIdx.y);
}

template <int KC>
__global__ void __launch_bounds__(256) k_update_g(const ProbView* __restrict__ v, GroupSel sel, int refresh) {
  const ProbView& p = v[sel.idx[blockIdx.z]];
  if ((int)blockIdx.y >= p.nb) return;
  update_body<KC>(p, refresh, blockIdx.x, blockIdx.y);
}

int launch_update_g(const ProbView* v, const GroupSel& sel, int refresh, int dmax, int kc, hipStream_t st) {
  if (sel.n <= 0) return SRP_OK;
  dim3 grid((dmax + kUpdRows - 1) / kUpdRows, 2, sel.n);
  if (kc == 16) hipLaunchKernelGGL(k_update_g<16>, grid, dim3(256), 0, st, v, sel, refresh);
  else hipLaunchKernelGGL(k_update_g<32>, grid, dim3(256), 0, st, v, sel, refresh);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

int launch_update(const ProbView& p, int refresh, hipStream_t st) {
  const int dmax = p.nb == 2 ? (p.s[0].d > p.s[1].d ? p.s[0].d : p.s[1].d) : p.s[0].d;
  dim3 grid((dmax + kUpdRows - 1) / kUpdRows, p.nb);
  if (p.k <= 16) hipLaunchKernelGGL(k_update<16>, grid, dim3(256), 0, st, p, refresh);
  else hipLaunchKernelGGL(k_update<32>, grid, dim3(256), 0, st, p, refresh);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

// ---------------------------------------------- Jacobi eigen-solver
// Parallel cyclic Jacobi (round-robin pairs) on a symmetric n x n matrix
// (n even, <= 64) by ONE wave: A is overwritten by the (near) diagonal
// matrix and V accumulates the rotations, A_in = V D V^T.  Scratch: T
// (2 n x n; A and V alternate with it round by round) and the rotation
// of each index.  Round r pairs the indices in slots i and n - 1 - i,
// slot 0 holding index 0 and slot s > 0 index 1 + (s - 1 + r) mod (n - 1);
// a lane finds the partner of an index from that rule, so a round reads
// the rotations and the matrix entries in one batch.
struct WaveJacobiScratch {
  double rc[64];   // cosine of the rotation of index i
  double rs[64];   // signed sine: -s for the first index of a pair, +s for the second
};

__device__ __forceinline__ int jac_index(int slot, int round, int n1) {
  if (slot == 0) return 0;
  int x = slot - 1 + round;
  if (x >= n1) x -= n1;
  return 1 + x;
}
__device__ __forceinline__ int jac_partner(int idx, int round, int n) {
  const int n1 = n - 1;
  int slot = 0;
  if (idx != 0) {
    int x = idx - 1 - round;
    if (x < 0) x += n1;
    slot = 1 + x;
  }
  return jac_index(n1 - slot, round, n1);
}

// Cosine (returned) and sine of the rotation that zeroes the (p, q) entry,
// t = sign(theta) / (|theta| + sqrt(theta^2 + 1)), c = 1 / sqrt(t^2 + 1):
// the arguments of the square roots and reciprocals are >= 1, so the
// Newton-refined hardware estimates serve (within an ulp). Past |theta| =
// 1e150 (theta^2 would overflow) t is 1 / (2 theta) to working precision
// (clamped at 1e300 so that an infinite theta gives t ~ 5e-301, c = 1).
__device__ __forceinline__ double jac_rotation(double theta, double* sn) {
  const double at = fabs(theta);
  const bool big = at >= 1e150;
  const double as = big ? 0.0 : at;
  const double h = fma(as, as, 1.0);
  const double den = big ? 2.0 * fmin(at, 1e300) : as + h * fast_rsq(h);
  const double tt = (theta >= 0.0 ? 1.0 : -1.0) * fast_rcp(den);
  const double cth = fast_rsq(fma(tt, tt, 1.0));
  *sn = tt * cth;
  return cth;
}

__device__ void wave_jacobi(double* A, double* V, double* T, int n, int lane, WaveJacobiScratch& w,
                            double tol2 = 1e-30) {
  const int nn = n * n, n1 = n - 1;
  double* a = A;
  double* v = V;
  double* a2 = T;
  double* v2 = T + nn;
  for (int e = lane; e < nn; e += 64) V[e] = (e == sdiv(e, n) * (n + 1)) ? 1.0 : 0.0;
  wave_sync();
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int e = lane; e < nn; e += 64) {
      const double x = a[e];
      if (e == sdiv(e, n) * (n + 1)) dia += x * x; else off += x * x;
    }
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_xor(off, o, 64);
      dia += __shfl_xor(dia, o, 64);
    }
    if (off <= tol2 * (dia + 1e-300)) break;
    for (int round = 0; round < n1; ++round) {
      if (lane < n / 2) {
        int pp = jac_index(lane, round, n1), qq = jac_index(n1 - lane, round, n1);
        if (pp > qq) { const int tmp = pp; pp = qq; qq = tmp; }
        const double apq = a[pp * n + qq], app = a[pp * n + pp], aqq = a[qq * n + qq];
        double cth = 1.0, sth = 0.0;
        if (apq != 0.0) {
          const double theta = (aqq - app) / (2.0 * apq);
          cth = jac_rotation(theta, &sth);
        }
        w.rc[pp] = cth; w.rs[pp] = -sth;
        w.rc[qq] = cth; w.rs[qq] = sth;
      }
      wave_sync();
      // A' = J^T A J, V' = V J with J[p][p] = c, J[p][q] = s, J[q][p] = -s, J[q][q] = c
      for (int e = lane; e < nn; e += 64) {
        const int r = sdiv(e, n), col = e - r * n;
        const int pr = jac_partner(r, round, n), pc = jac_partner(col, round, n);
        const double cr = w.rc[r], sr = w.rs[r], cc = w.rc[col], sc = w.rs[col];
        a2[e] = cr * (cc * a[r * n + col] + sc * a[r * n + pc]) + sr * (cc * a[pr * n + col] + sc * a[pr * n + pc]);
        v2[e] = v[r * n + col] * cc + v[r * n + pc] * sc;
      }
      wave_sync();
      double* t = a; a = a2; a2 = t;
      t = v; v = v2; v2 = t;
    }
  }
  if (a != A) {
    for (int e = lane; e < nn; e += 64) {
      A[e] = a[e];
      V[e] = v[e];
    }
  }
  wave_sync();
}

// The same rotations by a whole workgroup, one group of waves per matrix:
// nv symmetric n x n matrices (n even, <= 64; nv <= 2), matrix v handled
// by the threads with tid % nv == v (gt = tid / nv in the group, GW =
// blockDim / nv of them).  Every thread of the block calls it; the rounds
// are separated by block barriers, and a matrix that has converged stops
// rotating (its group only takes the barriers) while the others go on, so
// each matrix gets the same sweeps as alone.  (Further sweeps of a
// converged matrix would rotate freely inside nearly equal eigenvalues.)
// psum holds one (off, dia) pair per wave; the group sums read it in wave
// order, so every thread takes the same decisions.
__device__ void block_jacobi(double* const* Av, double* const* Vv, double* const* Tv, WaveJacobiScratch* w,
                             double (*psum)[2], int nv, int n, double tol2) {
  const int tid = threadIdx.x, nt = blockDim.x, nwaves = nt >> 6;
  const int v = tid % nv, gt = tid / nv, GW = nt / nv;
  const int nn = n * n, n1 = n - 1;
  double* a = Av[v];
  double* vv = Vv[v];
  double* a2 = Tv[v];
  double* v2 = Tv[v] + nn;
  for (int e = gt; e < nn; e += GW) vv[e] = (e == sdiv(e, n) * (n + 1)) ? 1.0 : 0.0;
  int flips = 0;
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int e = gt; e < nn; e += GW) {
      const double x = a[e];
      if (e == sdiv(e, n) * (n + 1)) dia += x * x; else off += x * x;
    }
    // per wave: lanes of one wave alternate between the matrices when nv = 2,
    // so reduce the lanes of each parity separately
    for (int o = 32; o >= nv; o >>= 1) {
      off += __shfl_xor(off, o, 64);
      dia += __shfl_xor(dia, o, 64);
    }
    if ((tid & 63) < nv) { psum[(tid >> 6) * nv + v][0] = off; psum[(tid >> 6) * nv + v][1] = dia; }
    __syncthreads();
    bool all = true, act = false;
    for (int m = 0; m < nv; ++m) {
      double so = 0.0, sd = 0.0;
      for (int q = 0; q < nwaves; ++q) { so += psum[q * nv + m][0]; sd += psum[q * nv + m][1]; }
      const bool cm = so <= tol2 * (sd + 1e-300);
      all = all && cm;
      if (m == v) act = !cm;
    }
    __syncthreads();
    if (all) break;
    for (int round = 0; round < n1; ++round) {
      if (act && gt < n / 2) {
        int pp = jac_index(gt, round, n1), qq = jac_index(n1 - gt, round, n1);
        if (pp > qq) { const int tmp = pp; pp = qq; qq = tmp; }
        const double apq = a[pp * n + qq], app = a[pp * n + pp], aqq = a[qq * n + qq];
        double cth = 1.0, sth = 0.0;
        if (apq != 0.0) {
          const double theta = (aqq - app) / (2.0 * apq);
          cth = jac_rotation(theta, &sth);
        }
        w[v].rc[pp] = cth; w[v].rs[pp] = -sth;
        w[v].rc[qq] = cth; w[v].rs[qq] = sth;
      }
      __syncthreads();
      if (act) {
        for (int e = gt; e < nn; e += GW) {
          const int r = sdiv(e, n), col = e - r * n;
          const int pr = jac_partner(r, round, n), pc = jac_partner(col, round, n);
          const double cr = w[v].rc[r], sr = w[v].rs[r], cc = w[v].rc[col], sc = w[v].rs[col];
          a2[e] = cr * (cc * a[r * n + col] + sc * a[r * n + pc]) + sr * (cc * a[pr * n + col] + sc * a[pr * n + pc]);
          v2[e] = vv[r * n + col] * cc + vv[r * n + pc] * sc;
        }
      }
      __syncthreads();
      if (act) {
        double* t = a; a = a2; a2 = t;
        t = vv; vv = v2; v2 = t;
        ++flips;
      }
    }
  }
  if (flips & 1) {   // the result sits in the scratch: copy it back (group-uniform)
    for (int e = gt; e < nn; e += GW) {
      Av[v][e] = a[e];
      Vv[v][e] = vv[e];
    }
  }
  __syncthreads();
}

// ------------------------------------------ register Jacobi, one wave
// The same parallel cyclic Jacobi for n <= 20 (n even) with the matrix in
// registers.  Positions 2i and 2i + 1 hold the two indices of pair i;
// lane b owns the 2 x 2 block of pair rows i and pair columns j (i <= j;
// the blocks below the diagonal are the transposes; P (P + 1) / 2 <= 64
// blocks for P = n / 2 pairs).
// A round rotates every block by the rotations of its two pairs, which
// each lane computes itself from the diagonal blocks of those pairs (read
// beside its own entries), then moves the entries to the next pairing in
// one exchange through LDS at fixed addresses: position u takes the index
// that stood at rr_src(u) (index 0 stays, the other n - 1 turn one step
// round a circle), so every two indices meet once in a sweep of n - 1
// rounds and a sweep ends in the order it began.  The entry a rotation
// annihilates is set to zero.  The rows of V do not move; its column pairs
// are rotated by lanes that already hold the pair's rotation: lane (i, j)
// keeps rows 2i, 2i + 1 of column pair j and, for i < j, rows 2j, 2j + 1
// of column pair i.  On return A holds the rotated matrix (the eigenvalues
// on its diagonal) and V the eigenvectors, A_in = V D V^T.  Scratch T:
// 2 n x n.
__device__ __forceinline__ int rr_src(int u, int P) {
  if (P == 1 || u == 0) return u;
  const int i = u >> 1;
  if ((u & 1) == 0) return i == 1 ? 1 : u - 2;
  return i == P - 1 ? u - 1 : u + 2;
}

// Rotation of a pair from its diagonal block (app, apq, aqq), free of
// divisions: x = aqq - app and y = 2 apq are scaled by a common power of
// two (exactly, so that no square below can overflow), r = sqrt(x^2 + y^2)
// and D = |x| + r give the tangent sign(x) y / D of the classical choice
// (the smaller angle), hence c = D / sqrt(D^2 + y^2) and
// s = sign(x) y / sqrt(D^2 + y^2) with two reciprocal square roots;
// c = 1, s = 0 when apq is zero.
__device__ __forceinline__ void pair_rot(double app, double apq, double aqq, double* c, double* s) {
  const double x0 = aqq - app, y0 = 2.0 * apq;
  const bool z = apq == 0.0;
  const int e = __builtin_amdgcn_frexp_exp(z ? 1.0 : fmax(fabs(x0), fabs(y0)));
  const double x = __builtin_amdgcn_ldexp(x0, -e), y = __builtin_amdgcn_ldexp(y0, -e);
  const double h = fma(x, x, y * y);   // in [1/4, 2)
  const double d = fabs(x) + h * fast_rsq(h);
  const double q = fast_rsq(fma(d, d, y * y));
  *c = z ? 1.0 : d * q;
  *s = z ? 0.0 : (x0 >= 0.0 ? y : -y) * q;
}

__device__ void pair_jacobi(double* A, double* V, double* T, int n, int lane, double tol2) {
  const int P = n >> 1;
  double* MA = T;
  double* MV = T + n * n;
  // this lane's block (i, j): the upper blocks row by row
  const bool ok = lane < P * (P + 1) / 2;
  int i = 0, rem = ok ? lane : 0;
  while (rem >= P - i) {
    rem -= P - i;
    ++i;
  }
  const int j = i + rem;
  const bool diag = i == j;
  // positions whose entries move to this lane's in the next round
  const int si0 = rr_src(2 * i, P), si1 = rr_src(2 * i + 1, P);
  const int sj0 = rr_src(2 * j, P), sj1 = rr_src(2 * j + 1, P);
  double x[4];    // entry (2i + r, 2j + c) at 2r + c
  double dg[6];   // diagonal blocks of pairs i and j: (pp, pq, qq) each
  double v[8];    // V: rows 2i + r of column pair j at 2r + c; rows 2j + r of pair i at 4 + 2r + c
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int r = e >> 1, c = e & 1;
    x[e] = A[(2 * i + r) * n + 2 * j + c];
    v[e] = (diag && r == c) ? 1.0 : 0.0;
    v[4 + e] = 0.0;
  }
  dg[0] = A[(2 * i) * n + 2 * i];
  dg[1] = A[(2 * i) * n + 2 * i + 1];
  dg[2] = A[(2 * i + 1) * n + 2 * i + 1];
  dg[3] = A[(2 * j) * n + 2 * j];
  dg[4] = A[(2 * j) * n + 2 * j + 1];
  dg[5] = A[(2 * j + 1) * n + 2 * j + 1];
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0.0, dia = 0.0;
    if (ok) {
      if (diag) {
        dia = x[0] * x[0] + x[3] * x[3];
        off = 2.0 * x[1] * x[1];
      } else {
        off = 2.0 * (x[0] * x[0] + x[1] * x[1] + x[2] * x[2] + x[3] * x[3]);
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_xor(off, o, 64);
      dia += __shfl_xor(dia, o, 64);
    }
    if (off <= tol2 * (dia + 1e-300)) break;
    for (int round = 0; round < n - 1; ++round) {
      double ci, si, cj, sj;
      pair_rot(dg[0], dg[1], dg[2], &ci, &si);
      pair_rot(dg[3], dg[4], dg[5], &cj, &sj);
      // right by the rotation of pair j, then left by that of pair i
      const double y00 = cj * x[0] - sj * x[1], y01 = cj * x[1] + sj * x[0];
      const double y10 = cj * x[2] - sj * x[3], y11 = cj * x[3] + sj * x[2];
      x[0] = ci * y00 - si * y10;
      x[1] = diag ? 0.0 : ci * y01 - si * y11;
      x[2] = diag ? 0.0 : ci * y10 + si * y00;
      x[3] = ci * y11 + si * y01;
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const double va = v[2 * r], vb = v[2 * r + 1];
        v[2 * r] = cj * va - sj * vb;
        v[2 * r + 1] = cj * vb + sj * va;
        const double wa = v[4 + 2 * r], wb = v[5 + 2 * r];
        v[4 + 2 * r] = ci * wa - si * wb;
        v[5 + 2 * r] = ci * wb + si * wa;
      }
      if (ok) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = e >> 1, c = e & 1;
          MA[(2 * i + r) * n + 2 * j + c] = x[e];
          MV[(2 * i + r) * n + 2 * j + c] = v[e];
          if (!diag) {
            MA[(2 * j + c) * n + 2 * i + r] = x[e];
            MV[(2 * j + r) * n + 2 * i + c] = v[4 + e];
          }
        }
      }
      wave_sync();
      x[0] = MA[si0 * n + sj0];
      x[1] = MA[si0 * n + sj1];
      x[2] = MA[si1 * n + sj0];
      x[3] = MA[si1 * n + sj1];
      dg[0] = MA[si0 * n + si0];
      dg[1] = MA[si0 * n + si1];
      dg[2] = MA[si1 * n + si1];
      dg[3] = MA[sj0 * n + sj0];
      dg[4] = MA[sj0 * n + sj1];
      dg[5] = MA[sj1 * n + sj1];
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        v[2 * r] = MV[(2 * i + r) * n + sj0];
        v[2 * r + 1] = MV[(2 * i + r) * n + sj1];
        v[4 + 2 * r] = MV[(2 * j + r) * n + si0];
        v[5 + 2 * r] = MV[(2 * j + r) * n + si1];
      }
      wave_sync();
    }
  }
  if (ok) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = e >> 1, c = e & 1;
      A[(2 * i + r) * n + 2 * j + c] = x[e];
      V[(2 * i + r) * n + 2 * j + c] = v[e];
      if (!diag) {
        A[(2 * j + c) * n + 2 * i + r] = x[e];
        V[(2 * j + r) * n + 2 * i + c] = v[4 + e];
      }
    }
  }
  wave_sync();
}

// ------------------------------------------------------- direction
// C = op(A) op(B) for k x k blocks (k <= KC) by one wave on FP64 matrix
// cores: 16x16 output tiles, 4 contraction steps per instruction; operands
// past k read as zero.  A(i, l) = A[i * lda + l] (or A[l * lda + i] when
// ta); likewise B.  C must not alias A or B.
template <int KC>
__device__ __forceinline__ void wave_mm_t(const double* A, int lda, bool ta, const double* B, int ldb, bool tb,
                                          double* C, int ldc, int k, int lane) {
  constexpr int T = (KC + 15) / 16;
  const int m16 = lane & 15, q = lane >> 4;
#pragma unroll
  for (int ti = 0; ti < T; ++ti)
#pragma unroll
    for (int tj = 0; tj < T; ++tj) {
      f64x4 acc = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kb = 0; kb < (KC + 3) / 4; ++kb) {
        const int i = 16 * ti + m16, l = 4 * kb + q, j = 16 * tj + m16;
        const int ic = i < k ? i : k - 1, lc = l < k ? l : k - 1, jc = j < k ? j : k - 1;
        const double av = ta ? A[lc * lda + ic] : A[ic * lda + lc];
        const double bv = tb ? B[jc * ldb + lc] : B[lc * ldb + jc];
        acc = mfma16x16x4((i < k && l < k) ? av : 0.0, (l < k && j < k) ? bv : 0.0, acc);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * ti + acc_row<double>(lane, r), col = 16 * tj + m16;
        if (row < k && col < k) C[row * ldc + col] = acc[r];
      }
    }
  wave_sync();
}

// wave_mm_t shared by the G waves of a group: wave g of the group computes
// the 16 x 16 output tiles t = g, g + G, ... (each tile as wave_mm_t
// computes it); the caller synchronises the workgroup before C is read.
template <int KC>
__device__ __forceinline__ void group_mm_t(const double* A, int lda, bool ta, const double* B, int ldb, bool tb,
                                           double* C, int ldc, int k, int lane, int g, int G) {
  constexpr int T = (KC + 15) / 16;
  const int m16 = lane & 15, q = lane >> 4;
  for (int t = g; t < T * T; t += G) {
    const int ti = t / T, tj = t - ti * T;
    f64x4 acc = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kb = 0; kb < (KC + 3) / 4; ++kb) {
      const int i = 16 * ti + m16, l = 4 * kb + q, j = 16 * tj + m16;
      const int ic = i < k ? i : k - 1, lc = l < k ? l : k - 1, jc = j < k ? j : k - 1;
      const double av = ta ? A[lc * lda + ic] : A[ic * lda + lc];
      const double bv = tb ? B[jc * ldb + lc] : B[lc * ldb + jc];
      acc = mfma16x16x4((i < k && l < k) ? av : 0.0, (l < k && j < k) ? bv : 0.0, acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * ti + acc_row<double>(lane, r), col = 16 * tj + m16;
      if (row < k && col < k) C[row * ldc + col] = acc[r];
    }
  }
}

// All threads first reduce the row-slice partials (P = BU^T M^-1 BU,
// Q = BU^T M^-1 E, BU^T xi, BU^T gold and three traces per side) into LDS;
// one wave per manifold block then diagonalises P (Jacobi, started from
// the previous iteration's eigenvectors, which nearly diagonalise the new
// P), solves the three Sylvester equations through it and reduces the
// trace terms; thread 0 forms the Polak-Ribiere+ coefficient, the descent
// test and the stopping test.
template <int KC>
__device__ __forceinline__ void ctrl_dir_body(const ProbView& p) {
  SolverCtrl* c = p.ctrl;
  if (c->done) return;
  extern __shared__ double sm[];
  __shared__ WaveJacobiScratch jsc[2];
  __shared__ double jpsum[16][2];
  __shared__ double terms[2][12];
  __shared__ double trv[2][3][KC];
  __shared__ double beta_sh;
  const int k = p.k, nb = p.nb, tid = threadIdx.x, lane = tid & 63, b = tid >> 6;
  const int n = (k + 1) & ~1;
  const int kk2 = k * k, nn = n * n;
  const int slices = 1;   // k_part_reduce left the slice sums in slice 0
  const int NR = 4 * k;
  const int64_t zs = (int64_t)(2 * k) * NR;
  const int64_t side_stride = (int64_t)p.part_slices * (4 * k) * (6 * k);   // as laid out by run_partials
  const int per_side = 9 * kk2 + 5 * nn;
  for (int e = tid; e < nb * 4 * kk2; e += 512) {
    const int sd = sdiv(e, 4 * kk2), r = e - sd * 4 * kk2, blk = sdiv(r, kk2), q = r - blk * kk2, i = sdiv(q, k), j = q - i * k;
    sm[(size_t)sd * per_side + r] =
        slice_sum(p.part + sd * side_stride, slices, zs, 1, (int64_t)i * NR + blk * k + j, 0, 0, 0, 1.0, 0.0, 0.0, 0.0);
  }
  for (int e = tid; e < nb * 3 * k; e += 512) {
    const int sd = sdiv(e, 3 * k), r = e - sd * 3 * k, which = sdiv(r, k), i = r - which * k;
    trv[sd][which][i] = slice_sum(p.part + sd * side_stride, slices, zs, 1, (int64_t)(k + i) * NR + (which + 1) * k + i,
                                  0, 0, 0, 1.0, 0.0, 0.0, 0.0);
  }
  __syncthreads();
  const bool warm = c->eig_ok && (c->iter % 32 != 0);
  double* P = sm + b * per_side;
  double* Q = P + kk2;
  double* cx = Q + kk2;
  double* cg = cx + kk2;
  double* S = cg + kk2;
  double* Sx = S + kk2;
  double* Sg = Sx + kk2;
  double* W1 = Sg + kk2;
  double* W2 = W1 + kk2;
  double* JA = W2 + kk2;
  double* JV = JA + nn;
  double* JT = JV + nn;   // 2 nn
  double* V0 = JT + 2 * nn;
  double tr3[3] = {0.0, 0.0, 0.0};
  if (b < nb) {
    for (int i = lane; i < k; i += 64) {
      tr3[0] += trv[b][0][i];
      tr3[1] += trv[b][1][i];
      tr3[2] += trv[b][2][i];
    }
    for (int q = 0; q < 3; ++q)
      for (int o = 32; o > 0; o >>= 1) tr3[q] += __shfl_xor(tr3[q], o, 64);
  }
  // The k x k algebra of a side runs on a group of four waves (side b / 4,
  // wave g = b % 4 of the group): products split by output tile, the three
  // Sylvester solves one per wave; each output is computed as a single
  // wave would compute it.
  constexpr int G = 4;
  const int sd = b / G, g = b - sd * G;
  const bool grp = sd < nb;
  const int gl = g * 64 + lane;          // lane within the group
  double* Pg = sm + (grp ? sd : 0) * per_side;
  double* JAg = Pg + 9 * kk2;
  double* JVg = JAg + nn;
  double* JTg = JVg + nn;
  double* V0g = JTg + 2 * nn;
  double* Vstg = kkslot(p, grp ? sd : 0, KK_EIG);
  if (grp) {
    for (int e = gl; e < nn; e += 64 * G) {
      const int i = sdiv(e, n), j = e - i * n;
      JAg[e] = (i < k && j < k) ? 0.5 * (Pg[i * k + j] + Pg[j * k + i]) : ((i == j) ? 1.0 : 0.0);
      if (warm) V0g[e] = Vstg[e];
    }
  }
  __syncthreads();
  if (warm) {
    if (grp) group_mm_t<KC>(JAg, n, false, V0g, n, false, JTg, n, n, lane, g, G);   // JA V0
    __syncthreads();
    if (grp) group_mm_t<KC>(V0g, n, true, JTg, n, false, JAg, n, n, lane, g, G);   // V0^T (JA V0)
    __syncthreads();
    if (grp)
      for (int e = gl; e < nn; e += 64 * G) {
        const int i = sdiv(e, n), j = e - i * n;
        JTg[e] = 0.5 * (JAg[i * n + j] + JAg[j * n + i]);
      }
    __syncthreads();
    if (grp)
      for (int e = gl; e < nn; e += 64 * G) JAg[e] = JTg[e];
    __syncthreads();
  }
  // Eigenvectors of P: one wave per block with the matrix in its registers
  // up to n = 20; beyond, the whole workgroup.
  if (n <= 20) {
    if (b < nb) pair_jacobi(JA, JV, JT, n, lane, p.eig_tol2);
  } else {
    double* Av[2];
    double* Vv[2];
    double* Tv[2];
    for (int s2 = 0; s2 < 2; ++s2) {
      double* base = sm + (s2 < nb ? s2 : 0) * per_side + 9 * kk2;
      Av[s2] = base;
      Vv[s2] = base + nn;
      Tv[s2] = base + 2 * nn;
    }
    block_jacobi(Av, Vv, Tv, jsc, jpsum, nb, n, p.eig_tol2);
  }
  __syncthreads();
  if (warm) {
    if (grp) group_mm_t<KC>(V0g, n, false, JVg, n, false, JTg, n, n, lane, g, G);   // V = V0 J
    __syncthreads();
    if (grp)
      for (int e = gl; e < nn; e += 64 * G) JVg[e] = JTg[e];
    __syncthreads();
  }
  if (grp && g < 3) {
    if (g == 0)
      for (int e = lane; e < nn; e += 64) Vstg[e] = JVg[e];
    // Sylvester: X = V ((V^T C V) ./ (w_i + w_j)) V^T for C = Z + Z^T, Z one
    // of Q, cx, cg; Y is this wave's scratch (W1, W2, or the free JT)
    double* Qg = Pg + kk2;
    const double* C = Qg + g * kk2;                 // Q, cx, cg
    double* X = Pg + (4 + g) * kk2;                 // S, Sx, Sg
    double* Y = g == 0 ? Pg + 7 * kk2 : (g == 1 ? Pg + 8 * kk2 : JTg);
    for (int e = lane; e < kk2; e += 64) {
      const int i = sdiv(e, k), j = e - i * k;
      Y[e] = C[i * k + j] + C[j * k + i];
    }
    wave_sync();
    wave_mm_t<KC>(Y, k, false, JVg, n, false, X, k, k, lane);   // (C + C^T) V
    wave_mm_t<KC>(JVg, n, true, X, k, false, Y, k, k, lane);    // V^T (C + C^T) V
    for (int e = lane; e < kk2; e += 64) {
      const int i = sdiv(e, k), j = e - i * k;
      Y[e] /= (JAg[i * n + i] + JAg[j * n + j]);
    }
    wave_sync();
    wave_mm_t<KC>(JVg, n, false, Y, k, false, X, k, k, lane);   // V (...)
    wave_mm_t<KC>(X, k, false, JVg, n, true, Y, k, k, lane);    // ... V^T
    // the solution is symmetric: keep it so (its two triangles are
    // rounded along different sums)
    for (int e = lane; e < kk2; e += 64) {
      const int i = sdiv(e, k), j = e - i * k;
      X[e] = 0.5 * (Y[i * k + j] + Y[j * k + i]);
    }
  }
  __syncthreads();
  if (b < nb) {
    wave_mm_t<KC>(P, k, false, S, k, false, W1, k, k, lane);   // W1 = P S
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int e = lane; e < kk2; e += 64) {
      v[0] += Q[e] * S[e];
      v[1] += S[e] * W1[e];
      v[2] += cg[e] * S[e];
      v[3] += Sg[e] * Q[e];
      v[4] += Sg[e] * W1[e];
      v[5] += cx[e] * S[e];
      v[6] += Sx[e] * Q[e];
      v[7] += Sx[e] * W1[e];
    }
    for (int q = 0; q < 8; ++q)
      for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_xor(v[q], o, 64);
    if (lane == 0) {
      for (int q = 0; q < 8; ++q) terms[b][q] = v[q];
      terms[b][8] = tr3[0];
      terms[b][9] = tr3[1];
      terms[b][10] = tr3[2];
    }
  }
  __syncthreads();
  if (tid == 0) {
    double gg = 0.0, gTg = 0.0, gTx = 0.0;
    for (int s2 = 0; s2 < nb; ++s2) {
      const double* t8 = terms[s2];
      gg += t8[8] - 2.0 * t8[0] + t8[1];
      gTg += t8[10] - t8[2] - t8[3] + t8[4];
      gTx += t8[9] - t8[5] - t8[6] + t8[7];
    }
    double beta = 0.0;
    if (!c->restart && c->iter > 0 && c->gg_old > 0.0) {
      beta = (gg - gTg) / c->gg_old;
      if (!(beta > 0.0)) beta = 0.0;
    }
    double df0 = -gg + beta * gTx;
    if (!(df0 < 0.0)) {
      beta = 0.0;
      df0 = -gg;
    }
    c->beta = beta;
    c->df0 = df0;
    c->gg = gg;
    c->gg_old = gg;
    c->restart = 0;
    c->eig_ok = 1;
    const double gnorm = sqrt(gg > 0.0 ? gg : 0.0);
    if (gnorm <= c->tol * fabs(c->f)) {
      c->done = 1;
      c->status = SRP_OK;
    } else if (c->iter >= c->max_iter) {
      c->done = 1;
      c->status = SRP_ENOCONV;
    }
    c->iter += 1;
    beta_sh = beta;
  }
  __syncthreads();
  if (b < nb) {
    const double beta = beta_sh;
    double* gS = kkslot(p, b, KK_S);
    double* gPhi = kkslot(p, b, KK_PHI);
    for (int e = lane; e < kk2; e += 64) {
      gS[e] = S[e];
      gPhi[e] = S[e] - beta * Sx[e];
    }
  }
}

template <int KC>
__global__ void __launch_bounds__(512) k_ctrl_dir(ProbView p) { ctrl_dir_body<KC>(p); }

template <int KC>
__global__ void __launch_bounds__(512) k_ctrl_dir_g(const ProbView* __restrict__ v, GroupSel sel) {
  ctrl_dir_body<KC>(v[sel.idx[blockIdx.x]]);
}

size_t ctrl_dir_lds(int k, int nb) {
  const int n = (k + 1) & ~1;
  const size_t per_side = (size_t)(9 * k * k + 5 * n * n);
  return (size_t)nb * per_side * sizeof(double);
}

int launch_ctrl_dir_g(const ProbView* v, const GroupSel& sel, size_t lds, int kc, hipStream_t st) {
  if (sel.n <= 0) return SRP_OK;
  if (kc == 16) {
    SRP_TRY(allow_dynamic_lds((const void*)k_ctrl_dir_g<16>, lds));
    hipLaunchKernelGGL(k_ctrl_dir_g<16>, dim3(sel.n), dim3(512), lds, st, v, sel);
  } else {
    SRP_TRY(allow_dynamic_lds((const void*)k_ctrl_dir_g<32>, lds));
    hipLaunchKernelGGL(k_ctrl_dir_g<32>, dim3(sel.n), dim3(512), lds, st, v, sel);
  }
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

template <int KC>
static int launch_ctrl_dir_t(const ProbView& p, hipStream_t st) {
  const size_t lds = ctrl_dir_lds(p.k, p.nb);
  SRP_TRY(allow_dynamic_lds((const void*)k_ctrl_dir<KC>, lds));
  hipLaunchKernelGGL(k_ctrl_dir<KC>, dim3(1), dim3(512), lds, st, p);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

int launch_ctrl_dir(const ProbView& p, hipStream_t st) {
  if (p.k <= 16) return launch_ctrl_dir_t<16>(p, st);
  return launch_ctrl_dir_t<32>(p, st);
}

// ------------------------------------------------------------ combine
// xi+ = -W_E + beta xi + W_B Phi ;  gold = W_E - W_B S   (element-wise).
template <int KC>
__device__ __forceinline__ void combine_body(const ProbView& p, int bx, int b) {
  const SolverCtrl* c = p.ctrl;
  if (c->done) return;
  const SideView& s = p.s[b];
  const int k = p.k;
  __shared__ double S[KMAX * KMAX], Phi[KMAX * KMAX];
  const double* gS = kkslot(p, b, KK_S);
  const double* gPhi = kkslot(p, b, KK_PHI);
  for (int e = threadIdx.x; e < k * k; e += 256) { S[e] = gS[e]; Phi[e] = gPhi[e]; }
  __syncthreads();
  const int64_t e = bx * 256ll + threadIdx.x;
  if (e >= (int64_t)s.d * k) return;
  const int i = sdiv((int)e, k), j = (int)e - i * k;
  const double* Wrow = s.Wz + (int64_t)i * 2 * k;   // [W_E | W_B]
  double wbphi = 0.0, wbs = 0.0;
#pragma unroll
  for (int l = 0; l < KC; ++l) {   // unconditional loads, masked terms
    const int lc = l < k ? l : 0;
    const double wb = Wrow[k + lc];
    const double a1 = wb * Phi[lc * k + j], a2 = wb * S[lc * k + j];
    wbphi += (l < k) ? a1 : 0.0;
    wbs += (l < k) ? a2 : 0.0;
  }
  const double we = Wrow[j];
  const double beta = c->beta;
  s.xi[e] = -we + beta * s.xi[e] + wbphi;
  s.gold[e] = we - wbs;
}

template <int KC>
__global__ void __launch_bounds__(256) k_combine(ProbView p) { combine_body<KC>(p, blockIdx.x, blockIdx.y); }

template <int KC>
__global__ void __launch_bounds__(256) k_combine_g(const ProbView* __restrict__ v, GroupSel sel) {
  const ProbView& p = v[sel.idx[blockIdx.z]];
  if ((int)blockIdx.y >= p.nb) return;
  combine_body<KC>(p, blockIdx.x, blockIdx.y);
}

int launch_combine_g(const ProbView* v, const GroupSel& sel, int64_t max_dk, int kc, hipStream_t st) {
  if (sel.n <= 0) return SRP_OK;
  dim3 grid((unsigned)((max_dk + 255) / 256), 2, sel.n);
  if (kc == 16) hipLaunchKernelGGL(k_combine_g<16>, grid, dim3(256), 0, st, v, sel);
  else hipLaunchKernelGGL(k_combine_g<32>, grid, dim3(256), 0, st, v, sel);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

int launch_combine(const ProbView& p, hipStream_t st) {
  const int dmax = p.nb == 2 ? (p.s[0].d > p.s[1].d ? p.s[0].d : p.s[1].d) : p.s[0].d;
  dim3 grid((unsigned)(((int64_t)dmax * p.k + 255) / 256), p.nb);
  if (p.k <= 16) hipLaunchKernelGGL(k_combine<16>, grid, dim3(256), 0, st, p);
  else hipLaunchKernelGGL(k_combine<32>, grid, dim3(256), 0, st, p);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

// -------------------------------------------------------------- final
// FP64 retraction onto the constraint and Rayleigh-Ritz rotation: with
// L_b L_b^T = U_b^T B_b U_b, CCA forms C = L_0^-1 (U_0^T Kc_0) L_1^-T and its
// SVD (Jacobi on [[0, C], [C^T, 0]]); FDA the eigen-decomposition of
// L^-1 (W^T S_B W) L^-T.  Rotations R_b = L_b^-T (singular/eigen vectors)
// are stored in the KK_ROT slots, sigma (descending) in sigma_out.
__global__ void __launch_bounds__(64) k_ctrl_final(ProbView p, double* sigma_out) {
  extern __shared__ double sm[];
  __shared__ WaveJacobiScratch jsc;
  __shared__ int order[64];
  const int k = p.k, nb = p.nb, lane = threadIdx.x;
  const int kk2 = k * k;
  const int slices = 1;   // k_part_reduce left the slice sums in slice 0
  const int64_t side_stride = (int64_t)p.part_slices * (4 * k) * (6 * k);
  double* G[2] = {sm, sm + 3 * kk2};
  double* Li[2] = {sm + kk2, sm + 4 * kk2};
  double* Cu[2] = {sm + 2 * kk2, sm + 5 * kk2};
  for (int b = 0; b < nb; ++b) {
    const double* part = p.part + b * side_stride;
    sum_block(part, slices, 1, 3, k, 0, 0, 1.0, G[b], lane, 64, false);
    sum_block(part, slices, 1, 3, k, 0, 1, p.s[b].lam, G[b], lane, 64, true);
    sum_block(part, slices, 1, 3, k, 0, 2, 1.0, Cu[b], lane, 64, false);
  }
  wave_sync();
  for (int b = 0; b < nb; ++b) {
    for (int e = lane; e < kk2; e += 64) {
      const int i = sdiv(e, k), j = e - i * k;
      if (i < j) {
        const double v = 0.5 * (G[b][i * k + j] + G[b][j * k + i]);
        G[b][i * k + j] = v;
        G[b][j * k + i] = v;
      }
    }
    wave_sync();
    if (!wave_chol(G[b], k, lane)) {
      if (lane == 0) { p.ctrl->status = SRP_ENOTSPD; p.ctrl->done = 1; }
      return;
    }
    wave_lower_inv(G[b], Li[b], k, lane);
  }
  // Cw = Li_0 Cu Li_1^T  (FDA: Li Cu Li^T)
  double* Cw = sm + 6 * kk2;
  double* Tm = Cw + kk2;
  const double* Lx = Li[0];
  const double* Ly = Li[nb == 2 ? 1 : 0];
  for (int e = lane; e < kk2; e += 64) {
    const int i = sdiv(e, k), j = e - i * k;
    double s = 0.0;
    for (int l = 0; l <= i; ++l) s += Lx[i * k + l] * Cu[0][l * k + j];
    Tm[e] = s;
  }
  wave_sync();
  for (int e = lane; e < kk2; e += 64) {
    const int i = sdiv(e, k), j = e - i * k;
    double s = 0.0;
    for (int l = 0; l <= j; ++l) s += Tm[i * k + l] * Ly[j * k + l];
    Cw[e] = s;
  }
  wave_sync();
  double* JA = Tm + kk2;
  if (!p.lda_cost) {
    // CCA: the singular pairs of Cw from the eigenpairs of Cw^T Cw (k x k,
    // even size, an odd k padded as in FDA below): v_j the eigenvectors,
    // sigma_j = sqrt(lambda_j), u_j = Cw v_j / sigma_j (so u_j^T Cw v_j =
    // sigma_j > 0).  When the smallest of the k is below 1e-6 of the
    // largest, u_j would lose accuracy: the augmented 2k x 2k problem below
    // is solved instead.
    const int mg = (k + 1) & ~1;
    double* GV = JA + mg * mg;
    double* GT = GV + mg * mg;
    double gf = 0.0;
    for (int e = lane; e < kk2; e += 64) {
      const int i = sdiv(e, k), j = e - i * k;
      double sg = 0.0;
      for (int l = 0; l < k; ++l) sg += Cw[l * k + i] * Cw[l * k + j];
      Tm[e] = sg;
      gf += sg * sg;
    }
    for (int o = 32; o > 0; o >>= 1) gf += __shfl_xor(gf, o, 64);
    wave_sync();
    const double gpad = -(1.0 + sqrt(gf));
    for (int e = lane; e < mg * mg; e += 64) {
      const int i = sdiv(e, mg), j = e - i * mg;
      JA[e] = (i < k && j < k) ? 0.5 * (Tm[i * k + j] + Tm[j * k + i]) : (i == j ? gpad : 0.0);
    }
    wave_sync();
    wave_jacobi(JA, GV, GT, mg, lane, jsc);
    if (lane < mg) {
      const double vi = JA[lane * mg + lane];
      int rank = 0;
      for (int j = 0; j < mg; ++j) {
        const double vj = JA[j * mg + j];
        rank += (vj > vi) || (vj == vi && j < lane);
      }
      order[rank] = lane;
    }
    wave_sync();
    const double l0 = JA[order[0] * mg + order[0]], lk = JA[order[k - 1] * mg + order[k - 1]];
    if (l0 > 0.0 && lk > 1e-12 * l0) {
      // Tm = Cw V_k diag(1 / sigma)
      for (int e = lane; e < kk2; e += 64) {
        const int i = sdiv(e, k), j = e - i * k;
        const int col = order[j];
        double sg = 0.0;
        for (int l = 0; l < k; ++l) sg += Cw[i * k + l] * GV[l * mg + col];
        Tm[e] = sg / sqrt(JA[col * mg + col]);
      }
      wave_sync();
      for (int b = 0; b < 2; ++b) {
        double* R = kkslot(p, b, KK_ROT);
        const double* Lb = Li[b];
        for (int e = lane; e < kk2; e += 64) {
          const int i = sdiv(e, k), j = e - i * k;
          double sg = 0.0;
          for (int l = i; l < k; ++l) sg += Lb[l * k + i] * (b == 0 ? Tm[l * k + j] : GV[l * mg + order[j]]);
          R[e] = sg;
        }
      }
      if (lane < k) sigma_out[lane] = sqrt(JA[order[lane] * mg + order[lane]]);
      if (lane == 0) {
        double f = 0.0;
        for (int i = 0; i < k; ++i) f += p.mu[i] * sqrt(JA[order[i] * mg + order[i]]);
        p.ctrl->f = -f;
      }
      return;
    }
    wave_sync();
  }
  const int m = p.lda_cost ? ((k + 1) & ~1) : 2 * k;  // even Jacobi size
  double* JV = JA + m * m;
  double* JT = JV + m * m;
  // FDA with odd k pads one decoupled row and column whose diagonal lies
  // below every eigenvalue (-(1 + ||Cw||_F)), so it sorts last; a finite
  // value of the matrix's own scale keeps the sweeps' convergence test (off
  // against the diagonal norm) meaningful.
  double fro = 0.0;
  for (int e = lane; e < kk2; e += 64) fro += Cw[e] * Cw[e];
  for (int o = 32; o > 0; o >>= 1) fro += __shfl_xor(fro, o, 64);
  const double pad = -(1.0 + sqrt(fro));
  for (int e = lane; e < m * m; e += 64) {
    const int i = sdiv(e, m), j = e - i * m;
    double v = 0.0;
    if (p.lda_cost) {
      if (i < k && j < k) v = 0.5 * (Cw[i * k + j] + Cw[j * k + i]);
      else v = (i == j) ? pad : 0.0;
    } else {
      if (i < k && j >= k) v = Cw[i * k + (j - k)];
      else if (i >= k && j < k) v = Cw[j * k + (i - k)];
    }
    JA[e] = v;
  }
  wave_sync();
  wave_jacobi(JA, JV, JT, m, lane, jsc);
  // order eigenvalues descending (rank of each by counting)
  if (lane < m) {
    const double vi = JA[lane * m + lane];
    int rank = 0;
    for (int j = 0; j < m; ++j) {
      const double vj = JA[j * m + j];
      rank += (vj > vi) || (vj == vi && j < lane);
    }
    order[rank] = lane;
  }
  wave_sync();
  // rotations: R_0 = Lx^T P_k, R_1 = Ly^T Q_k (CCA eigenvectors [a; b] scaled by sqrt 2)
  const double scl = p.lda_cost ? 1.0 : sqrt(2.0);
  for (int b = 0; b < nb; ++b) {
    double* R = kkslot(p, b, KK_ROT);
    const double* Lb = Li[b];
    const int off = (p.lda_cost || b == 0) ? 0 : k;
    for (int e = lane; e < kk2; e += 64) {
      const int i = sdiv(e, k), j = e - i * k;
      const int col = order[j];
      double s = 0.0;
      for (int l = i; l < k; ++l) s += Lb[l * k + i] * JV[(off + l) * m + col];
      R[e] = scl * s;
    }
  }
  if (lane < k) sigma_out[lane] = JA[order[lane] * m + order[lane]];
  if (lane == 0) {
    double f = 0.0;
    for (int i = 0; i < k; ++i) f += p.mu[i] * JA[order[i] * m + order[i]];
    p.ctrl->f = p.lda_cost ? -0.5 * f : -f;
  }
}

int launch_ctrl_final(const ProbView& p, double* sigma_out, hipStream_t st) {
  const int k = p.k;
  const int m = p.lda_cost ? ((k + 1) & ~1) : 2 * k;
  const size_t lds = (size_t)(8 * k * k + 4 * m * m) * sizeof(double);
  SRP_TRY(allow_dynamic_lds((const void*)k_ctrl_final, lds));
  hipLaunchKernelGGL(k_ctrl_final, dim3(1), dim3(64), lds, st, p, sigma_out);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

// U_b <- U_b R_b (rows in place).
template <int KC>
__global__ void __launch_bounds__(256) k_apply_rot(ProbView p) {
  const int b = blockIdx.y;
  const SideView& s = p.s[b];
  const int k = p.k;
  __shared__ double R[KC * KC];
  const double* gR = kkslot(p, b, KK_ROT);
  for (int e = threadIdx.x; e < k * k; e += 256) R[e] = gR[e];
  __syncthreads();
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= s.d) return;
  double* Ui = s.U + (int64_t)i * k;
  double v[KC];
#pragma unroll
  for (int j = 0; j < KC; ++j) v[j] = (j < k) ? Ui[j] : 0.0;
#pragma unroll
  for (int j = 0; j < KC; ++j)
    if (j < k) {
      double a = 0.0;
#pragma unroll
      for (int l = 0; l < KC; ++l)
        a += (l < k) ? v[l] * R[(l < k ? l : 0) * k + j] : 0.0;
      Ui[j] = a;
    }
}

int launch_apply_rot(const ProbView& p, hipStream_t st) {
  const int dmax = p.nb == 2 ? (p.s[0].d > p.s[1].d ? p.s[0].d : p.s[1].d) : p.s[0].d;
  dim3 grid((dmax + 255) / 256, p.nb);
  if (p.k <= 16) hipLaunchKernelGGL((k_apply_rot<16>), grid, dim3(256), 0, st, p);
  else hipLaunchKernelGGL((k_apply_rot<32>), grid, dim3(256), 0, st, p);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

// Sign convention: flip column j of every block so that the entry of
// largest magnitude in U_0[:, j] is positive (ties: lowest index).
__global__ void __launch_bounds__(256) k_sign_fix(ProbView p) {
  const int j = blockIdx.x, k = p.k;
  const SideView& s0 = p.s[0];
  __shared__ double bv[256];
  __shared__ int bi[256];
  double best = -1.0;
  int idx = 0x7fffffff;
  for (int i = threadIdx.x; i < s0.d; i += 256) {
    const double v = fabs(s0.U[(int64_t)i * k + j]);
    if (v > best) { best = v; idx = i; }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = idx;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      const double a = bv[threadIdx.x + off];
      const int ai = bi[threadIdx.x + off];
      if (a > bv[threadIdx.x] || (a == bv[threadIdx.x] && ai < bi[threadIdx.x])) {
        bv[threadIdx.x] = a;
        bi[threadIdx.x] = ai;
      }
    }
    __syncthreads();
  }
  // One thread reads the winning entry's sign; every thread waits for it
  // before any write to the column (the thread that owns that row negates it).
  __shared__ int flip_sh;
  if (threadIdx.x == 0) flip_sh = s0.U[(int64_t)bi[0] * k + j] < 0.0;
  __syncthreads();
  if (!flip_sh) return;
  for (int b = 0; b < p.nb; ++b) {
    const SideView& s = p.s[b];
    for (int i = threadIdx.x; i < s.d; i += 256) s.U[(int64_t)i * k + j] = -s.U[(int64_t)i * k + j];
  }
}

int launch_sign_fix(const ProbView& p, hipStream_t st) {
  hipLaunchKernelGGL(k_sign_fix, dim3(p.k), dim3(256), 0, st, p);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

// ------------------------------------------------ exact sketched solves
// Small dense steps of the warm start (the exact CCA / FDA solution of the
// sketched problem, Algorithms CCAopt and LDAopt): the Cholesky-QR factor of
// a block Gram and the Rayleigh-Ritz eigensolve of a q x q block.

// B = L^-T for L L^T = G + delta I (G q x q symmetric, only its lower
// triangle read; q <= Q <= 64; delta = 1e-14 tr(G) / q keeps a numerically
// singular block factorable, and the next iteration re-orthonormalises
// anyway), written as a Q x Q row-major matrix (ld Q) whose rows and
// columns past q are those of the identity.  W B then has orthonormal
// columns in the inner product G was taken in.  *flag = 1 when the factor
// breaks down (non-finite or non-positive pivot).  One wave, registers:
// for the factor lane i keeps row i of the trailing matrix (the shift is
// added to each pivot as it is used) and the pivot column goes through
// LDS; for the inverse lane c builds column c of L^-1 by forward
// substitution against L in LDS (uniform addresses: every read is a
// broadcast).  The scheduling barrier per step keeps the compiler from
// hoisting later steps' LDS reads, and the stores are unconditional: both
// keep the wave within its registers.
template <int Q>
__global__ void __launch_bounds__(64) k_cholqr_factor(const double* __restrict__ G, int q, double* __restrict__ B,
                                                      int* __restrict__ flag) {
  __shared__ double Lm[Q * Q];
  __shared__ double col[64];
  const int i = threadIdx.x;
  double tr = (i < q) ? G[i * q + i] : 0.0;
  for (int o = 32; o > 0; o >>= 1) tr += __shfl_xor(tr, o, 64);
  const double delta = 1e-14 * tr / q;
  bool ok = true;
  {
    double a[Q];
#pragma unroll
    for (int c = 0; c < Q; ++c) a[c] = (i < q && c < q) ? G[i * q + c] : (c == i ? 1.0 : 0.0);
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const double piv = __shfl(a[j], j, 64) + (j < q ? delta : 0.0);
      ok = ok && piv > 0.0;
      const double inv = 1.0 / sqrt(piv);
      const double lij = (i == j) ? piv * inv : a[j] * inv;   // L[i][j] for i >= j
      a[j] = lij;
      col[i] = lij;
      wave_sync();
#pragma unroll
      for (int c = j + 1; c < Q; ++c) a[c] -= lij * col[c];
      wave_sync();
      __builtin_amdgcn_sched_barrier(0);
    }
    if (i < Q) {
#pragma unroll
      for (int c = 0; c < Q; ++c) Lm[i * Q + c] = (c <= i) ? a[c] : 0.0;
    }
  }
  wave_sync();
  if (i < Q) {
    // column i of L^-1: x[r] = (delta_ri - sum_{l < r} L[r][l] x[l]) / L[r][r]
    double x[Q];
#pragma unroll
    for (int r = 0; r < Q; ++r) {
      double sacc = (r == i) ? 1.0 : 0.0;
#pragma unroll
      for (int l = 0; l < r; ++l) sacc -= Lm[r * Q + l] * x[l];
      x[r] = sacc / Lm[r * Q + r];
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int r = 0; r < Q; ++r) B[i * Q + r] = x[r];    // B = L^-T: B[i][r] = (L^-1)[r][i]
  }
  if (i == 0 && !ok) *flag = 1;
}

int cholqr_block(int q) { return q <= 16 ? 16 : (q <= 32 ? 32 : 64); }

int launch_cholqr_factor(const double* G, int q, double* B, int* flag, hipStream_t st) {
  if (q < 1 || q > 64) {
    set_error("cholqr: block of %d columns (1 to 64)", q);
    return SRP_EINVAL;
  }
  switch (cholqr_block(q)) {
    case 16: hipLaunchKernelGGL((k_cholqr_factor<16>), dim3(1), dim3(64), 0, st, G, q, B, flag); break;
    case 32: hipLaunchKernelGGL((k_cholqr_factor<32>), dim3(1), dim3(64), 0, st, G, q, B, flag); break;
    default: hipLaunchKernelGGL((k_cholqr_factor<64>), dim3(1), dim3(64), 0, st, G, q, B, flag); break;
  }
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

// Rayleigh-Ritz: eigenvectors of the symmetric q x q G (q <= 64), ordered by
// eigenvalue, descending; the first k go to Q (q x k, row-major) and their
// eigenvalues to ev.  An odd q is padded with one decoupled row and column
// whose diagonal -(1 + ||G||_F) lies below every eigenvalue.  One
// workgroup, cyclic Jacobi in parallel rounds (the round-robin pairing of
// the controllers' eigensolver): per round the pair threads compute the
// rotations into LDS tables, then every thread rotates whole 2 x 2 blocks
// (a row pair against a column pair) in place, and rows of V against
// column pairs; two barriers per round, no scratch copy.  Sweeps stop at
// off-diagonal norm <= 1e-13 of the diagonal norm.
__global__ void __launch_bounds__(256) k_rr_eig(const double* __restrict__ G, int q, int k, double* __restrict__ Q,
                                                double* __restrict__ ev) {
  __shared__ double A[64 * 64];
  __shared__ double V[64 * 64];
  __shared__ double rc[32], rs[32];
  __shared__ int rp[32], rq[32];
  __shared__ double red[4][2];
  __shared__ int order[64];
  const int n = (q + 1) & ~1, P = n / 2, n1 = n - 1, tid = threadIdx.x;
  double fro = 0.0;
  for (int e = tid; e < q * q; e += 256) fro += G[e] * G[e];
  for (int o = 32; o > 0; o >>= 1) fro += __shfl_xor(fro, o, 64);
  if ((tid & 63) == 0) red[tid >> 6][0] = fro;
  __syncthreads();
  const double pad = -(1.0 + sqrt(red[0][0] + red[1][0] + red[2][0] + red[3][0]));
  for (int e = tid; e < n * n; e += 256) {
    const int i = e / n, j = e - i * n;
    A[i * 64 + j] = (i < q && j < q) ? 0.5 * (G[i * q + j] + G[j * q + i]) : (i == j ? pad : 0.0);
    V[i * 64 + j] = (i == j) ? 1.0 : 0.0;
  }
  for (int sweep = 0; sweep < 40; ++sweep) {
    __syncthreads();
    double off = 0.0, dia = 0.0;
    for (int e = tid; e < n * n; e += 256) {
      const int i = e / n, j = e - i * n;
      const double x = A[i * 64 + j];
      if (i == j) dia += x * x; else off += x * x;
    }
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_xor(off, o, 64);
      dia += __shfl_xor(dia, o, 64);
    }
    if ((tid & 63) == 0) { red[tid >> 6][0] = off; red[tid >> 6][1] = dia; }
    __syncthreads();
    const double so = red[0][0] + red[1][0] + red[2][0] + red[3][0];
    const double sd = red[0][1] + red[1][1] + red[2][1] + red[3][1];
    if (so <= 1e-26 * (sd + 1e-300)) break;   // uniform
    for (int round = 0; round < n1; ++round) {
      if (tid < P) {
        int pp = jac_index(tid, round, n1), qq = jac_index(n1 - tid, round, n1);
        if (pp > qq) { const int t = pp; pp = qq; qq = t; }
        const double apq = A[pp * 64 + qq];
        double cth = 1.0, sth = 0.0;
        if (apq != 0.0) cth = jac_rotation((A[qq * 64 + qq] - A[pp * 64 + pp]) / (2.0 * apq), &sth);
        rc[tid] = cth; rs[tid] = sth; rp[tid] = pp; rq[tid] = qq;
      }
      __syncthreads();
      // A <- J^T A J: new row p = c row_p - s row_q, new row q = s row_p + c row_q (likewise columns)
      for (int e = tid; e < P * P; e += 256) {
        const int m1 = e / P, m2 = e - m1 * P;
        const int p1 = rp[m1], q1 = rq[m1], p2 = rp[m2], q2 = rq[m2];
        const double c1 = rc[m1], s1 = rs[m1], c2 = rc[m2], s2 = rs[m2];
        const double b00 = A[p1 * 64 + p2], b01 = A[p1 * 64 + q2], b10 = A[q1 * 64 + p2], b11 = A[q1 * 64 + q2];
        const double t00 = c1 * b00 - s1 * b10, t01 = c1 * b01 - s1 * b11;
        const double t10 = s1 * b00 + c1 * b10, t11 = s1 * b01 + c1 * b11;
        double n01 = s2 * t00 + c2 * t01, n10 = c2 * t10 - s2 * t11;
        if (m1 == m2) { n01 = 0.0; n10 = 0.0; }   // the rotated pair's coupling
        A[p1 * 64 + p2] = c2 * t00 - s2 * t01;
        A[p1 * 64 + q2] = n01;
        A[q1 * 64 + p2] = n10;
        A[q1 * 64 + q2] = s2 * t10 + c2 * t11;
      }
      // V <- V J
      for (int e = tid; e < n * P; e += 256) {
        const int r = e / P, m = e - r * P;
        const int pp = rp[m], qq = rq[m];
        const double cm = rc[m], sm = rs[m];
        const double vp = V[r * 64 + pp], vq = V[r * 64 + qq];
        V[r * 64 + pp] = cm * vp - sm * vq;
        V[r * 64 + qq] = sm * vp + cm * vq;
      }
      __syncthreads();
    }
  }
  __syncthreads();
  if (tid < n) {
    const double vi = A[tid * 64 + tid];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double vj = A[j * 64 + j];
      rank += (vj > vi) || (vj == vi && j < tid);
    }
    order[rank] = tid;
  }
  __syncthreads();
  for (int e = tid; e < q * k; e += 256) {
    const int i = e / k, j = e - i * k;
    Q[e] = V[i * 64 + order[j]];
  }
  if (tid < k) ev[tid] = A[order[tid] * 64 + order[tid]];
}

int launch_rr_eig(const double* G, int q, int k, double* Q, double* ev, hipStream_t st) {
  if (q < 1 || q > 64 || k < 1 || k > q) {
    set_error("rayleigh-ritz: block of %d columns, %d wanted (1 <= k <= q <= 64)", q, k);
    return SRP_EINVAL;
  }
  hipLaunchKernelGGL(k_rr_eig, dim3(1), dim3(256), 0, st, G, q, k, Q, ev);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

// ---------------------------------------------------------- misc
// Standard normal draws: Box-Muller on two SplitMix64 outputs per entry.
__global__ void k_gauss_fill(double* p, int64_t count, uint64_t seed) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= count) return;
  const uint64_t w1 = splitmix64(seed, 2 * (uint64_t)i), w2 = splitmix64(seed, 2 * (uint64_t)i + 1);
  const double u1 = ((double)(w1 >> 11) + 1.0) * 0x1.0p-53;  // (0, 1]
  const double u2 = (double)(w2 >> 11) * 0x1.0p-53;          // [0, 1)
  p[i] = sqrt(-2.0 * log(u1)) * cospi(2.0 * u2);
}

int launch_gauss_fill(double* p, int64_t count, uint64_t seed, hipStream_t st) {
  hipLaunchKernelGGL(k_gauss_fill, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, p, count, seed);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

__global__ void k_ctrl_init(SolverCtrl* c, double tol, int max_iter) {
  c->t = 0.0; c->t_guess = 0.0; c->f = 0.0; c->gg = 0.0; c->gg_old = 0.0; c->df0 = 0.0;
  c->beta = 0.0; c->tol = tol; c->done = 0; c->status = SRP_OK; c->iter = 0; c->max_iter = max_iter;
  c->restart = 1; c->ls_fail = 0; c->fixed_step = 1; c->eig_ok = 0;
}

int launch_ctrl_init(SolverCtrl* c, double tol, int max_iter, hipStream_t st) {
  hipLaunchKernelGGL(k_ctrl_init, dim3(1), dim3(1), 0, st, c, tol, max_iter);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

__global__ void k_set_fixed(SolverCtrl* c, int on) {
  c->fixed_step = on;
  c->done = 0;
  c->status = SRP_OK;
  c->restart = 1;
}

int launch_set_fixed_step(SolverCtrl* c, int on, hipStream_t st) {
  hipLaunchKernelGGL(k_set_fixed, dim3(1), dim3(1), 0, st, c, on);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

}  // namespace srp
