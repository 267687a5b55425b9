// Fused tall-skinny data pass: for data blocks A_0 (n x d0), A_1 (n x d1)
// and directions W_0, W_1 (d_b x k) compute, in one read of the data,
//     J_b = A_b^T [A_0 W_0 | A_1 W_1]        (d_b x NB k).
// These are the products with the data matrices that every Riemannian
// component of Table 1 needs (X^T X U, X^T Y V, ...; costs in Table costs:
// O(n d p) per product).
//
// Work split: a workgroup of 8 waves streams 16-row blocks of [A_0 | A_1].
// Each row block is handled by a PAIR of workgroups (block indices 8 apart,
// so both run on the same XCD and the second read of the block is served
// by that XCD's L2): both form the full P from their LDS copy, and each
// accumulates A_b^T [P_0 | P_1] for half of the columns, which halves the
// accumulator registers a wave must keep.
// The block is staged in LDS (row-major, row pitch = 4 mod 64 elements so
// both access patterns below are bank-conflict free); while the matrix
// cores work on block i, the global loads of the workgroup's next block are
// already in flight into registers.  The direction operands of a wave's
// P tiles stay in registers for the whole launch when they fit (64 per
// lane); otherwise they are re-read from L2 per block, before the next
// block's loads are issued, so that a wait on them never waits on HBM.  Columns are cut into 16-wide tiles;
// wave w owns tiles w, w+8, ...  For each block a wave
//   (b) accumulates its tiles' share of P_b = A_b W_b (16 x k) on the matrix
//       cores (A-operand lane: row = lane%16, column = 4 step + lane/16),
//   (c) the 8 partial P's are summed through LDS,
//   (d) accumulates its tiles' rows of A_b^T [P_0 | P_1] (A-operand lane:
//       column = lane%16, row = 4 (lane/16) + step).
// Each workgroup keeps its accumulators in registers over all its row
// blocks and writes one partial; a second kernel sums the partials in a
// fixed order (deterministic, no atomics).
#include "common.hpp"
#include "kernels.hpp"

namespace srp {

constexpr int kPassWaves = 8;
constexpr int kPassThreads = 64 * kPassWaves;
constexpr int kPassLds = 150 * 1024;   // LDS budget of the row-block stage

// Largest d0 + d1 per compute type, and loads per row per thread.
template <class CT> struct PassCfg;
// jpf of the jpr 512-column chunks of a row block are prefetched into
// registers during the previous block's math; the rest load on demand.
template <> struct PassCfg<float> { static constexpr int dmax = 2048; static constexpr int jpr = 4; static constexpr int jpf = 4; };
template <> struct PassCfg<double> { static constexpr int dmax = 896; static constexpr int jpr = 2; static constexpr int jpf = 2; };

__host__ __device__ constexpr int pass_pitch(int D) { return ((D + 63) / 64) * 64 + 4; }

// Pack double d_b x k directions into zero-padded (ceil16(d_b) x kpad) CT
// matrices, both blocks in one launch (block 1 follows block 0's elements).
template <class CT>
__global__ void k_pack_dir(const double* __restrict__ W0, int d0, int dpad0, CT* __restrict__ Wp0,
                           const double* __restrict__ W1, int d1, int dpad1, CT* __restrict__ Wp1, int k, int kpad) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t n0 = (int64_t)dpad0 * kpad;
  const double* W = W0;
  CT* Wp = Wp0;
  int d = d0;
  if (i >= n0) {
    i -= n0;
    if (i >= (int64_t)dpad1 * kpad) return;
    W = W1;
    Wp = Wp1;
    d = d1;
  }
  const int r = (int)(i / kpad), c = (int)(i - (int64_t)r * kpad);
  Wp[i] = (r < d && c < k) ? (CT)W[(int64_t)r * k + c] : CT(0);
}

template <class CT>
static int pack_dirs(const double* W0, int d0, int dp0, CT* Wp0, const double* W1, int d1, int dp1, CT* Wp1, int k,
                     int KP, hipStream_t st) {
  const int64_t tot = (int64_t)dp0 * KP + (Wp1 ? (int64_t)dp1 * KP : 0);
  hipLaunchKernelGGL((k_pack_dir<CT>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, W0, d0, dp0, Wp0, W1,
                     d1, Wp1 ? dp1 : 0, Wp1, k, KP);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

template <class CT, class DT> __device__ __forceinline__ CT cvt(DT v);
template <> __device__ __forceinline__ float cvt<float, float>(float v) { return v; }
template <> __device__ __forceinline__ float cvt<float, bf16>(bf16 v) { return __bfloat162float(v); }
template <> __device__ __forceinline__ double cvt<double, double>(double v) { return v; }
template <> __device__ __forceinline__ double cvt<double, float>(float v) { return (double)v; }
template <> __device__ __forceinline__ double cvt<double, bf16>(bf16 v) { return (double)__bfloat162float(v); }


constexpr int kPassSplit = 2;   // column halves per row block
constexpr int kXcds = 8;

template <class DT, class CT, int NB, int KT>
__global__ void __launch_bounds__(kPassThreads) k_pass(const DT* __restrict__ A0, const DT* __restrict__ A1,
                                                       int64_t n, int d0, int d1, int k,
                                                       const CT* __restrict__ Wp0, const CT* __restrict__ Wp1,
                                                       int nrb, CT* __restrict__ partial,
                                                       const int* __restrict__ done) {
  if (done && *done) return;
  constexpr int DMAX = PassCfg<CT>::dmax;
  constexpr int JPR = PassCfg<CT>::jpr;
  constexpr int JPF = PassCfg<CT>::jpf;
  constexpr int TPW = (DMAX / 16 + kPassWaves * kPassSplit - 1) / (kPassWaves * kPassSplit);
  constexpr int NT = NB * KT;
  constexpr int KP = KT * 16;
  constexpr int TPB = (DMAX / 16 + kPassWaves - 1) / kPassWaves;        // P tiles per wave
  constexpr bool WREG = TPB * 4 * KT * (int)sizeof(CT) <= 64 * 4;       // W operands in registers
  using acc_t = typename Acc4<CT>::type;
  extern __shared__ unsigned char pass_smem[];
  const int D = d0 + (NB == 2 ? d1 : 0);
  const int pitch = pass_pitch(D);
  CT* xs = reinterpret_cast<CT*>(pass_smem);                 // [16][pitch]
  CT* red = xs + 16 * pitch;                                  // [waves][NT][256]
  CT* pfull = red + kPassWaves * NT * 256;                    // [NT][16][17]

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, l16 = lane & 15;
  const int T0 = (d0 + 15) >> 4;
  const int TT = T0 + (NB == 2 ? ((d1 + 15) >> 4) : 0);
  // pair mapping: XCD x, half h, group q  ->  row group rg
  const int bx = blockIdx.x;
  const int xcd = bx % kXcds, half = (bx / kXcds) % kPassSplit, grp = bx / (kXcds * kPassSplit);
  const int rg = grp * kXcds + xcd;
  const int ngroups = gridDim.x / kPassSplit;
  const int TH = (TT + kPassSplit - 1) / kPassSplit;     // tiles per half
  const int tbeg = half * TH, tend = min(TT, tbeg + TH);
  const __amdgpu_buffer_rsrc_t wr0 = make_rsrc(Wp0, (int64_t)((d0 + 15) / 16 * 16) * KP * sizeof(CT));
  const __amdgpu_buffer_rsrc_t wr1 =
      make_rsrc(NB == 2 ? Wp1 : Wp0, (int64_t)((((NB == 2 ? d1 : d0) + 15) / 16) * 16) * KP * sizeof(CT));
  const int wvoff = (g * KP + l16) * (int)sizeof(CT);

  acc_t acc[TPW][NT];
#pragma unroll
  for (int i = 0; i < TPW; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

  // direction operands of this wave's P tiles: tile t = w + 8 i, step s2
  CT wreg[WREG ? TPB : 1][4][KT];
  auto w_operand = [&](int t, int s2, int kt) __attribute__((always_inline)) -> CT {
    const bool b1 = (NB == 2) && (t >= T0);
    const int ct = b1 ? t - T0 : t;
    const int soff = ((ct * 16 + 4 * s2) * KP + kt * 16) * (int)sizeof(CT);
    return b1 ? buf_load<CT>(wr1, wvoff + soff, 0) : buf_load<CT>(wr0, wvoff + soff, 0);
  };
  if (WREG) {
#pragma unroll
    for (int i = 0; i < (WREG ? TPB : 1); ++i)
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2)
#pragma unroll
        for (int kt = 0; kt < KT; ++kt) {
          const int t = w + kPassWaves * i;
          wreg[i][s2][kt] = (t < TT) ? w_operand(t, s2, kt) : CT(0);
        }
  }

  // Row r of the block gets its own buffer resource (scalar), holding
  // exactly the d_b elements of that row, or none past row n; a lane reads
  // column c of [A_0 | A_1] with one lane offset for all rows, and every
  // out-of-row, out-of-block or out-of-matrix element reads as zero.
  auto row_rsrc = [&](const DT* A, int db, int64_t row) __attribute__((always_inline)) {
    return make_rsrc(A + row * db, row < n ? (int64_t)db * (int64_t)sizeof(DT) : 0);
  };
  auto load_elem = [&](int64_t row, int j) __attribute__((always_inline)) -> DT {
    const int cb = kPassThreads * j;        // uniform chunk start
    const int c = cb + tid;
    const int v0 = c * (int)sizeof(DT);
    if (NB == 1 || cb + kPassThreads <= d0) return buf_load<DT>(row_rsrc(A0, d0, row), v0, 0);
    const int v1 = (c - d0) * (int)sizeof(DT);   // negative = out of range
    if (cb >= d0) return buf_load<DT>(row_rsrc(A1, d1, row), v1, 0);
    const DT x0 = buf_load<DT>(row_rsrc(A0, d0, row), v0, 0);
    const DT x1 = buf_load<DT>(row_rsrc(A1, d1, row), v1, 0);
    return (c < d0) ? x0 : x1;
  };
  DT pf[16][JPF];
  auto prefetch = [&](int rbk) __attribute__((always_inline)) {
    const int64_t r0 = (int64_t)rbk * 16;
#pragma unroll
    for (int j = 0; j < JPF; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) pf[r][j] = load_elem(r0 + r, j);
  };

  int rb = rg;
  if (rb < nrb) prefetch(rb);
  for (; rb < nrb; rb += ngroups) {
    __syncthreads();   // previous block fully consumed
#pragma unroll
    for (int j = 0; j < JPF; ++j) {
      const int c = tid + kPassThreads * j;
#pragma unroll
      for (int r = 0; r < 16; ++r)
        if (c < pitch) xs[r * pitch + c] = (c < D) ? cvt<CT>(pf[r][j]) : CT(0);
    }
    if (JPF < JPR) {
#pragma unroll
      for (int j = JPF; j < JPR; ++j) {
        const int c = tid + kPassThreads * j;
        if (kPassThreads * j < pitch) {
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const DT v = load_elem((int64_t)rb * 16 + r, j);
            if (c < pitch) xs[r * pitch + c] = (c < D) ? cvt<CT>(v) : CT(0);
          }
        }
      }
    }
    __syncthreads();
    if (WREG && rb + ngroups < nrb) prefetch(rb + ngroups);   // in flight during the math
    // (b) P_b partials
    acc_t pacc[NB][KT];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int kt = 0; kt < KT; ++kt) pacc[b][kt] = acc_t{0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < TPB; ++i) {
      const int t = w + kPassWaves * i;
      if (t < TT) {
        const bool b1 = (NB == 2) && (t >= T0);
        const int ct = b1 ? t - T0 : t;
        const int cbase = (b1 ? d0 : 0) + ct * 16;   // column of the tile in xs
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) {
          const CT a = xs[l16 * pitch + cbase + 4 * s2 + g];
#pragma unroll
          for (int kt = 0; kt < KT; ++kt) {
            const CT bw = WREG ? wreg[WREG ? i : 0][s2][kt] : w_operand(t, s2, kt);
            if (b1) pacc[NB - 1][kt] = mfma16x16x4(a, bw, pacc[NB - 1][kt]);
            else pacc[0][kt] = mfma16x16x4(a, bw, pacc[0][kt]);
          }
        }
      }
    }
    if (!WREG && rb + ngroups < nrb) prefetch(rb + ngroups);   // in flight during (c), (d)
    // (c) reduce P over waves
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int kt = 0; kt < KT; ++kt)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          red[(w * NT + b * KT + kt) * 256 + acc_row<CT>(lane, r) * 16 + l16] = pacc[b][kt][r];
    __syncthreads();
    for (int e = tid; e < NT * 256; e += kPassThreads) {
      const int nt = e >> 8, q = e & 255;
      CT v = CT(0);
#pragma unroll
      for (int ww = 0; ww < kPassWaves; ++ww) v += red[(ww * NT + nt) * 256 + q];
      pfull[nt * 272 + (q >> 4) * 17 + (q & 15)] = v;
    }
    __syncthreads();
    // (d) A_b^T [P_0 | P_1] for this workgroup's half of the tiles
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int t = tbeg + w + kPassWaves * i;
      if (t < tend) {
        const bool b1 = (NB == 2) && (t >= T0);
        const int cbase = (b1 ? d0 + (t - T0) * 16 : t * 16) + l16;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const CT a = xs[(4 * g + s) * pitch + cbase];
#pragma unroll
          for (int nt = 0; nt < NT; ++nt)
            acc[i][nt] = mfma16x16x4(a, pfull[nt * 272 + (4 * g + s) * 17 + l16], acc[i][nt]);
        }
      }
    }
  }
  // epilogue: this workgroup's partial (rows = concatenated columns of A)
  const int W_out = NB * k;
  CT* out = partial + (int64_t)rg * D * W_out;
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    const int t = tbeg + w + kPassWaves * i;
    if (t < tend) {
      const bool b1 = (NB == 2) && (t >= T0);
      const int db = b1 ? d1 : d0;
      const int ct = b1 ? t - T0 : t;
      const int rowbase = b1 ? d0 : 0;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int bsrc = nt / KT, kt = nt % KT;
        const int col = kt * 16 + l16;
        if (col < k) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int c = ct * 16 + acc_row<CT>(lane, r);
            if (c < db) out[(int64_t)(rowbase + c) * W_out + bsrc * k + col] = acc[i][nt][r];
          }
        }
      }
    }
  }
}

// ------------------------------------------------------------------
// FP32 data and arithmetic: the same products with the row blocks moved
// straight from HBM into LDS by the load unit (buffer loads with the LDS
// flag, no VGPRs), double-buffered, so a workgroup can own whole rows:
//   * 8-row blocks; block i+1 streams into the second LDS buffer while the
//     matrix cores work on block i, and the only wait on it is at the top
//     of the next iteration;
//   * the barriers inside an iteration wait on LDS traffic only (an LDS
//     fence would also wait on the in-flight block);
//   * the direction operands of a wave's tiles stay in registers for the
//     launch, and each wave accumulates A_b^T [P_0 | P_1] for the same
//     tiles it used for P (no column split, no duplicated P).
// Tile t of [A_0 | A_1] (16 columns; A_1's tiles follow A_0's) sits at LDS
// column 16 t, so every operand address is one base register plus a
// compile-time offset.  A load instruction moves CH = 64 VEC consecutive
// floats of one row; the last chunk of each block is shifted back to end
// on the block's last tile (it rewrites identical values), so no chunk
// spills into the other block's columns.  The row pitch is 4 mod 32 floats
// (bank-conflict free for both operand patterns).  The 16 MFMA rows of the
// P products hold the block's 8 rows twice: rows 0-7 accumulate A_0 W_0 and
// rows 8-15 A_1 W_1 (each lane zeroes the operand of the other view), so
// one accumulator serves both views and the tile loop has no view branch.
constexpr int kDmaRows = 8;
constexpr int kDmaWaves = 8;
constexpr int kDmaThreads = 64 * kDmaWaves;
constexpr int kDmaMaxTiles = 128;   // 2048 columns of [A_0 | A_1]
// The FP32 pass runs 16 waves (4 per SIMD, 128 registers each): a wave
// holds the direction operands and the J accumulators of at most 8 tiles.
constexpr int kF32Waves = 16;
constexpr int kF32Threads = 64 * kF32Waves;

__device__ __forceinline__ void lds_only_barrier() {
  // LDS traffic of this wave done, then the workgroup barrier; in-flight
  // global-to-LDS loads of the next block are deliberately not waited on.
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

template <int VEC>
__device__ __forceinline__ void dma_row_chunk(__amdgpu_buffer_rsrc_t r, float* lds_dst, int voff) {
  if constexpr (VEC == 4)
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (__attribute__((address_space(3))) void*)lds_dst, 16, voff, 0, 0, 0);
  else
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (__attribute__((address_space(3))) void*)lds_dst, 4, voff, 0, 0, 0);
}

__host__ __device__ constexpr int dma_pitch(int TT) { return ((TT * 16 + 31) / 32) * 32 + 4; }

template <int NB, int TPB, int VEC>
__global__ void __launch_bounds__(kF32Threads) k_pass_dma(const float* __restrict__ A0, const float* __restrict__ A1,
                                                          int64_t n, int d0, int d1, int k,
                                                          const float* __restrict__ Wp0,
                                                          const float* __restrict__ Wp1, int nrb,
                                                          float* __restrict__ partial, const int* __restrict__ done) {
  if (done && *done) return;
  constexpr int R = kDmaRows;
  constexpr int CH = 64 * VEC;
  constexpr int NT = NB;                                        // [P_0 | P_1] tiles of the J phase
  using acc_t = f32x4;
  extern __shared__ float dsm[];
  const int T0 = (d0 + 15) >> 4;
  const int T1 = NB == 2 ? ((d1 + 15) >> 4) : 0;
  const int TT = T0 + T1;
  const int nch0 = (T0 * 16 + CH - 1) / CH, nch1 = NB == 2 ? (T1 * 16 + CH - 1) / CH : 0;
  const int nch = nch0 + nch1;
  const int pitch = dma_pitch(kF32Waves * TPB);
  float* red = dsm + 2 * R * pitch;              // [waves][16 x 16]
  float* pfull = red + kF32Waves * 256;          // [NB][R][17]

  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, l16 = lane & 15;
  const __amdgpu_buffer_rsrc_t wr0 = make_rsrc(Wp0, (int64_t)T0 * 16 * 16 * 4);
  const __amdgpu_buffer_rsrc_t wr1 = make_rsrc(NB == 2 ? Wp1 : Wp0, (int64_t)(NB == 2 ? T1 : T0) * 16 * 16 * 4);
  const int wvoff = (g * 16 + l16) * 4;

  // Slot i of wave w is tile t = w + 16 i (TPB >= the tiles / 16); slots past
  // the last tile have a zero direction operand and read zero LDS columns,
  // so every wave runs the same branch-free instruction stream.  keep[i]
  // zeroes, in the P products, the lanes of MFMA rows that belong to the
  // other view (rows 0-7: A_0, rows 8-15: A_1).
  float wreg[TPB][4];
  float keep[TPB];
  acc_t acc[TPB][NT];
#pragma unroll
  for (int i = 0; i < TPB; ++i) {
    const int t = w + kF32Waves * i;
    const bool b1 = (NB == 2) && (t >= T0);
    keep[i] = (NB == 1 || (l16 >> 3) == (int)b1) ? 1.f : 0.f;
    const int ct = b1 ? t - T0 : t;
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) {
      const int soff = (ct * 16 + 4 * s2) * 16 * 4;
      float v = 0.f;
      if (t < TT) v = b1 ? buf_load<float>(wr1, wvoff + soff, 0) : buf_load<float>(wr0, wvoff + soff, 0);
      wreg[i][s2] = v;
    }
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[i][j] = acc_t{0, 0, 0, 0};
  }
  // The columns of the slots past the last tile are never loaded: zero both
  // row buffers once.
  for (int e = tid; e < 2 * R * pitch; e += kF32Threads) dsm[e] = 0.f;
  __syncthreads();

  // Loads of row block rbk into buffer xb: wave w moves chunks j = w, w + 16,
  // ... of every row.  One buffer resource per view and block; rows past n
  // lie past its num_records and read as zero.  A chunk's tail past the
  // view's last column reads the next row's leading values (finite; they
  // meet zero direction rows in P and land in J rows that are not stored).
  auto issue_block = [&](int rbk, float* xb) __attribute__((always_inline)) {
    const int64_t row0 = (int64_t)rbk * R;
    const int rows = (int)(n - row0 < R ? n - row0 : R);
    const __amdgpu_buffer_rsrc_t r0 = make_rsrc(A0 + row0 * d0, (int64_t)rows * d0 * 4);
    const __amdgpu_buffer_rsrc_t r1 =
        NB == 2 ? make_rsrc(A1 + row0 * d1, (int64_t)rows * d1 * 4) : r0;
    for (int j = w; j < nch; j += kF32Waves) {
      const bool s1 = (NB == 2) && (j >= nch0);
      const int jj = s1 ? j - nch0 : j;
      const int span = (s1 ? T1 : T0) * 16;
      const int o = min(jj * CH, span - CH);
      const int db4 = (s1 ? d1 : d0) * 4;
      float* dst = xb + (s1 ? T0 * 16 : 0) + o;
      const int vbase = (o + lane * VEC) * 4;
      const __amdgpu_buffer_rsrc_t rs = s1 ? r1 : r0;
#pragma unroll
      for (int r = 0; r < R; ++r) dma_row_chunk<VEC>(rs, dst + r * pitch, vbase + r * db4);
    }
  };

  // per-lane operand bases (floats); slot i adds 16 (w + 16 i)
  const int base_b = (l16 & (R - 1)) * pitch + g + 16 * w;   // P phase: row l16 mod 8, column 4 s2 + g
  const int base_d = g * pitch + l16 + 16 * w;               // J phase: row g + 4 s, column l16
  const int pf_b = g * 17 + l16;                              // pfull row g + 4 s (as the J-phase A operand)

  int rb = blockIdx.x;
  int boff = 0;   // float offset of the current buffer
  if (rb < nrb) issue_block(rb, dsm);
  for (; rb < nrb; rb += gridDim.x) {
    __builtin_amdgcn_s_waitcnt(0);   // this wave's loads of the block have landed
    __syncthreads();                 // ... and every wave's; the other buffer is free
    const float* xs = dsm + boff;
    if (rb + (int)gridDim.x < nrb) issue_block(rb + gridDim.x, dsm + (R * pitch - boff));
    // (b) P partials over this wave's slots.  Both views share one
    // accumulator: MFMA rows 0-7 take A_0 W_0 (the lanes of rows 8-15 read
    // zero on A_0 tiles) and rows 8-15 take A_1 W_1; two accumulators
    // alternate to break the dependence chain.
    acc_t pacc[2] = {acc_t{0, 0, 0, 0}, acc_t{0, 0, 0, 0}};
#pragma unroll
    for (int i = 0; i < TPB; ++i) {
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2) {
        float a = xs[base_b + 16 * kF32Waves * i + 4 * s2];
        if (NB == 2) a *= keep[i];
        pacc[i & 1] = mfma16x16x4(a, wreg[i][s2], pacc[i & 1]);
      }
    }
    // (c) sum P over the waves
#pragma unroll
    for (int r = 0; r < 4; ++r) red[w * 256 + (4 * g + r) * 16 + l16] = pacc[0][r] + pacc[1][r];
    lds_only_barrier();
    if (tid < NB * R * 16) {
      float v = 0.f;
#pragma unroll
      for (int ww = 0; ww < kF32Waves; ++ww) v += red[ww * 256 + tid];
      const int row = tid >> 4, col = tid & 15;
      pfull[(row >> 3) * (R * 17) + (row & 7) * 17 + col] = v;
    }
    lds_only_barrier();
    // (d) A_b^T [P_0 | P_1] for this wave's slots
    float pb[R / 4][NT];
#pragma unroll
    for (int s = 0; s < R / 4; ++s)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) pb[s][nt] = pfull[nt * (R * 17) + pf_b + 4 * s * 17];
#pragma unroll
    for (int i = 0; i < TPB; ++i) {
#pragma unroll
      for (int s = 0; s < R / 4; ++s) {
        const float a = xs[base_d + 4 * s * pitch + 16 * kF32Waves * i];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[i][nt] = mfma16x16x4(a, pb[s][nt], acc[i][nt]);
      }
    }
    boff = R * pitch - boff;
  }
  // epilogue: this workgroup's partial (rows = concatenated columns of A)
  const int W_out = NB * k;
  const int D = d0 + (NB == 2 ? d1 : 0);
  float* out = partial + (int64_t)blockIdx.x * D * W_out;
#pragma unroll
  for (int i = 0; i < TPB; ++i) {
    const int t = w + kF32Waves * i;
    if (t < TT) {
      const bool b1 = (NB == 2) && (t >= T0);
      const int db = b1 ? d1 : d0;
      const int ct = b1 ? t - T0 : t;
      const int rowbase = b1 ? d0 : 0;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int col = l16;
        if (col < k) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int c = ct * 16 + acc_row<float>(lane, r);
            if (c < db) out[(int64_t)(rowbase + c) * W_out + nt * k + col] = acc[i][nt][r];
          }
        }
      }
    }
  }
}

// ------------------------------------------------------------------
// FP32, two views: the DMA-fed pass above with the narrow products on 4x4
// matrix-core blocks (v_mfma_f32_4x4x1f32: sixteen independent 4 x 4 outer
// products per instruction), which removes most of the zero padding that
// 16 x 16 tiles carry for 8-row blocks and k <= 12:
//   * P_b = A_b W_b (8 rows x k): waves 0-7 work on view 0, waves 8-15 on
//     view 1.  A block is 4 rows x 4 direction columns of one tile over one
//     of every four of its columns: the four 16-lane rows take four tiles,
//     the four blocks of a row the four column phases, rows 0-3 and 4-7 are
//     separate instructions.  The four tiles are summed in registers by
//     lane-row swaps and the column phases by two DPP rotations, so each
//     wave publishes one partial to the cross-wave sum.
//   * J_b = A_b^T [P_0 | P_1]: whole 16-column tiles of [P_0 | P_1] on the
//     16 x 16 x 4 products; the remaining 4-column groups on 4x4 blocks,
//     one row of the block per instruction over four tiles at once (the
//     16-lane rows take the tiles, the blocks of a row 4 of its columns).
// [P_0 | P_1] is packed tight (2k columns; C4 = ceil(k / 2) groups of 4).
// In the P products wave w takes tiles w % 8 + 8 (4 G + row) of view w / 8
// (G < SV / 2); in the J products it owns SV tiles of each view (slot
// i < SV: tile w + 16 i of view 0, slot SV + i: tile w + 16 i of view 1).
// Tiles past a view's last have a zero direction operand and their J rows
// are not stored.  The row-block stream (DMA loads, double buffer,
// barriers) is that of k_pass_dma.
template <int N>
__device__ __forceinline__ float dpp_row_ror(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x120 + N, 0xF, 0xF, false));
}
__device__ __forceinline__ f32x4 mfma4x4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 0);
}

// Row pitch of the 4x4-block pass: 16 mod 64 floats, so that four rows of
// 16 consecutive columns (the J-phase operand) fall on 64 distinct banks,
// as do the P operands' column quadruples of one 16-lane row.
__host__ __device__ constexpr int quad_pitch(int TPB) { return ((16 * 16 * TPB + 63) / 64) * 64 + 16; }

// The matrix-core results in p are complete before the lane swaps below
// read them (the swaps are inline assembly, outside the compiler's hazard
// tracking): 19 wait states cover the longest result latency.
template <int KH>
__device__ __forceinline__ void xdl_settle(f32x4 (&p)[KH]) {
  if constexpr (KH == 1) asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 3" : "+v"(p[0]));
  else if constexpr (KH == 2) asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 3" : "+v"(p[0]), "+v"(p[1]));
  else if constexpr (KH == 3) asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 3" : "+v"(p[0]), "+v"(p[1]), "+v"(p[2]));
  else {
    static_assert(KH == 4, "up to four accumulators");
    asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 3" : "+v"(p[0]), "+v"(p[1]), "+v"(p[2]), "+v"(p[3]));
  }
}

// Sums of the four values x[0..3] over the four 16-lane rows, scattered:
// afterwards 16-lane row g holds the sum of x[r], r = (0, 2, 1, 3)[g].
// v_permlane32_swap exchanges the upper half of its first operand with the
// lower half of its second, so the sum of the swapped pair (x[0], x[1])
// holds x[0] over rows (g, g + 2) in rows 0-1 and x[1] in rows 2-3;
// v_permlane16_swap (odd rows of the first operand with even rows of the
// second) then finishes two such pairs in one step.  Four swaps and four
// adds reduce four values, against two swaps and three adds per value for
// separate full sums.
__device__ __forceinline__ float rows_scatter_sum(f32x4 x) {
  float u0 = x[0], v0 = x[1], u1 = x[2], v1 = x[3];
  asm("s_nop 1\n\tv_permlane32_swap_b32 %0, %1\n\tv_permlane32_swap_b32 %2, %3\n\ts_nop 1"
      : "+v"(u0), "+v"(v0), "+v"(u1), "+v"(v1));
  float p = u0 + v0, q = u1 + v1;
  asm("s_nop 1\n\tv_permlane16_swap_b32 %0, %1\n\ts_nop 1" : "+v"(p), "+v"(q));
  return p + q;
}

// The same settle for two rows of KG accumulators.
template <int KG>
__device__ __forceinline__ void xdl_settle2(f32x4 (&p)[2][KG]) {
  if constexpr (KG == 1) asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 3" : "+v"(p[0][0]), "+v"(p[1][0]));
  else if constexpr (KG == 2)
    asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 3" : "+v"(p[0][0]), "+v"(p[0][1]), "+v"(p[1][0]), "+v"(p[1][1]));
  else if constexpr (KG == 3)
    asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 3"
                 : "+v"(p[0][0]), "+v"(p[0][1]), "+v"(p[0][2]), "+v"(p[1][0]), "+v"(p[1][1]), "+v"(p[1][2]));
  else {
    static_assert(KG == 4, "up to four accumulators per row group");
    asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 3"
                 : "+v"(p[0][0]), "+v"(p[0][1]), "+v"(p[0][2]), "+v"(p[0][3]), "+v"(p[1][0]), "+v"(p[1][1]),
                   "+v"(p[1][2]), "+v"(p[1][3]));
  }
}

template <int SV, int C4>
struct QuadShape {
  static constexpr int TPB = 2 * SV;        // tile slots per wave
  static constexpr int KG = (C4 + 1) / 2;   // 4-column groups of one view's P
  static constexpr int JQ = C4 / 4;         // whole 16-column tiles of [P_0 | P_1]
  static constexpr int JR = C4 % 4;         // remaining 4-column groups
  static constexpr int NG = TPB / 4;        // 4-slot groups of the remainder products
  static constexpr int PP = 4 * C4 + 1;     // row pitch of [P_0 | P_1] in LDS
  static constexpr int PG = SV / 2;        // 4-tile groups of a wave's P products
  static constexpr int RED = kDmaRows * 4 * KG;   // one P partial (8 rows x 4 KG)
  // LDS pitch of the wave partials: 8 mod 32 floats, so that the four lanes
  // of a reducing quad (partials 2 apart) fall on different banks
  static constexpr int REDP = RED + 8;
};

// Per-block work of k_pass_quad.  The LDS regions arrive as separate
// restrict pointers: the inlined accesses then carry alias scopes, and the
// compiler's wait insertion can see that the reads of the current block,
// the P partials and [P_0 | P_1] are disjoint from the next block's
// in-flight DMA (without that it waits for the DMA before the first LDS
// read, and the double buffer overlaps nothing).  The next block's DMA is
// issued here when next_row0 >= 0.
template <int SV, int C4, int VEC>
__device__ __forceinline__ void quad_step(const float* __restrict__ xs, float* __restrict__ xnext,
                                          float* __restrict__ red, float* __restrict__ pfull, int64_t next_row0,
                                          const float* A0, const float* A1, int64_t n, int d0, int d1, int k,
                                          int T0, int T1, int nch0, int nch, int pitch, int w, int lane,
                                          const float (&wreg)[QuadShape<SV, C4>::PG][4][QuadShape<SV, C4>::KG],
                                          const int (&pcol)[QuadShape<SV, C4>::PG],
                                          const int (&rbase)[QuadShape<SV, C4>::NG],
                                          f32x4 (&acc)[QuadShape<SV, C4>::TPB][QuadShape<SV, C4>::JQ > 0 ? QuadShape<SV, C4>::JQ : 1],
                                          f32x4 (&accr)[QuadShape<SV, C4>::NG][QuadShape<SV, C4>::JR > 0 ? QuadShape<SV, C4>::JR : 1],
                                          bool dma_only) {
  using Q = QuadShape<SV, C4>;
  constexpr int R = kDmaRows;
  constexpr int CH = 64 * VEC;
  constexpr int TPB = Q::TPB, KG = Q::KG, JQ = Q::JQ, JR = Q::JR, NG = Q::NG, PP = Q::PP, PG = Q::PG;
  constexpr int RED = Q::RED, REDP = Q::REDP;
  const int tid = threadIdx.x;
  const int g = lane >> 4, l16 = lane & 15, cs = (lane >> 2) & 3, q4 = lane & 3;
  if (next_row0 >= 0) {
    // waves 0-7 move chunks j = w, w + 8, ... of every row (the other
    // eight waves go straight to the products); one buffer resource per
    // view, rows past n read as zero
    const int rows = (int)(n - next_row0 < R ? n - next_row0 : R);
    const __amdgpu_buffer_rsrc_t r0 = make_rsrc(A0 + next_row0 * d0, (int64_t)rows * d0 * 4);
    const __amdgpu_buffer_rsrc_t r1 = make_rsrc(A1 + next_row0 * d1, (int64_t)rows * d1 * 4);
    for (int j = w; j < nch && w < kF32Waves / 2; j += kF32Waves / 2) {
      const bool s1 = j >= nch0;
      const int jj = s1 ? j - nch0 : j;
      const int span = (s1 ? T1 : T0) * 16;
      const int o = min(jj * CH, span - CH);
      const int db4 = (s1 ? d1 : d0) * 4;
      float* dst = xnext + (s1 ? T0 * 16 : 0) + o;
      const int vbase = (o + lane * VEC) * 4;
      const __amdgpu_buffer_rsrc_t rs = s1 ? r1 : r0;
#pragma unroll
      for (int r = 0; r < R; ++r) dma_row_chunk<VEC>(rs, dst + r * pitch, vbase + r * db4);
    }
  }
  if (dma_only) return;
  // (b) P partials of this wave's view over its tiles: rows 4 rg + q4,
  // columns 4 cs .. 4 cs + 3 of each tile
  {
    f32x4 pacc[R / 4][KG];
#pragma unroll
    for (int rg = 0; rg < R / 4; ++rg)
#pragma unroll
      for (int kg = 0; kg < KG; ++kg) pacc[rg][kg] = f32x4{0, 0, 0, 0};
    // all operand reads of the block issued before the first product
    float4 a4[PG][R / 4];
#pragma unroll
    for (int G = 0; G < PG; ++G)
#pragma unroll
      for (int rg = 0; rg < R / 4; ++rg) a4[G][rg] = *reinterpret_cast<const float4*>(xs + (4 * rg + q4) * pitch + pcol[G]);
#pragma unroll
    for (int G = 0; G < PG; ++G)
#pragma unroll
      for (int rg = 0; rg < R / 4; ++rg) {
        const float av[4] = {a4[G][rg].x, a4[G][rg].y, a4[G][rg].z, a4[G][rg].w};
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int kg = 0; kg < KG; ++kg) pacc[rg][kg] = mfma4x4(av[s], wreg[G][s][kg], pacc[rg][kg]);
      }
    // The wave's partial: the four tiles of a 16-lane row by a scattered
    // row sum, then the four column phases (in every lane, so that both
    // rotations fold into the adds); lane (g, 0, q4) holds row 4 rg + r,
    // r = (0, 2, 1, 3)[g], direction column 4 kg + q4: element
    // ((rg KG + kg) 4 + q4) 4 + r of the partial.
    xdl_settle2<KG>(pacc);
    float sums[2][KG];
#pragma unroll
    for (int rg = 0; rg < 2; ++rg)
#pragma unroll
      for (int kg = 0; kg < KG; ++kg) {
        float x = rows_scatter_sum(pacc[rg][kg]);
        x += dpp_row_ror<4>(x);
        x += dpp_row_ror<8>(x);
        asm volatile("" : "+v"(x));
        sums[rg][kg] = x;
      }
    if (cs == 0) {
      const int r = ((g & 1) << 1) | (g >> 1);
      float* rw = red + w * REDP + 4 * q4 + r;
#pragma unroll
      for (int rg = 0; rg < 2; ++rg)
#pragma unroll
        for (int kg = 0; kg < KG; ++kg) rw[(rg * KG + kg) * 16] = sums[rg][kg];
    }
  }
  lds_only_barrier();
  // Sum over a view's 8 wave partials in a fixed order: the four lanes of a
  // quad add two partials each, then two quad exchanges combine them.  The indexes are recomputed per
  // block (an opaque copy of tid): hoisted out of the loop they would stay
  // live through the whole block and be spilled.
  for (int t4 = tid; t4 < 8 * RED; t4 += kF32Threads) {
    int t = t4;
    asm volatile("" : "+v"(t));
    const int o = t >> 2, j = t & 3;
    const int v = o / RED, e = o - v * RED;
    const float* src = red + (v * kF32Waves / 2 + 2 * j) * REDP + e;
    float sum = src[0] + src[REDP];
    sum += __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, sum), 0xB1, 0xF, 0xF, true));
    sum += __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, sum), 0x4E, 0xF, 0xF, true));
    const int r = e & 3, q = (e >> 2) & 3, rk = e >> 4;
    const int rg = rk / KG, kg = rk - rg * KG;
    const int col = 4 * kg + q;
    if (j == 0 && col < k) pfull[(4 * rg + r) * PP + v * k + col] = sum;
  }
  lds_only_barrier();
  // (d) J = A_b^T [P_0 | P_1]
  if constexpr (JQ > 0) {
    float pb[R / 4][JQ];
#pragma unroll
    for (int s = 0; s < R / 4; ++s)
#pragma unroll
      for (int jq = 0; jq < JQ; ++jq) pb[s][jq] = pfull[(g + 4 * s) * PP + 16 * jq + l16];
#pragma unroll
    for (int i = 0; i < TPB; ++i) {
      const int col = 16 * (i < SV ? w + 16 * i : T0 + w + 16 * (i - SV));
#pragma unroll
      for (int s = 0; s < R / 4; ++s) {
        const float a = xs[(g + 4 * s) * pitch + col + l16];
#pragma unroll
        for (int jq = 0; jq < JQ; ++jq) acc[i][jq] = mfma16x16x4(a, pb[s][jq], acc[i][jq]);
      }
    }
  }
  if constexpr (JR > 0) {
    // step rho: lane row g takes block row (rho + g) mod R (the four tiles
    // of an instruction then read different banks)
#pragma unroll
    for (int rho = 0; rho < R; ++rho) {
      const int row = (rho + g) & (R - 1);
      float b[JR];
#pragma unroll
      for (int jr = 0; jr < JR; ++jr) b[jr] = pfull[row * PP + 16 * JQ + 4 * jr + q4];
#pragma unroll
      for (int G = 0; G < NG; ++G) {
        const float a = xs[row * pitch + rbase[G]];
#pragma unroll
        for (int jr = 0; jr < JR; ++jr) accr[G][jr] = mfma4x4(a, b[jr], accr[G][jr]);
      }
    }
  }
}

template <int SV, int C4, int VEC>
__global__ void __launch_bounds__(kF32Threads) k_pass_quad(const float* __restrict__ A0, const float* __restrict__ A1,
                                                           int64_t n, int d0, int d1, int k,
                                                           const double* __restrict__ W0,
                                                           const double* __restrict__ W1, int nrb,
                                                           float* __restrict__ partial, const int* __restrict__ done) {
  if (done && *done) return;
  using Q = QuadShape<SV, C4>;
  constexpr int R = kDmaRows;
  constexpr int CH = 64 * VEC;
  constexpr int TPB = Q::TPB, KG = Q::KG, JQ = Q::JQ, JR = Q::JR, NG = Q::NG, PP = Q::PP, PG = Q::PG;
  extern __shared__ float dsm[];
  const int T0 = (d0 + 15) >> 4, T1 = (d1 + 15) >> 4;
  const int nch0 = (T0 * 16 + CH - 1) / CH, nch1 = (T1 * 16 + CH - 1) / CH;
  const int nch = nch0 + nch1;
  const int pitch = quad_pitch(TPB);
  float* red = dsm + 2 * R * pitch;                 // [wave] partials, pitch REDP
  float* pfull = red + kF32Waves * Q::REDP;         // [R][PP]

  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, l16 = lane & 15;
  const int cs = (lane >> 2) & 3, q4 = lane & 3;
  const int pv = w >> 3;   // view of this wave's P products (wave-uniform)

  // direction operands of the P blocks: group G, tile tv = w % 8 + 8 (4 G +
  // g) of view pv, its column 4 cs + s, direction column 4 kg + q4, read
  // from the FP64 directions (d x k row-major; rows past d lie past the
  // resource and read zero, columns past k take the zero offset)
  const __amdgpu_buffer_rsrc_t wrs = make_rsrc(pv ? W1 : W0, (int64_t)(pv ? d1 : d0) * k * 8);
  float wreg[PG][4][KG];
  int pcol[PG];   // LDS column of the tile's phase-cs quadruple
#pragma unroll
  for (int G = 0; G < PG; ++G) {
    const int tv = (w & 7) + 8 * (4 * G + g);
    const bool ok = tv < (pv ? T1 : T0);
    pcol[G] = 16 * (pv ? T0 + tv : tv) + 4 * cs;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int kg = 0; kg < KG; ++kg) {
        const int col = 4 * kg + q4;
        const int off = (ok && col < k) ? ((16 * tv + 4 * cs + s) * k + col) * 8 : kOob;
        wreg[G][s][kg] = (float)buf_load<double>(wrs, off, 0);
      }
  }
  f32x4 acc[TPB][JQ > 0 ? JQ : 1];
  f32x4 accr[NG][JR > 0 ? JR : 1];
#pragma unroll
  for (int i = 0; i < TPB; ++i)
#pragma unroll
    for (int j = 0; j < (JQ > 0 ? JQ : 1); ++j) acc[i][j] = f32x4{0, 0, 0, 0};
#pragma unroll
  for (int G = 0; G < NG; ++G)
#pragma unroll
    for (int j = 0; j < (JR > 0 ? JR : 1); ++j) accr[G][j] = f32x4{0, 0, 0, 0};
  int rbase[NG];   // remainder blocks: slot 4 G + g, column l16
#pragma unroll
  for (int G = 0; G < NG; ++G) {
    const int i = 4 * G + g;
    rbase[G] = 16 * (i < SV ? w + 16 * i : T0 + w + 16 * (i - SV)) + l16;
  }
  // Columns past the last tile are never loaded and the padding columns of
  // [P_0 | P_1] never written: zero both row buffers and pfull once.
  for (int e = tid; e < 2 * R * pitch; e += kF32Threads) dsm[e] = 0.f;
  for (int e = tid; e < R * PP; e += kF32Threads) pfull[e] = 0.f;
  __syncthreads();

  int rb = blockIdx.x;
  int boff = 0;
  if (rb < nrb)
    quad_step<SV, C4, VEC>(dsm + R * pitch, dsm, red, pfull, (int64_t)rb * R, A0, A1, n, d0, d1, k, T0, T1, nch0,
                           nch, pitch, w, lane, wreg, pcol, rbase, acc, accr, true);
  for (; rb < nrb; rb += gridDim.x) {
    __builtin_amdgcn_s_waitcnt(0);   // this wave's loads of the block have landed
    __syncthreads();                 // ... and every wave's; the other buffer is free
    const int64_t nxt = rb + (int)gridDim.x < nrb ? (int64_t)(rb + gridDim.x) * R : -1;
    quad_step<SV, C4, VEC>(dsm + boff, dsm + (R * pitch - boff), red, pfull, nxt, A0, A1, n, d0, d1, k, T0, T1,
                           nch0, nch, pitch, w, lane, wreg, pcol, rbase, acc, accr, false);
    boff = R * pitch - boff;
  }
  // epilogue: this workgroup's partial (rows = concatenated columns of A,
  // columns = [P_0 | P_1])
  const int W_out = 2 * k;
  const int D = d0 + d1;
  float* out = partial + (int64_t)blockIdx.x * D * W_out;
  if constexpr (JQ > 0) {
#pragma unroll
    for (int i = 0; i < TPB; ++i) {
      const int v = i < SV ? 0 : 1;
      const int tv = w + 16 * (i - v * SV);
      if (tv < (v ? T1 : T0)) {
        const int db = v ? d1 : d0, rowbase = v ? d0 : 0;
#pragma unroll
        for (int jq = 0; jq < JQ; ++jq) {
          const int c = 16 * jq + l16;
          if (c < W_out) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = 16 * tv + acc_row<float>(lane, r);
              if (row < db) out[(int64_t)(rowbase + row) * W_out + c] = acc[i][jq][r];
            }
          }
        }
      }
    }
  }
  if constexpr (JR > 0) {
#pragma unroll
    for (int G = 0; G < NG; ++G) {
      const int i = 4 * G + g;
      const int v = i < SV ? 0 : 1;
      const int tv = w + 16 * (i - v * SV);
      if (tv < (v ? T1 : T0)) {
        const int db = v ? d1 : d0, rowbase = v ? d0 : 0;
#pragma unroll
        for (int jr = 0; jr < JR; ++jr) {
          const int c = 16 * JQ + 4 * jr + q4;
          if (c < W_out) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = 16 * tv + 4 * cs + r;
              if (row < db) out[(int64_t)(rowbase + row) * W_out + c] = accr[G][jr][r];
            }
          }
        }
      }
    }
  }
}


// ------------------------------------------------------------------
// FP32, one view (FDA: J = A^T (A W), k <= 20): the same row stream with
// the narrow products on 4x4 blocks.
//   * P = A W (8 rows x k): wave w takes tiles w + 16 (4 G + g) (the four
//     16-lane rows g of an instruction take four tiles); a block is 4 rows
//     x 4 direction columns over one column in four; rows 0-3 and 4-7 are
//     done one after the other (20 accumulator registers at k = 20).  The
//     four tiles of an instruction are summed by lane-row swaps
//     (v_permlane32_swap, v_permlane16_swap) that scatter the sums of four
//     values over the four lane rows, the column phases by two DPP
//     rotations, so each wave publishes one 8 x 4 KG partial.
//   * J = A^T P: whole 16-column tiles of P on 16x16x4, the remaining
//     4-column groups on 4x4 blocks over four tiles at once, as above.
// Wave w owns J slots w + 16 i (i < TPB); slots and P tiles past the last
// tile have zero directions and their rows are not stored.
template <int TPB, int KG>
struct Quad1Shape {
  static constexpr int PG = TPB / 4;        // 4-tile groups of a wave's P products
  static constexpr int JQ = KG / 4;         // whole 16-column tiles of P
  static constexpr int JR = KG % 4;         // remaining 4-column groups
  static constexpr int NG = TPB / 4;        // 4-slot groups of the remainder products
  static constexpr int PP = 4 * KG + 1;     // row pitch of P in LDS
  static constexpr int RED = kDmaRows * 4 * KG;
  // LDS pitch of the wave partials: 4 mod 16 floats, so that the four lanes
  // of a reducing quad (partials 4 apart) fall on different banks
  static constexpr int REDP = RED + 4;
};

template <int TPB, int KG, int VEC>
__device__ __forceinline__ void quad1_step(const float* __restrict__ xs, float* __restrict__ xnext,
                                           float* __restrict__ red, float* __restrict__ pfull, int64_t next_row0,
                                           const float* A0, int64_t n, int d0, int k, int T0, int nch0, int pitch,
                                           int w, int lane, const float (&wreg)[TPB / 4][4][KG],
                                           f32x4 (&acc)[TPB][Quad1Shape<TPB, KG>::JQ > 0 ? Quad1Shape<TPB, KG>::JQ : 1],
                                           f32x4 (&accr)[TPB / 4][Quad1Shape<TPB, KG>::JR > 0 ? Quad1Shape<TPB, KG>::JR : 1],
                                           bool dma_only) {
  using Q = Quad1Shape<TPB, KG>;
  constexpr int R = kDmaRows;
  constexpr int CH = 64 * VEC;
  constexpr int JQ = Q::JQ, JR = Q::JR, NG = Q::NG, PP = Q::PP, PG = Q::PG, RED = Q::RED, REDP = Q::REDP;
  const int tid = threadIdx.x;
  const int g = lane >> 4, l16 = lane & 15, cs = (lane >> 2) & 3, q4 = lane & 3;
  if (next_row0 >= 0) {
    const int rows = (int)(n - next_row0 < R ? n - next_row0 : R);
    const __amdgpu_buffer_rsrc_t r0 = make_rsrc(A0 + next_row0 * d0, (int64_t)rows * d0 * 4);
    const int span = T0 * 16;
    const int db4 = d0 * 4;
    for (int j = w; j < nch0; j += kF32Waves) {
      const int o = min(j * CH, span - CH);
      float* dst = xnext + o;
      const int vbase = (o + lane * VEC) * 4;
#pragma unroll
      for (int r = 0; r < R; ++r) dma_row_chunk<VEC>(r0, dst + r * pitch, vbase + r * db4);
    }
  }
  if (dma_only) return;
  // (b) P partial of this wave: rows 4 rg + q4, one half at a time; with
  // five direction-column groups also in two passes over the groups (the
  // accumulators of all five would not fit beside the J accumulators)
  constexpr int KH = KG >= 5 ? (KG + 1) / 2 : KG;
#pragma unroll
  for (int rg = 0; rg < 2; ++rg)
#pragma unroll
  for (int k0 = 0; k0 < KG; k0 += KH) {
    f32x4 pacc[KH];
#pragma unroll
    for (int kk = 0; kk < KH; ++kk) pacc[kk] = f32x4{0, 0, 0, 0};
#pragma unroll
    for (int G = 0; G < PG; ++G) {
      const int col = 16 * (w + 16 * (4 * G + g)) + 4 * cs;
      const float4 a = *reinterpret_cast<const float4*>(xs + (4 * rg + q4) * pitch + col);
      const float av[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int kk = 0; kk < KH; ++kk)
          if (k0 + kk < KG) pacc[kk] = mfma4x4(av[s], wreg[G][s][k0 + kk], pacc[kk]);
    }
    // the wave's partial: the four tiles of a lane row by a scattered
    // row sum, then the four column phases (in every lane, so that both
    // rotations fold into the adds); lane (g, 0, q4) holds row 4 rg + r,
    // r = (0, 2, 1, 3)[g], direction column 4 kg + q4
    xdl_settle<KH>(pacc);
    float sums[KH];
#pragma unroll
    for (int kk = 0; kk < KH; ++kk) {
      float x = rows_scatter_sum(pacc[kk]);
      x += dpp_row_ror<4>(x);
      x += dpp_row_ror<8>(x);
      asm volatile("" : "+v"(x));
      sums[kk] = x;
    }
    if (cs == 0) {
      const int r = ((g & 1) << 1) | (g >> 1);
#pragma unroll
      for (int kk = 0; kk < KH; ++kk)
        if (k0 + kk < KG) red[w * REDP + (4 * rg + r) * (4 * KG) + 4 * (k0 + kk) + q4] = sums[kk];
    }
  }
  lds_only_barrier();
  // Sum over the 16 wave partials in a fixed order: the four lanes of a
  // quad add four partials each, then two quad exchanges combine them.
  for (int t4 = tid; t4 < 4 * RED; t4 += kF32Threads) {
    int t = t4;
    asm volatile("" : "+v"(t));
    const int e = t >> 2, j = t & 3;
    const float* src = red + 4 * j * REDP + e;
    float sum = 0.f;
#pragma unroll
    for (int h = 0; h < 4; ++h) sum += src[h * REDP];
    sum += __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, sum), 0xB1, 0xF, 0xF, true));
    sum += __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, sum), 0x4E, 0xF, 0xF, true));
    const int row = e / (4 * KG), col = e - row * (4 * KG);
    if (j == 0 && col < k) pfull[row * PP + col] = sum;
  }
  lds_only_barrier();
  // (d) J = A^T P
  if constexpr (JQ > 0) {
    float pb[2][JQ];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int jq = 0; jq < JQ; ++jq) pb[s][jq] = pfull[(g + 4 * s) * PP + 16 * jq + l16];
#pragma unroll
    for (int i = 0; i < TPB; ++i) {
      const int col = 16 * (w + 16 * i);
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const float a = xs[(g + 4 * s) * pitch + col + l16];
#pragma unroll
        for (int jq = 0; jq < JQ; ++jq) acc[i][jq] = mfma16x16x4(a, pb[s][jq], acc[i][jq]);
      }
    }
  }
  if constexpr (JR > 0) {
#pragma unroll
    for (int rho = 0; rho < R; ++rho) {
      const int row = (rho + g) & (R - 1);
      float b[JR];
#pragma unroll
      for (int jr = 0; jr < JR; ++jr) b[jr] = pfull[row * PP + 16 * JQ + 4 * jr + q4];
#pragma unroll
      for (int G = 0; G < NG; ++G) {
        const float a = xs[row * pitch + 16 * (w + 16 * (4 * G + g)) + l16];
#pragma unroll
        for (int jr = 0; jr < JR; ++jr) accr[G][jr] = mfma4x4(a, b[jr], accr[G][jr]);
      }
    }
  }
}

template <int TPB, int KG, int VEC>
__global__ void __launch_bounds__(kF32Threads) k_pass_quad1(const float* __restrict__ A0, int64_t n, int d0, int k,
                                                            const float* __restrict__ Wp0, int nrb,
                                                            float* __restrict__ partial, const int* __restrict__ done) {
  if (done && *done) return;
  using Q = Quad1Shape<TPB, KG>;
  constexpr int R = kDmaRows;
  constexpr int CH = 64 * VEC;
  constexpr int JQ = Q::JQ, JR = Q::JR, NG = Q::NG, PP = Q::PP, PG = Q::PG;
  extern __shared__ float dsm[];
  const int T0 = (d0 + 15) >> 4;
  const int nch0 = (T0 * 16 + CH - 1) / CH;
  const int pitch = quad_pitch(TPB);
  float* red = dsm + 2 * R * pitch;          // [wave][R][4 KG], pitch REDP
  float* pfull = red + kF32Waves * Q::REDP;  // [R][PP]
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, l16 = lane & 15, cs = (lane >> 2) & 3, q4 = lane & 3;

  // direction operands of the P blocks: tile w + 16 (4 G + g), its column
  // 4 cs + s, direction column 4 kg + q4, from the directions packed to
  // FP32 (4 KG columns, zero padded; every workgroup reads all of them, and
  // at k = 19 the FP64 iterate would double that L2 traffic)
  const __amdgpu_buffer_rsrc_t wrs = make_rsrc(Wp0, (int64_t)T0 * 16 * (4 * KG) * 4);
  float wreg[PG][4][KG];
#pragma unroll
  for (int G = 0; G < PG; ++G) {
    const int tv = w + 16 * (4 * G + g);
    const bool ok = tv < T0;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int kg = 0; kg < KG; ++kg) {
        const int off = ok ? ((16 * tv + 4 * cs + s) * (4 * KG) + 4 * kg + q4) * 4 : kOob;
        wreg[G][s][kg] = buf_load<float>(wrs, off, 0);
      }
  }
  f32x4 acc[TPB][JQ > 0 ? JQ : 1];
  f32x4 accr[NG][JR > 0 ? JR : 1];
#pragma unroll
  for (int i = 0; i < TPB; ++i)
#pragma unroll
    for (int j = 0; j < (JQ > 0 ? JQ : 1); ++j) acc[i][j] = f32x4{0, 0, 0, 0};
#pragma unroll
  for (int G = 0; G < NG; ++G)
#pragma unroll
    for (int j = 0; j < (JR > 0 ? JR : 1); ++j) accr[G][j] = f32x4{0, 0, 0, 0};
  for (int e = tid; e < 2 * R * pitch; e += kF32Threads) dsm[e] = 0.f;
  for (int e = tid; e < R * PP; e += kF32Threads) pfull[e] = 0.f;
  __syncthreads();

  int rb = blockIdx.x;
  int boff = 0;
  if (rb < nrb)
    quad1_step<TPB, KG, VEC>(dsm + R * pitch, dsm, red, pfull, (int64_t)rb * R, A0, n, d0, k, T0, nch0, pitch, w,
                             lane, wreg, acc, accr, true);
  for (; rb < nrb; rb += gridDim.x) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    const int64_t nxt = rb + (int)gridDim.x < nrb ? (int64_t)(rb + gridDim.x) * R : -1;
    quad1_step<TPB, KG, VEC>(dsm + boff, dsm + (R * pitch - boff), red, pfull, nxt, A0, n, d0, k, T0, nch0, pitch,
                             w, lane, wreg, acc, accr, false);
    boff = R * pitch - boff;
  }
  // epilogue: this workgroup's partial (d0 x k)
  float* out = partial + (int64_t)blockIdx.x * d0 * k;
  if constexpr (JQ > 0) {
#pragma unroll
    for (int i = 0; i < TPB; ++i) {
      const int tv = w + 16 * i;
      if (tv < T0) {
#pragma unroll
        for (int jq = 0; jq < JQ; ++jq) {
          const int c = 16 * jq + l16;
          if (c < k) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = 16 * tv + acc_row<float>(lane, r);
              if (row < d0) out[(int64_t)row * k + c] = acc[i][jq][r];
            }
          }
        }
      }
    }
  }
  if constexpr (JR > 0) {
#pragma unroll
    for (int G = 0; G < NG; ++G) {
      const int tv = w + 16 * (4 * G + g);
      if (tv < T0) {
#pragma unroll
        for (int jr = 0; jr < JR; ++jr) {
          const int c = 16 * JQ + 4 * jr + q4;
          if (c < k) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = 16 * tv + 4 * cs + r;
              if (row < d0) out[(int64_t)row * k + c] = accr[G][jr][r];
            }
          }
        }
      }
    }
  }
}

// Tile slots per wave: the smallest instance (2, 4, 6 or 8) covering
// the tiles of [A_0 | A_1].
static int dma_slots(int d0, int d1) {
  const int TT = (d0 + 15) / 16 + (d1 > 0 ? (d1 + 15) / 16 : 0);
  const int need = (TT + kF32Waves - 1) / kF32Waves;
  return need <= 2 ? 2 : need <= 4 ? 4 : need <= 6 ? 6 : 8;
}

static size_t dma_lds_bytes(int d0, int d1, int NT) {
  const size_t pitch = (size_t)dma_pitch(kF32Waves * dma_slots(d0, d1));
  return (2 * kDmaRows * pitch + (size_t)kF32Waves * 256 + (size_t)NT * kDmaRows * 17) * sizeof(float);
}

// 16-byte loads need rows that start on 16-byte boundaries and blocks of
// at least 16 tiles (one 256-float chunk); 4-byte loads blocks of 4 tiles.
static int dma_vec(const void* A0, const void* A1, int d0, int d1) {
  const int T0 = (d0 + 15) / 16, T1 = A1 ? (d1 + 15) / 16 : 0;
  const bool al = ((uintptr_t)A0 % 16 == 0) && (!A1 || (uintptr_t)A1 % 16 == 0) && d0 % 4 == 0 && (!A1 || d1 % 4 == 0);
  if (al && T0 >= 16 && (!A1 || T1 >= 16)) return 4;
  if (T0 >= 4 && (!A1 || T1 >= 4)) return 1;
  return 0;
}

static bool dma_fits(int d0, int d1, int k, int nb, int vec) {
  if (vec == 0) return false;
  if (k > 16) return false;   // two k-tiles would not fit the registers
  const int TT = (d0 + 15) / 16 + (nb == 2 ? (d1 + 15) / 16 : 0);
  if (TT > kDmaMaxTiles) return false;
  const int NT = nb * ((k + 15) / 16);
  return dma_lds_bytes(d0, nb == 2 ? d1 : 0, NT) <= (size_t)kPassLds + 8 * 1024;
}

template <class CT> static size_t pass_lds_bytes(int D, int NT) {
  return ((size_t)16 * pass_pitch(D) + (size_t)kPassWaves * NT * 256 + (size_t)NT * 272) * sizeof(CT);
}

// Counter that the pass reductions of the current gram_pass_run call on
// this host thread bump (null: none).  Set for the length of one call.
static thread_local int* t_pass_ran = nullptr;

// J_b[c][j] = sum over partials, in a fixed order: each of 4 thread groups
// sums a contiguous quarter of the partials, then the quarters are added.
// A pass that ran (no done flag set) also counts itself in *ran when given.
template <class CT>
__global__ void __launch_bounds__(256) k_pass_reduce(const CT* __restrict__ partial, int nparts, int d0, int d1,
                                                     int W_out, double* __restrict__ J0, double* __restrict__ J1,
                                                     const int* __restrict__ done, int* __restrict__ ran) {
  if (done && *done) return;
  if (ran && blockIdx.x == 0 && threadIdx.x == 0) ++*ran;
  __shared__ double q4[4][64];
  const int64_t Dtot = d0 + d1;
  const int64_t count = Dtot * W_out;
  const int grp = threadIdx.x >> 6, lanei = threadIdx.x & 63;
  const int64_t i = blockIdx.x * 64ll + lanei;
  const int per = (nparts + 3) / 4;
  const int z0 = grp * per, z1 = min(nparts, z0 + per);
  double v = 0.0;
  if (i < count) {
    // loads in batches of 16 (all in flight together), added in z order
    int z = z0;
    for (; z + 16 <= z1; z += 16) {
      CT t[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) t[u] = partial[(int64_t)(z + u) * count + i];
#pragma unroll
      for (int u = 0; u < 16; ++u) v += (double)t[u];
    }
    for (; z < z1; ++z) v += (double)partial[(int64_t)z * count + i];
  }
  q4[grp][lanei] = v;
  __syncthreads();
  if (grp == 0 && i < count) {
    const double tot = ((q4[0][lanei] + q4[1][lanei]) + q4[2][lanei]) + q4[3][lanei];
    const int64_t row = i / W_out, col = i % W_out;
    if (row < d0) J0[row * W_out + col] = tot;
    else J1[(row - d0) * W_out + col] = tot;
  }
}

// ------------------------------------------------------------------
// BF16 data with BF16 matrix-core products (FP32 accumulation): the
// low-precision form of the pass.  Same streaming scheme as the FP32 DMA
// pass (double-buffered global-to-LDS row blocks, direction operands in
// registers, one workgroup owns whole rows), with 16-row blocks:
//   (b) P_b = A_b W_b on 16x16x32 BF16 MFMA over 32-column tiles (A_1's
//       tiles start on a 32-column boundary, so no tile mixes the blocks;
//       the pad columns are zero in LDS and in the packed direction);
//   (c) the wave partials of P are summed in FP32 and rounded to BF16,
//       stored pcol-major so a lane's four rows are one 8-byte read;
//   (d) A_b^T [P_0 | P_1] on 16x16x16 BF16 MFMA, the 16 rows of the block
//       as the contraction.
constexpr int kBfRows = 16;
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef short s16x4_t __attribute__((ext_vector_type(4)));

struct BfGeom {
  int T0, T1, T0p, T1p, TTp, pitch;   // pitch in bf16 elements
};
__host__ __device__ inline BfGeom bf_geom(int d0, int d1) {
  BfGeom g;
  g.T0 = (d0 + 15) / 16;
  g.T1 = (d1 + 15) / 16;
  g.T0p = (g.T0 + 1) & ~1;
  g.T1p = (g.T1 + 1) & ~1;
  g.TTp = g.T0p + g.T1p;
  g.pitch = g.TTp * 16 + 8;
  return g;
}

template <int VEC>
__device__ __forceinline__ void dma_row_chunk_bf(__amdgpu_buffer_rsrc_t r, unsigned short* lds_dst, int voff) {
  if constexpr (VEC == 8)
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (__attribute__((address_space(3))) void*)lds_dst, 16, voff, 0, 0, 0);
  else
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (__attribute__((address_space(3))) void*)lds_dst, 4, voff, 0, 0, 0);
}

// Pack double d x k directions into zero-padded (ceil32(d) x 16) BF16.
__global__ void k_pack_dir_bf(const double* __restrict__ W0, int d0, int dp0, unsigned short* __restrict__ Wp0,
                              const double* __restrict__ W1, int d1, int dp1, unsigned short* __restrict__ Wp1,
                              int k) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n0 = dp0 * 16;
  const double* W = W0;
  unsigned short* Wp = Wp0;
  int d = d0;
  if (i >= n0) {
    i -= n0;
    if (i >= dp1 * 16) return;
    W = W1; Wp = Wp1; d = d1;
  }
  const int r = i >> 4, c = i & 15;
  const float v = (r < d && c < k) ? (float)W[(int64_t)r * k + c] : 0.0f;
  Wp[i] = bf16_rne_bits(v);
}

// Per-block work of k_pass_bf; the LDS regions arrive as separate restrict
// pointers so that the reads of the current block, the partials and P carry
// alias scopes disjoint from the next block's in-flight DMA (see quad_step).
template <int NB, int VEC>
__device__ __forceinline__ void bf_step(const unsigned short* __restrict__ xs, unsigned short* __restrict__ xnext,
                                        float* __restrict__ red, unsigned short* __restrict__ pb, int next_rb,
                                        const unsigned short* A0, const unsigned short* A1, int64_t n, int d0,
                                        int d1, const BfGeom& G, int nch0, int nch, int w, int lane,
                                        const bf16x8_t (&wreg)[(kDmaMaxTiles / 2 + kDmaWaves - 1) / kDmaWaves],
                                        f32x4 (&acc)[(kDmaMaxTiles + kDmaWaves - 1) / kDmaWaves][NB], bool dma_only) {
  constexpr int R = kBfRows;
  constexpr int CH = 64 * VEC;
  constexpr int NT = NB;
  constexpr int TPB32 = (kDmaMaxTiles / 2 + kDmaWaves - 1) / kDmaWaves;
  constexpr int TPB = (kDmaMaxTiles + kDmaWaves - 1) / kDmaWaves;
  const int tid = threadIdx.x;
  const int g = lane >> 4, l16 = lane & 15;
  const int pitch = G.pitch;
  if (next_rb >= 0) {
    const int nq = R * nch;
    for (int q = w; q < nq; q += kDmaWaves) {
      const int r = q / nch, j = q - r * nch;
      const int64_t row = (int64_t)next_rb * R + r;
      const bool s1 = (NB == 2) && (j >= nch0);
      const int jj = s1 ? j - nch0 : j;
      const int span = (s1 ? G.T1 : G.T0) * 16;
      const int o = min(jj * CH, span - CH);
      unsigned short* dst = xnext + r * pitch + (s1 ? G.T0p * 16 : 0) + o;
      const int voff = (o + lane * VEC) * 2;
      if (s1) dma_row_chunk_bf<VEC>(make_rsrc(A1 + row * d1, row < n ? (int64_t)d1 * 2 : 0), dst, voff);
      else dma_row_chunk_bf<VEC>(make_rsrc(A0 + row * d0, row < n ? (int64_t)d0 * 2 : 0), dst, voff);
    }
  }
  if (dma_only) return;
  const int base_b = l16 * pitch + 8 * g + 32 * w;    // P phase: row l16, columns 32 T + 8 g .. + 7
  const int base_d = (4 * g) * pitch + l16 + 16 * w;  // J phase: rows 4 g .. 4 g + 3, column 16 t + l16
  // (b)
  f32x4 pacc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) pacc[b] = f32x4{0, 0, 0, 0};
#pragma unroll
  for (int i = 0; i < TPB32; ++i) {
    const int T = w + kDmaWaves * i;
    if (2 * T < G.TTp) {
      const bf16x8_t a = *reinterpret_cast<const bf16x8_t*>(xs + base_b + 32 * kDmaWaves * i);
      if (NB == 2 && 2 * T >= G.T0p) pacc[NB - 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, wreg[i], pacc[NB - 1], 0, 0, 0);
      else pacc[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, wreg[i], pacc[0], 0, 0, 0);
    }
  }
  // (c)
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) red[(w * NT + b) * 256 + (4 * g + r) * 16 + l16] = pacc[b][r];
  lds_only_barrier();
  for (int e = tid; e < NT * 256; e += kDmaThreads) {
    const int nt = e >> 8, q = e & 255;   // q = row * 16 + pcol
    float v = 0.f;
#pragma unroll
    for (int ww = 0; ww < kDmaWaves; ++ww) v += red[(ww * NT + nt) * 256 + q];
    pb[nt * 256 + (q & 15) * 16 + (q >> 4)] = bf16_rne_bits(v);
  }
  lds_only_barrier();
  // (d)
  s16x4_t bop[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) bop[nt] = *reinterpret_cast<const s16x4_t*>(pb + nt * 256 + l16 * 16 + 4 * g);
#pragma unroll
  for (int i = 0; i < TPB; ++i) {
    const int t = w + kDmaWaves * i;
    if (t < G.TTp) {
      const unsigned short* xp = xs + base_d + 16 * kDmaWaves * i;
      s16x4_t a;
      a[0] = (short)xp[0];
      a[1] = (short)xp[pitch];
      a[2] = (short)xp[2 * pitch];
      a[3] = (short)xp[3 * pitch];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[i][nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bop[nt], acc[i][nt], 0, 0, 0);
    }
  }
}

template <int NB, int VEC>
__global__ void __launch_bounds__(kDmaThreads) k_pass_bf(const unsigned short* __restrict__ A0,
                                                         const unsigned short* __restrict__ A1, int64_t n, int d0,
                                                         int d1, int k, const unsigned short* __restrict__ Wp0,
                                                         const unsigned short* __restrict__ Wp1, int nrb,
                                                         float* __restrict__ partial, const int* __restrict__ done) {
  if (done && *done) return;
  constexpr int R = kBfRows;
  constexpr int CH = 64 * VEC;          // bf16 elements per load instruction
  constexpr int NT = NB;                // k <= 16: one k-tile per block
  constexpr int TPB32 = (kDmaMaxTiles / 2 + kDmaWaves - 1) / kDmaWaves;   // 32-column P tiles per wave
  constexpr int TPB = (kDmaMaxTiles + kDmaWaves - 1) / kDmaWaves;         // 16-column J tiles per wave
  extern __shared__ unsigned short bsm[];
  const BfGeom G = bf_geom(d0, NB == 2 ? d1 : 0);
  const int pitch = G.pitch;
  unsigned short* xsb0 = bsm;
  float* red = reinterpret_cast<float*>(bsm + 2 * R * pitch);          // [waves][NT][256]
  unsigned short* pb = reinterpret_cast<unsigned short*>(red + kDmaWaves * NT * 256);   // [NT][16 pcol][16 row]

  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, l16 = lane & 15;
  const int nch0 = (G.T0 * 16 + CH - 1) / CH, nch1 = NB == 2 ? (G.T1 * 16 + CH - 1) / CH : 0;
  const int nch = nch0 + nch1;

  // zero the pad columns of both buffers once (no load ever writes them)
  for (int e = tid; e < 2 * R * (G.TTp * 16); e += kDmaThreads) {
    const int rr = e / (G.TTp * 16), c = e - rr * (G.TTp * 16);
    const bool pad = (c >= G.T0 * 16 && c < G.T0p * 16) || (c >= G.T0p * 16 + G.T1 * 16);
    if (pad) xsb0[rr * pitch + c] = 0;
  }
  // direction operands: 32-column tile T = w + 8 i, lane (l16, g) holds
  // W[32 T + 8 g + e][l16] for e < 8 (A_1's rows start at T0p / 2)
  bf16x8_t wreg[TPB32];
#pragma unroll
  for (int i = 0; i < TPB32; ++i) {
    const int T = w + kDmaWaves * i;
    const bool b1 = (NB == 2) && (2 * T >= G.T0p);
    const int rowb = b1 ? 32 * T - 16 * G.T0p : 32 * T;
    const unsigned short* Wp = b1 ? Wp1 : Wp0;
    const int lim = b1 ? G.T1p * 16 : G.T0p * 16;
    bf16x8_t v;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int r = rowb + 8 * g + e;
      const unsigned short bits = (2 * T < G.TTp && r < lim) ? Wp[r * 16 + l16] : (unsigned short)0;
      v[e] = __builtin_bit_cast(__bf16, bits);
    }
    wreg[i] = v;
  }
  f32x4 acc[TPB][NT];
#pragma unroll
  for (int i = 0; i < TPB; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[i][j] = f32x4{0, 0, 0, 0};

  int rb = blockIdx.x;
  int boff = 0;
  if (rb < nrb)
    bf_step<NB, VEC>(bsm + R * pitch, bsm, red, pb, rb, A0, A1, n, d0, d1, G, nch0, nch, w, lane, wreg, acc, true);
  for (; rb < nrb; rb += gridDim.x) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    const int nxt = rb + (int)gridDim.x < nrb ? rb + (int)gridDim.x : -1;
    bf_step<NB, VEC>(bsm + boff, bsm + (R * pitch - boff), red, pb, nxt, A0, A1, n, d0, d1, G, nch0, nch, w, lane,
                     wreg, acc, false);
    boff = R * pitch - boff;
  }
  // epilogue: tile t of the padded space -> block and tile, pads skipped
  const int W_out = NB * k;
  const int D = d0 + (NB == 2 ? d1 : 0);
  float* out = partial + (int64_t)blockIdx.x * D * W_out;
#pragma unroll
  for (int i = 0; i < TPB; ++i) {
    const int t = w + kDmaWaves * i;
    if (t < G.TTp) {
      bool b1 = false, ok = true;
      int ct = t;
      if (t >= G.T0) {
        if (NB == 2 && t >= G.T0p && t < G.T0p + G.T1) { b1 = true; ct = t - G.T0p; }
        else ok = false;
      }
      if (ok) {
        const int db = b1 ? d1 : d0;
        const int rowbase = b1 ? d0 : 0;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const int col = l16;
          if (col < k) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int c = ct * 16 + acc_row<float>(lane, r);
              if (c < db) out[(int64_t)(rowbase + c) * W_out + nt * k + col] = acc[i][nt][r];
            }
          }
        }
      }
    }
  }
}

static size_t bf_lds_bytes(int d0, int d1, int NT) {
  const BfGeom G = bf_geom(d0, d1);
  return (size_t)2 * kBfRows * G.pitch * 2 + (size_t)kDmaWaves * NT * 256 * 4 + (size_t)NT * 256 * 2;
}

static int bf_vec(const void* A0, const void* A1, int d0, int d1) {
  const int T0 = (d0 + 15) / 16, T1 = A1 ? (d1 + 15) / 16 : 0;
  const bool al16 = ((uintptr_t)A0 % 16 == 0) && (!A1 || (uintptr_t)A1 % 16 == 0) && d0 % 8 == 0 &&
                    (!A1 || d1 % 8 == 0);
  if (al16 && T0 * 16 >= 512 && (!A1 || T1 * 16 >= 512)) return 8;
  const bool al4 = ((uintptr_t)A0 % 4 == 0) && (!A1 || (uintptr_t)A1 % 4 == 0) && d0 % 2 == 0 && (!A1 || d1 % 2 == 0);
  if (al4 && T0 * 16 >= 128 && (!A1 || T1 * 16 >= 128)) return 2;
  return 0;
}

static bool bf_fits(int d0, int d1, int k, int nb, int vec) {
  if (vec == 0 || k > 16) return false;
  const BfGeom G = bf_geom(d0, nb == 2 ? d1 : 0);
  if (G.TTp > kDmaMaxTiles) return false;
  return bf_lds_bytes(d0, nb == 2 ? d1 : 0, nb) <= (size_t)kPassLds + 8 * 1024;
}

template <int NB, int VEC>
static int pass_launch_bf(const unsigned short* A0, const unsigned short* A1, int64_t n, int d0, int d1, int k,
                          const double* W0, const double* W1, double* J0, double* J1, const int* done, Arena& ws,
                          hipStream_t st, hipEvent_t before_pass, hipEvent_t after_pass) {
  const BfGeom G = bf_geom(d0, NB == 2 ? d1 : 0);
  const int dp0 = G.T0p * 16, dp1 = NB == 2 ? G.T1p * 16 : 0;
  unsigned short* Wp0 = ws.take<unsigned short>((size_t)dp0 * 16);
  unsigned short* Wp1 = NB == 2 ? ws.take<unsigned short>((size_t)dp1 * 16) : nullptr;
  const int nrb = (int)((n + kBfRows - 1) / kBfRows);
  const int grid = std::max(1, std::min(num_cus(), (nrb + 3) / 4));
  const int Dtot = d0 + (NB == 2 ? d1 : 0);
  float* part = ws.take<float>((size_t)grid * Dtot * NB * k);
  if (!Wp0 || !part || (NB == 2 && !Wp1)) { set_error("gram_pass: workspace too small"); return SRP_ENOMEM; }
  const int tot = dp0 * 16 + dp1 * 16;
  hipLaunchKernelGGL(k_pack_dir_bf, dim3((tot + 255) / 256), dim3(256), 0, st, W0, d0, dp0, Wp0, W1, d1, dp1, Wp1,
                     k);
  SRP_LAUNCH_CHECK();
  const size_t lds = bf_lds_bytes(d0, NB == 2 ? d1 : 0, NB);
  SRP_TRY(allow_dynamic_lds((const void*)k_pass_bf<NB, VEC>, kPassLds + 8 * 1024));
  if (before_pass) SRP_HIP(hipEventRecord(before_pass, st));
  hipLaunchKernelGGL((k_pass_bf<NB, VEC>), dim3(grid), dim3(kDmaThreads), lds, st, A0, A1, n, d0, NB == 2 ? d1 : 0,
                     k, Wp0, Wp1, nrb, part, done);
  SRP_LAUNCH_CHECK();
  if (after_pass) SRP_HIP(hipEventRecord(after_pass, st));
  const int64_t count = (int64_t)Dtot * NB * k;
  hipLaunchKernelGGL((k_pass_reduce<float>), dim3((unsigned)((count + 63) / 64)), dim3(256), 0, st, part, grid, d0,
                     NB == 2 ? d1 : 0, NB * k, J0, J1, done, t_pass_ran);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

static int pass_dispatch_bf(const unsigned short* A0, const unsigned short* A1, int64_t n, int d0, int d1, int k,
                            const double* W0, const double* W1, double* J0, double* J1, const int* done, Arena& ws,
                            hipStream_t st, hipEvent_t ev0, hipEvent_t ev) {
  const int vec = bf_vec(A0, A1, d0, d1);
  if (A1) {
    if (vec == 8) return pass_launch_bf<2, 8>(A0, A1, n, d0, d1, k, W0, W1, J0, J1, done, ws, st, ev0, ev);
    return pass_launch_bf<2, 2>(A0, A1, n, d0, d1, k, W0, W1, J0, J1, done, ws, st, ev0, ev);
  }
  if (vec == 8) return pass_launch_bf<1, 8>(A0, A1, n, d0, 0, k, W0, W1, J0, J1, done, ws, st, ev0, ev);
  return pass_launch_bf<1, 2>(A0, A1, n, d0, 0, k, W0, W1, J0, J1, done, ws, st, ev0, ev);
}

int pass_limits_ok(int dtype, int compute, int d0, int d1, int k, int nblocks) {
  if (compute == SRP_BF16) {
    if (dtype != SRP_BF16 || k > 16) return 0;
    const BfGeom G = bf_geom(d0, nblocks == 2 ? d1 : 0);
    if (G.TTp <= kDmaMaxTiles && bf_lds_bytes(d0, nblocks == 2 ? d1 : 0, nblocks) <= (size_t)kPassLds + 8 * 1024)
      return 1;
    return pass_limits_ok(SRP_BF16, SRP_F32, d0, d1, k, nblocks);   // the FP32-arithmetic pass takes it
  }
  const int D = d0 + (nblocks == 2 ? d1 : 0);
  const bool f64 = (compute == SRP_F64);
  if (dtype == SRP_F64 && !f64) return 0;
  if (nblocks == 2 && k > 16) return 0;
  if (nblocks == 1 && k > 32) return 0;
  const int NT = nblocks * ((k + 15) / 16);
  if (f64) {
    if (D > PassCfg<double>::dmax || pass_lds_bytes<double>(D, NT) > (size_t)kPassLds) return 0;
  } else {
    if (D > PassCfg<float>::dmax || pass_lds_bytes<float>(D, NT) > (size_t)kPassLds) return 0;
  }
  return 1;
}

// Number of row groups (each served by kPassSplit workgroups); a multiple
// of the XCD count so that the pair of a group shares an XCD.
static int pass_groups(int64_t n) {
  const int64_t nrb = (n + 15) / 16;
  int64_t g = num_cus() / kPassSplit;
  if (g > nrb) g = nrb;
  g = ((g + kXcds - 1) / kXcds) * kXcds;
  if (g < kXcds) g = kXcds;
  return (int)g;
}

size_t pass_ws_bytes(int64_t n, int d0, int d1, int k, int compute) {
  const size_t cs = compute == SRP_F64 ? 8 : 4;
  const int KT = (k + 15) / 16;
  const int nb = d1 > 0 ? 2 : 1;
  const size_t D = (size_t)d0 + (nb == 2 ? d1 : 0);
  const size_t wp = (((size_t)(d0 + 15) / 16 * 16) + ((size_t)(d1 + 15) / 16 * 16)) * KT * 16 * cs;
  const size_t slots = std::max<size_t>((size_t)pass_groups(n) * kPassSplit, (size_t)num_cus());
  return ((wp + 1023) & ~size_t(255)) + ((slots * D * nb * k * cs + 255) & ~size_t(255));
}

template <class DT, class CT, int NB, int KT>
static int pass_launch(const DT* A0, const DT* A1, int64_t n, int d0, int d1, int k, const double* W0,
                       const double* W1, double* J0, double* J1, const int* done, Arena& ws, hipStream_t st,
                       hipEvent_t before_pass, hipEvent_t after_pass) {
  const int dp0 = (d0 + 15) / 16 * 16, dp1 = NB == 2 ? (d1 + 15) / 16 * 16 : 0;
  const int KP = KT * 16;
  CT* Wp0 = ws.take<CT>((size_t)dp0 * KP);
  CT* Wp1 = NB == 2 ? ws.take<CT>((size_t)dp1 * KP) : nullptr;
  const int groups = pass_groups(n);
  const int grid = groups * kPassSplit;
  const int Dtot = d0 + (NB == 2 ? d1 : 0);
  CT* part = ws.take<CT>((size_t)groups * Dtot * NB * k);
  if (!Wp0 || !part || (NB == 2 && !Wp1)) { set_error("gram_pass: workspace too small"); return SRP_ENOMEM; }
  SRP_TRY(pack_dirs<CT>(W0, d0, dp0, Wp0, W1, d1, dp1, Wp1, k, KP, st));
  const int nrb = (int)((n + 15) / 16);
  const size_t lds = pass_lds_bytes<CT>(Dtot, NB * KT);
  SRP_TRY(allow_dynamic_lds((const void*)k_pass<DT, CT, NB, KT>, kPassLds));
  if (before_pass) SRP_HIP(hipEventRecord(before_pass, st));
  hipLaunchKernelGGL((k_pass<DT, CT, NB, KT>), dim3(grid), dim3(kPassThreads), lds, st, A0, A1, n, d0,
                     NB == 2 ? d1 : 0, k, Wp0, Wp1, nrb, part, done);
  SRP_LAUNCH_CHECK();
  if (after_pass) SRP_HIP(hipEventRecord(after_pass, st));
  const int64_t count = (int64_t)Dtot * NB * k;
  hipLaunchKernelGGL((k_pass_reduce<CT>), dim3((unsigned)((count + 63) / 64)), dim3(256), 0, st, part, groups, d0,
                     NB == 2 ? d1 : 0, NB * k, J0, J1, done, t_pass_ran);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

template <int NB, int TPB, int VEC>
static int pass_launch_dma(const float* A0, const float* A1, int64_t n, int d0, int d1, int k, const double* W0,
                           const double* W1, double* J0, double* J1, const int* done, Arena& ws, hipStream_t st,
                           hipEvent_t before_pass, hipEvent_t after_pass) {
  const int dp0 = (d0 + 15) / 16 * 16, dp1 = NB == 2 ? (d1 + 15) / 16 * 16 : 0;
  const int KP = 16;
  float* Wp0 = ws.take<float>((size_t)dp0 * KP);
  float* Wp1 = NB == 2 ? ws.take<float>((size_t)dp1 * KP) : nullptr;
  const int nrb = (int)((n + kDmaRows - 1) / kDmaRows);
  // at least 4 blocks per workgroup (fewer partials to add for short data)
  const int grid = std::max(1, std::min(num_cus(), (nrb + 3) / 4));
  const int Dtot = d0 + (NB == 2 ? d1 : 0);
  float* part = ws.take<float>((size_t)grid * Dtot * NB * k);
  if (!Wp0 || !part || (NB == 2 && !Wp1)) { set_error("gram_pass: workspace too small"); return SRP_ENOMEM; }
  SRP_TRY(pack_dirs<float>(W0, d0, dp0, Wp0, W1, d1, dp1, Wp1, k, KP, st));
  const size_t lds = dma_lds_bytes(d0, NB == 2 ? d1 : 0, NB);
  SRP_TRY(allow_dynamic_lds((const void*)k_pass_dma<NB, TPB, VEC>, kPassLds + 8 * 1024));
  if (before_pass) SRP_HIP(hipEventRecord(before_pass, st));
  hipLaunchKernelGGL((k_pass_dma<NB, TPB, VEC>), dim3(grid), dim3(kF32Threads), lds, st, A0, A1, n, d0,
                     NB == 2 ? d1 : 0, k, Wp0, Wp1, nrb, part, done);
  SRP_LAUNCH_CHECK();
  if (after_pass) SRP_HIP(hipEventRecord(after_pass, st));
  const int64_t count = (int64_t)Dtot * NB * k;
  hipLaunchKernelGGL((k_pass_reduce<float>), dim3((unsigned)((count + 63) / 64)), dim3(256), 0, st, part, grid, d0,
                     NB == 2 ? d1 : 0, NB * k, J0, J1, done, t_pass_ran);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

static int pass_dispatch_dma(const float* A0, const float* A1, int64_t n, int d0, int d1, int k, const double* W0,
                             const double* W1, double* J0, double* J1, const int* done, Arena& ws, hipStream_t st,
                             hipEvent_t ev0, hipEvent_t ev) {
  const int vec = dma_vec(A0, A1, d0, d1);
  const int slots = dma_slots(d0, A1 ? d1 : 0);
#define SRP_DMA_CASE(NB_, TPB_)                                                                             \
  if (slots == TPB_)                                                                                        \
    return vec == 4 ? pass_launch_dma<NB_, TPB_, 4>(A0, A1, n, d0, d1, k, W0, W1, J0, J1, done, ws, st, ev0, ev) \
                    : pass_launch_dma<NB_, TPB_, 1>(A0, A1, n, d0, d1, k, W0, W1, J0, J1, done, ws, st, ev0, ev);
  if (A1) {
    SRP_DMA_CASE(2, 2) SRP_DMA_CASE(2, 4) SRP_DMA_CASE(2, 6) SRP_DMA_CASE(2, 8)
  } else {
    d1 = 0;
    SRP_DMA_CASE(1, 2) SRP_DMA_CASE(1, 4) SRP_DMA_CASE(1, 6) SRP_DMA_CASE(1, 8)
  }
#undef SRP_DMA_CASE
  set_error("gram_pass: no DMA pass instance for %d tile slots", slots);
  return SRP_EINVAL;
}

// The 4x4-block pass: two views, each of at most 64 tiles (1024 columns);
// SV = 2 tile slots per view and wave up to 32 tiles, else 4.  k <= 10
// with 4 slots (beyond that the registers no longer hold the accumulators
// and operands of a block without spilling inside the row loop), k <= 16
// with 2.
static int quad_sv(int d0, int d1) {
  const int tmax = std::max((d0 + 15) / 16, (d1 + 15) / 16);
  return tmax <= 32 ? 2 : tmax <= 64 ? 4 : 0;
}

static size_t quad_lds_bytes(int sv, int c4) {
  const size_t pitch = (size_t)quad_pitch(2 * sv);
  const size_t kg = (size_t)(c4 + 1) / 2;
  return (2 * kDmaRows * pitch + (size_t)kF32Waves * (kDmaRows * 4 * kg + 8) + (size_t)kDmaRows * (4 * c4 + 1)) *
         sizeof(float);
}

static bool quad_fits(int d0, int d1, int k, int nb, int vec) {
  if (nb != 2 || vec == 0 || k < 1) return false;
  const int sv = quad_sv(d0, d1);
  const int c4 = (k + 1) / 2;
  if (sv == 0 || c4 > (sv == 4 ? 5 : 8)) return false;
  return quad_lds_bytes(sv, c4) <= (size_t)kPassLds + 8 * 1024;
}

template <int SV, int C4, int VEC>
static int pass_launch_quad(const float* A0, const float* A1, int64_t n, int d0, int d1, int k, const double* W0,
                            const double* W1, double* J0, double* J1, const int* done, Arena& ws, hipStream_t st,
                            hipEvent_t before_pass, hipEvent_t after_pass) {
  const int nrb = (int)((n + kDmaRows - 1) / kDmaRows);
  // at least 4 blocks per workgroup (fewer partials to add for short data)
  const int grid = std::max(1, std::min(num_cus(), (nrb + 3) / 4));
  const int Dtot = d0 + d1;
  float* part = ws.take<float>((size_t)grid * Dtot * 2 * k);
  if (!part) { set_error("gram_pass: workspace too small"); return SRP_ENOMEM; }
  if ((int64_t)std::max(d0, d1) * k * 8 >= 0x7ffff000ll) { set_error("gram_pass: directions too large"); return SRP_EINVAL; }
  const size_t lds = quad_lds_bytes(SV, C4);
  SRP_TRY(allow_dynamic_lds((const void*)k_pass_quad<SV, C4, VEC>, kPassLds + 8 * 1024));
  if (before_pass) SRP_HIP(hipEventRecord(before_pass, st));
  hipLaunchKernelGGL((k_pass_quad<SV, C4, VEC>), dim3(grid), dim3(kF32Threads), lds, st, A0, A1, n, d0, d1, k, W0,
                     W1, nrb, part, done);
  SRP_LAUNCH_CHECK();
  if (after_pass) SRP_HIP(hipEventRecord(after_pass, st));
  const int64_t count = (int64_t)Dtot * 2 * k;
  hipLaunchKernelGGL((k_pass_reduce<float>), dim3((unsigned)((count + 63) / 64)), dim3(256), 0, st, part, grid, d0,
                     d1, 2 * k, J0, J1, done, t_pass_ran);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

static int pass_dispatch_quad(const float* A0, const float* A1, int64_t n, int d0, int d1, int k, const double* W0,
                              const double* W1, double* J0, double* J1, const int* done, Arena& ws, hipStream_t st,
                              hipEvent_t ev0, hipEvent_t ev) {
  const int vec = dma_vec(A0, A1, d0, d1);
  const int sv = quad_sv(d0, d1);
  const int c4 = (k + 1) / 2;
#define SRP_QUAD_CASE(SV_, C4_)                                                                                     \
  if (sv == SV_ && c4 == C4_)                                                                                       \
    return vec == 4 ? pass_launch_quad<SV_, C4_, 4>(A0, A1, n, d0, d1, k, W0, W1, J0, J1, done, ws, st, ev0, ev) \
                    : pass_launch_quad<SV_, C4_, 1>(A0, A1, n, d0, d1, k, W0, W1, J0, J1, done, ws, st, ev0, ev);
  SRP_QUAD_CASE(2, 1) SRP_QUAD_CASE(2, 2) SRP_QUAD_CASE(2, 3) SRP_QUAD_CASE(2, 4)
  SRP_QUAD_CASE(2, 5) SRP_QUAD_CASE(2, 6) SRP_QUAD_CASE(2, 7) SRP_QUAD_CASE(2, 8)
  SRP_QUAD_CASE(4, 1) SRP_QUAD_CASE(4, 2) SRP_QUAD_CASE(4, 3) SRP_QUAD_CASE(4, 4)
  SRP_QUAD_CASE(4, 5)
#undef SRP_QUAD_CASE
  set_error("gram_pass: no 4x4-block pass instance for %d slots, k = %d", sv, k);
  return SRP_EINVAL;
}

// The one-view 4x4-block pass: k <= 20, at most 128 tiles (2048 columns);
// 4 J slots per wave up to 64 tiles, else 8.
static int quad1_tpb(int d0) {
  const int T0 = (d0 + 15) / 16;
  return T0 <= 64 ? 4 : T0 <= 128 ? 8 : 0;
}

static size_t quad1_lds_bytes(int tpb, int kg) {
  return (2 * kDmaRows * (size_t)quad_pitch(tpb) + (size_t)kF32Waves * (kDmaRows * 4 * kg + 4) +
          (size_t)kDmaRows * (4 * kg + 1)) * sizeof(float);
}

static bool quad1_fits(int d0, int k, int nb, int vec) {
  if (nb != 1 || vec == 0 || k < 1 || k > 20) return false;
  const int tpb = quad1_tpb(d0);
  if (tpb == 0) return false;
  return quad1_lds_bytes(tpb, (k + 3) / 4) <= (size_t)kPassLds + 8 * 1024;
}

template <int TPB, int KG, int VEC>
static int pass_launch_quad1(const float* A0, int64_t n, int d0, int k, const double* W0, double* J0,
                             const int* done, Arena& ws, hipStream_t st, hipEvent_t before_pass,
                             hipEvent_t after_pass) {
  const int dp0 = (d0 + 15) / 16 * 16;
  const int KP = 4 * KG;
  float* Wp0 = ws.take<float>((size_t)dp0 * KP);
  const int nrb = (int)((n + kDmaRows - 1) / kDmaRows);
  const int grid = std::max(1, std::min(num_cus(), (nrb + 3) / 4));
  float* part = ws.take<float>((size_t)grid * d0 * k);
  if (!Wp0 || !part) { set_error("gram_pass: workspace too small"); return SRP_ENOMEM; }
  SRP_TRY(pack_dirs<float>(W0, d0, dp0, Wp0, nullptr, 0, 0, nullptr, k, KP, st));
  const size_t lds = quad1_lds_bytes(TPB, KG);
  SRP_TRY(allow_dynamic_lds((const void*)k_pass_quad1<TPB, KG, VEC>, kPassLds + 8 * 1024));
  if (before_pass) SRP_HIP(hipEventRecord(before_pass, st));
  hipLaunchKernelGGL((k_pass_quad1<TPB, KG, VEC>), dim3(grid), dim3(kF32Threads), lds, st, A0, n, d0, k, Wp0, nrb,
                     part, done);
  SRP_LAUNCH_CHECK();
  if (after_pass) SRP_HIP(hipEventRecord(after_pass, st));
  const int64_t count = (int64_t)d0 * k;
  hipLaunchKernelGGL((k_pass_reduce<float>), dim3((unsigned)((count + 63) / 64)), dim3(256), 0, st, part, grid, d0,
                     0, k, J0, (double*)nullptr, done, t_pass_ran);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

static int pass_dispatch_quad1(const float* A0, int64_t n, int d0, int k, const double* W0, double* J0,
                               const int* done, Arena& ws, hipStream_t st, hipEvent_t ev0, hipEvent_t ev) {
  const int vec = dma_vec(A0, nullptr, d0, 0);
  const int tpb = quad1_tpb(d0);
  const int kg = (k + 3) / 4;
#define SRP_QUAD1_CASE(TPB_, KG_)                                                                              \
  if (tpb == TPB_ && kg == KG_)                                                                                \
    return vec == 4 ? pass_launch_quad1<TPB_, KG_, 4>(A0, n, d0, k, W0, J0, done, ws, st, ev0, ev)            \
                    : pass_launch_quad1<TPB_, KG_, 1>(A0, n, d0, k, W0, J0, done, ws, st, ev0, ev);
  SRP_QUAD1_CASE(4, 1) SRP_QUAD1_CASE(4, 2) SRP_QUAD1_CASE(4, 3) SRP_QUAD1_CASE(4, 4) SRP_QUAD1_CASE(4, 5)
  SRP_QUAD1_CASE(8, 1) SRP_QUAD1_CASE(8, 2) SRP_QUAD1_CASE(8, 3) SRP_QUAD1_CASE(8, 4) SRP_QUAD1_CASE(8, 5)
#undef SRP_QUAD1_CASE
  set_error("gram_pass: no one-view 4x4-block pass instance for %d slots, k = %d", tpb, k);
  return SRP_EINVAL;
}

template <class DT, class CT>
static int pass_dispatch_k(const DT* A0, const DT* A1, int64_t n, int d0, int d1, int k, const double* W0,
                           const double* W1, double* J0, double* J1, const int* done, Arena& ws, hipStream_t st,
                           hipEvent_t ev0, hipEvent_t ev) {
  if (A1) return pass_launch<DT, CT, 2, 1>(A0, A1, n, d0, d1, k, W0, W1, J0, J1, done, ws, st, ev0, ev);
  if (k <= 16) return pass_launch<DT, CT, 1, 1>(A0, A1, n, d0, 0, k, W0, W1, J0, J1, done, ws, st, ev0, ev);
  return pass_launch<DT, CT, 1, 2>(A0, A1, n, d0, 0, k, W0, W1, J0, J1, done, ws, st, ev0, ev);
}

// Name of the pass kernel gram_pass_run launches for a shape, for rows
// that start on 16-byte boundaries (the row alignment only changes the
// load width), or nullptr outside the limits.
const char* gram_pass_kernel_name(int dtype, int compute, int d0, int d1, int k) {
  const int nb = d1 > 0 ? 2 : 1;
  if (nb == 1) d1 = 0;
  if (!pass_limits_ok(dtype, compute, d0, d1, k, nb)) return nullptr;
  const int T0 = (d0 + 15) / 16, T1 = nb == 2 ? (d1 + 15) / 16 : 0;
  const bool al = d0 % 4 == 0 && (nb == 1 || d1 % 4 == 0);
  if (compute == SRP_BF16) {
    if (dtype != SRP_BF16) return nullptr;
    const int bvec = ((d0 * 2) % 4 == 0 && (nb == 1 || (d1 * 2) % 4 == 0)) ? 1 : 0;
    return bf_fits(d0, d1, k, nb, bvec ? 1 : 0) ? "k_pass_bf" : "k_pass";
  }
  if (compute == SRP_F32 && dtype == SRP_F32) {
    const int vec = (al && T0 >= 16 && (nb == 1 || T1 >= 16)) ? 4 : (T0 >= 4 && (nb == 1 || T1 >= 4)) ? 1 : 0;
    if (quad1_fits(d0, k, nb, vec)) return "k_pass_quad1";
    if (quad_fits(d0, d1, k, nb, vec)) return "k_pass_quad";
    if (dma_fits(d0, d1, k, nb, vec)) return "k_pass_dma";
  }
  return "k_pass";
}

int gram_pass_run(const void* A0, const void* A1, int dtype, int compute, int64_t n, int d0, int d1, int k,
                  const double* W0, const double* W1, double* J0, double* J1, const int* done, Arena& ws,
                  hipStream_t st, hipEvent_t before_pass, hipEvent_t after_pass, int* ran) {
  struct RanScope {
    explicit RanScope(int* r) { t_pass_ran = r; }
    ~RanScope() { t_pass_ran = nullptr; }
  } ran_scope(ran);
  const int nb = A1 ? 2 : 1;
  if (!pass_limits_ok(dtype, compute, d0, d1, k, nb)) {
    set_error("gram_pass: unsupported shape (d0=%d d1=%d k=%d dtype=%d compute=%d)", d0, d1, k, dtype, compute);
    return SRP_EINVAL;
  }
  if (compute == SRP_BF16) {   // BF16 matrix-core products: BF16 data only
    if (dtype != SRP_BF16) {
      set_error("gram_pass: BF16 products need BF16 data");
      return SRP_EINVAL;
    }
    if (bf_fits(d0, nb == 2 ? d1 : 0, k, nb, bf_vec(A0, A1, d0, d1)))
      return pass_dispatch_bf((const unsigned short*)A0, (const unsigned short*)A1, n, d0, d1, k, W0, W1, J0, J1,
                              done, ws, st, before_pass, after_pass);
    // views narrower than one 64-lane row chunk (or rows not 4-byte
    // aligned): the FP32-arithmetic pass reads the same BF16 data
    return pass_dispatch_k<bf16, float>((const bf16*)A0, (const bf16*)A1, n, d0, d1, k, W0, W1, J0, J1, done, ws, st,
                                        before_pass, after_pass);
  }
  if (compute == SRP_F64) {
    switch (dtype) {
      case SRP_F64: return pass_dispatch_k<double, double>((const double*)A0, (const double*)A1, n, d0, d1, k, W0, W1, J0, J1, done, ws, st, before_pass, after_pass);
      case SRP_F32: return pass_dispatch_k<float, double>((const float*)A0, (const float*)A1, n, d0, d1, k, W0, W1, J0, J1, done, ws, st, before_pass, after_pass);
      case SRP_BF16: return pass_dispatch_k<bf16, double>((const bf16*)A0, (const bf16*)A1, n, d0, d1, k, W0, W1, J0, J1, done, ws, st, before_pass, after_pass);
    }
  } else {
    switch (dtype) {
      case SRP_F32:
        if (quad1_fits(d0, k, nb, dma_vec(A0, A1, d0, d1)))
          return pass_dispatch_quad1((const float*)A0, n, d0, k, W0, J0, done, ws, st, before_pass, after_pass);
        if (quad_fits(d0, nb == 2 ? d1 : 0, k, nb, dma_vec(A0, A1, d0, d1)))
          return pass_dispatch_quad((const float*)A0, (const float*)A1, n, d0, d1, k, W0, W1, J0, J1, done, ws, st,
                                    before_pass, after_pass);
        if (dma_fits(d0, nb == 2 ? d1 : 0, k, nb, dma_vec(A0, A1, d0, d1)))
          return pass_dispatch_dma((const float*)A0, (const float*)A1, n, d0, d1, k, W0, W1, J0, J1, done, ws, st,
                                   before_pass, after_pass);
        return pass_dispatch_k<float, float>((const float*)A0, (const float*)A1, n, d0, d1, k, W0, W1, J0, J1, done, ws, st, before_pass, after_pass);
      case SRP_BF16: return pass_dispatch_k<bf16, float>((const bf16*)A0, (const bf16*)A1, n, d0, d1, k, W0, W1, J0, J1, done, ws, st, before_pass, after_pass);
    }
  }
  set_error("gram_pass: bad dtype/compute (%d/%d)", dtype, compute);
  return SRP_EINVAL;
}

}  // namespace srp
