// Sketching transforms on the GPU: CountSketch (Section 3) and the
// subsampled randomized Hadamard transform (Appendix A, Definition SRHT).
//
// CountSketch: (S A)_b = sum over rows i with h(i) = b of g(i) A_i.  Rows are
// bucketed by a counting sort (count, scan, fill), each bucket's row list is
// put in ascending order, and one workgroup per bucket streams its rows with
// coalesced row reads and sums them in that fixed order, so the result is
// bitwise reproducible.
//
// SRHT: S A = sqrt(n'/s) R H D [A; 0] with the normalised Hadamard matrix,
// i.e. (S A)_j = s^-1/2 sum_i (-1)^popcount(r_j & i) D_i A_i.  With
// n' = A_blocks * B and i = a B + b, r = alpha B + beta the sign factorises,
// so level 1 takes the length-B Walsh-Hadamard transform inside every block
// of B consecutive rows (in LDS), and level 2 forms each sampled output row
// as a +-sum over the blocks of level-1 row beta.  Only the s sampled rows
// are ever formed.  The row sample (s smallest SplitMix64 keys) is found by
// a 4-round 16-bit radix select and an order-preserving compaction.
#include "common.hpp"
#include "kernels.hpp"

#include <cmath>
#include <type_traits>

namespace srp {

// ------------------------------------------------------------ utilities
__global__ void k_fill_i32(int* p, int64_t count, int v) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

int fill_i32(int* p, int64_t count, int v, hipStream_t st) {
  if (count <= 0) return SRP_OK;
  int64_t blocks = (count + 255) / 256;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)blocks), dim3(256), 0, st, p, count, v);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

// Exclusive scan of `count` ints (single workgroup of 1024 threads).
// Writes offsets[0..count] (offsets[count] = total) and, if cursor != NULL,
// a copy of offsets[0..count) into cursor.
__global__ void __launch_bounds__(1024) k_scan_excl(const int* in, int count, int* offsets, int* cursor) {
  __shared__ int part[1024];
  const int t = threadIdx.x, T = blockDim.x;
  const int per = (count + T - 1) / T;
  const int b0 = min(count, t * per), b1 = min(count, b0 + per);
  int sum = 0;
  for (int b = b0; b < b1; ++b) sum += in[b];
  part[t] = sum;
  __syncthreads();
  for (int off = 1; off < T; off <<= 1) {
    int v = (t >= off) ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = (t == 0) ? 0 : part[t - 1];
  for (int b = b0; b < b1; ++b) {
    offsets[b] = run;
    if (cursor) cursor[b] = run;
    run += in[b];
  }
  if (t == T - 1) offsets[count] = part[T - 1];
}

// -------------------------------------------------------- CountSketch
__global__ void k_cs_count(int64_t n, int s, uint64_t seed, int* counts) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) atomicAdd(&counts[cs_bucket(splitmix64(seed, (uint64_t)i), s)], 1);
}

__global__ void k_cs_fill(int64_t n, int s, uint64_t seed, int* cursor, int* list) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) {
    int b = cs_bucket(splitmix64(seed, (uint64_t)i), s);
    int pos = atomicAdd(&cursor[b], 1);
    list[pos] = (int)i;
  }
}

// Rank sort of every bucket's rows into ascending order (rows are distinct).
__global__ void k_cs_sort(const int* offsets, const int* list, int* sorted) {
  const int b = blockIdx.x;
  const int beg = offsets[b], cnt = offsets[b + 1] - beg;
  for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
    const int v = list[beg + e];
    int r = 0;
    for (int j = 0; j < cnt; ++j) r += (list[beg + j] < v);
    sorted[beg + r] = v;
  }
}

// One workgroup per bucket; each thread owns up to CPT columns.  The
// bucket's row indices and signs are staged in LDS first, then the rows are
// read four at a time (all their loads in flight together) and added in
// ascending row order, one after the other.
template <class T, class Acc, int CPT>
__global__ void __launch_bounds__(256) k_cs_gather(const T* __restrict__ A, int d, uint64_t seed,
                                                   const int* __restrict__ offsets,
                                                   const int* __restrict__ sorted, Acc* __restrict__ out,
                                                   int col_base) {
  constexpr int RB = 4;
  __shared__ int rows_s[256];
  __shared__ Acc sgn_s[256];
  const int b = blockIdx.x;
  const int beg = offsets[b], cnt = offsets[b + 1] - beg;
  const int c0 = col_base + threadIdx.x;
  Acc acc[CPT];
#pragma unroll
  for (int j = 0; j < CPT; ++j) acc[j] = Acc(0);
  const int nt = blockDim.x;   // <= 256: one index per thread and chunk
  for (int base = 0; base < cnt; base += nt) {
    const int m = min(nt, cnt - base);
    __syncthreads();   // the previous chunk's indices are consumed
    if ((int)threadIdx.x < m) {
      const int row = sorted[beg + base + threadIdx.x];
      rows_s[threadIdx.x] = row;
      sgn_s[threadIdx.x] = (Acc)cs_sign(splitmix64(seed, (uint64_t)row));
    }
    __syncthreads();
    int e = 0;
    for (; e + RB <= m; e += RB) {
      Acc v[RB][CPT];
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const T* Ar = A + (int64_t)rows_s[e + r] * d;
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
          const int c = c0 + j * (int)blockDim.x;
          v[r][j] = c < d ? load_as<Acc>(Ar + c) : Acc(0);
        }
      }
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const Acc g = sgn_s[e + r];
#pragma unroll
        for (int j = 0; j < CPT; ++j) acc[j] += g * v[r][j];
      }
    }
    for (; e < m; ++e) {
      const Acc g = sgn_s[e];
      const T* Ar = A + (int64_t)rows_s[e] * d;
#pragma unroll
      for (int j = 0; j < CPT; ++j) {
        const int c = c0 + j * (int)blockDim.x;
        if (c < d) acc[j] += g * load_as<Acc>(Ar + c);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    const int c = c0 + j * (int)blockDim.x;
    if (c < d) out[(int64_t)b * d + c] = acc[j];
  }
}

size_t countsketch_ws_bytes(int64_t n, int s) {
  return 3 * bytes_of<int>(s + 1) + 2 * bytes_of<int>(n);
}

template <class T, class Acc>
static int cs_gather_launch(const T* A, int d, int s, uint64_t seed, const int* offsets,
                            const int* sorted, Acc* out, hipStream_t st) {
  const int threads = d >= 256 ? 256 : ((d + 63) / 64) * 64;
  constexpr int CPT = 8;
  for (int col = 0; col < d; col += threads * CPT) {
    hipLaunchKernelGGL((k_cs_gather<T, Acc, CPT>), dim3(s), dim3(threads), 0, st, A, d, seed,
                       offsets, sorted, out, col);
    SRP_LAUNCH_CHECK();
  }
  return SRP_OK;
}

int scan_excl_i32(const int* in, int count, int* offsets, hipStream_t st) {
  hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(1024), 0, st, in, count, offsets, (int*)nullptr);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

int countsketch_buckets(int64_t n, int s, uint64_t seed, Arena& ws, const int** offsets_out,
                        const int** sorted_out, hipStream_t st) {
  int* counts = ws.take<int>(s + 1);
  int* offsets = ws.take<int>(s + 1);
  int* cursor = ws.take<int>(s + 1);
  int* list = ws.take<int>(n);
  int* sorted = ws.take<int>(n);
  if (!sorted) { set_error("countsketch: workspace too small"); return SRP_ENOMEM; }
  SRP_TRY(fill_i32(counts, s, 0, st));
  const unsigned nb = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_cs_count, dim3(nb), dim3(256), 0, st, n, s, seed, counts);
  SRP_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(1024), 0, st, counts, s, offsets, cursor);
  SRP_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_cs_fill, dim3(nb), dim3(256), 0, st, n, s, seed, cursor, list);
  SRP_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_cs_sort, dim3(s), dim3(64), 0, st, offsets, list, sorted);
  SRP_LAUNCH_CHECK();
  *offsets_out = offsets;
  *sorted_out = sorted;
  return SRP_OK;
}

int countsketch_run(const void* A, int dtype, int64_t n, int d, int s, uint64_t seed, void* out,
                    Arena& ws, hipStream_t st) {
  const int* offsets = nullptr;
  const int* sorted = nullptr;
  SRP_TRY(countsketch_buckets(n, s, seed, ws, &offsets, &sorted, st));
  switch (dtype) {
    case SRP_F64:
      return cs_gather_launch((const double*)A, d, s, seed, offsets, sorted, (double*)out, st);
    case SRP_F32:
      return cs_gather_launch((const float*)A, d, s, seed, offsets, sorted, (float*)out, st);
    case SRP_BF16:
      return cs_gather_launch((const bf16*)A, d, s, seed, offsets, sorted, (float*)out, st);
    case SRP_FP8E4M3:
      return cs_gather_launch((const fp8e4m3*)A, d, s, seed, offsets, sorted, (float*)out, st);
  }
  set_error("countsketch: bad dtype %d", dtype);
  return SRP_EINVAL;
}

// --------------------------------------------------------------- SRHT
struct SelectState {
  uint64_t prefix;   // digits fixed so far (all 64 bits once done)
  int need;          // how many keys still to take at or below the prefix
  int done;          // the threshold is final: a whole bucket was taken
};

__global__ void k_sel_init(SelectState* st, int s) {
  st->prefix = 0;
  st->need = s;
  st->done = 0;
}

// Histogram of 16-bit digit `round` (0 = most significant) over keys whose
// higher digits equal the prefix found so far.
__global__ void k_sel_hist(int64_t n_pad, uint64_t seed, int round, const SelectState* st, int* hist) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n_pad || st->done) return;
  const uint64_t key = splitmix64(seed, (uint64_t)i);
  if (round > 0 && (key >> (64 - 16 * round)) != st->prefix) return;
  const int digit = (int)((key >> (48 - 16 * round)) & 0xFFFFull);
  atomicAdd(&hist[digit], 1);
}

// Find the digit holding the need-th smallest remaining key; zero hist.
// Thread t owns digits 64 t .. 64 t + 63 (sixteen 16-byte loads in flight),
// the counts are scanned by lane shuffles within a wave and the sixteen
// wave totals through LDS.  When the need-th key closes its bucket (the
// bucket is taken whole) the threshold is that bucket's prefix followed by
// all ones, the same key set as finishing the remaining rounds, and they
// are skipped.
__global__ void __launch_bounds__(1024) k_sel_pick(int* hist, SelectState* st, int round) {
  __shared__ int wsum[16];
  __shared__ int found_digit, found_before, found_count;
  if (st->done) return;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  int4* h4 = reinterpret_cast<int4*>(hist) + 16 * t;
  int4 v[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) v[j] = h4[j];
  int sum = 0;
#pragma unroll
  for (int j = 0; j < 16; ++j) sum += v[j].x + v[j].y + v[j].z + v[j].w;
  int incl = sum;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int u = __shfl_up(incl, o, 64);
    if (lane >= o) incl += u;
  }
  if (lane == 63) wsum[wv] = incl;
  __syncthreads();
  for (int k = 0; k < wv; ++k) incl += wsum[k];
  const int need = st->need;
  const int before = incl - sum;
  if (before < need && need <= incl) {
    int run = before;
    bool done = false;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int c4[4] = {v[j].x, v[j].y, v[j].z, v[j].w};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (!done && run + c4[q] >= need) {
          found_digit = 64 * t + 4 * j + q;
          found_before = run;
          found_count = c4[q];
          done = true;
        }
        run += c4[q];
      }
    }
  }
#pragma unroll
  for (int j = 0; j < 16; ++j) h4[j] = make_int4(0, 0, 0, 0);
  __syncthreads();
  if (t == 0) {
    const uint64_t prefix = (st->prefix << 16) | (uint64_t)found_digit;
    const int left = need - found_before;
    const int rest = 16 * (3 - round);   // key bits below this digit
    if (rest > 0 && left == found_count) {
      st->prefix = (prefix << rest) | ((uint64_t(1) << rest) - 1);
      st->done = 1;
    } else {
      st->prefix = prefix;
    }
    st->need = left;
  }
}

constexpr int kSelChunk = 1024;

__global__ void __launch_bounds__(256) k_sel_count(int64_t n_pad, uint64_t seed, const SelectState* st, int* counts) {
  __shared__ int red[256];
  const int64_t base = (int64_t)blockIdx.x * kSelChunk;
  const uint64_t T = st->prefix;
  int c = 0;
  for (int j = threadIdx.x; j < kSelChunk; j += 256) {
    const int64_t i = base + j;
    if (i < n_pad && splitmix64(seed, (uint64_t)i) <= T) ++c;
  }
  red[threadIdx.x] = c;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) counts[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) k_sel_write(int64_t n_pad, uint64_t seed, const SelectState* st,
                                                   const int* offsets, int64_t* rows) {
  __shared__ int pre[256];
  const int64_t base = (int64_t)blockIdx.x * kSelChunk;
  const uint64_t T = st->prefix;
  // each thread owns 4 consecutive indices
  int flags[4];
  int c = 0;
  for (int j = 0; j < 4; ++j) {
    const int64_t i = base + threadIdx.x * 4 + j;
    flags[j] = (i < n_pad && splitmix64(seed, (uint64_t)i) <= T) ? 1 : 0;
    c += flags[j];
  }
  pre[threadIdx.x] = c;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    int v = ((int)threadIdx.x >= off) ? pre[threadIdx.x - off] : 0;
    __syncthreads();
    pre[threadIdx.x] += v;
    __syncthreads();
  }
  int pos = offsets[blockIdx.x] + pre[threadIdx.x] - c;
  for (int j = 0; j < 4; ++j)
    if (flags[j]) rows[pos++] = base + threadIdx.x * 4 + j;
}

struct SrhtGeom {
  int64_t n_pad;
  int m, A, B, A_eff, logB;
};

// H_{n'} = H_A (x) H_B with row index a B + b: level 1 transforms blocks of
// B rows, level 2 combines the A blocks for the sampled rows only.  B is
// chosen so that about 16 to 32 sampled rows share each low part b: level
// 2's matrix-core work, s A d products, falls as B grows while level 1's
// rows coalesce better as it shrinks (groups of 16 rows), within
// 2^6 .. 2^10 (level 1 holds
// 64 rows per lane and at most 16 row groups across lanes), and at least
// 2^ceil(m / 2) when s is too small to decide (few samples per b).
static SrhtGeom srht_geom(int64_t n, int s = 0) {
  SrhtGeom g;
  g.m = 1;
  while ((int64_t(1) << g.m) < n) ++g.m;
  g.n_pad = int64_t(1) << g.m;
  int mb = (g.m + 1) / 2;
  if (s >= 1024) {
    mb = 0;
    while ((int64_t(16) << (mb + 1)) <= s) ++mb;   // floor(log2(s / 16))
    mb = std::max(6, std::min(10, mb));
  }
  mb = std::min(mb, g.m);
  g.logB = mb;
  g.B = 1 << mb;
  g.A = 1 << (g.m - mb);
  g.A_eff = (int)((n + g.B - 1) / g.B);
  return g;
}

static int srht_select_rows(int64_t n_pad, int s, uint64_t seed, int64_t* rows, Arena& ws, hipStream_t st) {
  const uint64_t seedR = seed ^ kSrhtRowSalt;
  int* hist = ws.take<int>(65536);
  SelectState* state = ws.take<SelectState>(1);
  const int chunks = (int)((n_pad + kSelChunk - 1) / kSelChunk);
  int* counts = ws.take<int>(chunks + 1);
  int* offsets = ws.take<int>(chunks + 1);
  if (!offsets) { set_error("srht: workspace too small"); return SRP_ENOMEM; }
  SRP_TRY(fill_i32(hist, 65536, 0, st));
  hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(1), 0, st, state, s);
  SRP_LAUNCH_CHECK();
  const unsigned nb = (unsigned)((n_pad + 255) / 256);
  for (int round = 0; round < 4; ++round) {
    hipLaunchKernelGGL(k_sel_hist, dim3(nb), dim3(256), 0, st, n_pad, seedR, round, state, hist);
    SRP_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sel_pick, dim3(1), dim3(1024), 0, st, hist, state, round);
    SRP_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_sel_count, dim3(chunks), dim3(256), 0, st, n_pad, seedR, state, counts);
  SRP_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(1024), 0, st, counts, chunks, offsets, (int*)nullptr);
  SRP_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_sel_write, dim3(chunks), dim3(256), 0, st, n_pad, seedR, state, offsets, rows);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

// Group the sampled rows by beta = r mod B (single workgroup).  For every
// beta: goff[beta] .. goff[beta+1] index into galpha / gslot, listing the
// sampled rows with that beta (alpha = r / B, slot = j).  The order inside
// a group does not affect any sum (level 2 sums over all blocks for every
// row), so positions come from LDS atomics.
__global__ void __launch_bounds__(1024) k_srht_group(const int64_t* rows, int s, int B, int logB,
                                                     int* goff, int* galpha, int* gslot) {
  __shared__ int cnt[1024];
  __shared__ int off[1025];
  const int t = threadIdx.x;
  for (int b = t; b < B; b += 1024) cnt[b] = 0;
  __syncthreads();
  for (int j = t; j < s; j += 1024) atomicAdd(&cnt[(int)(rows[j] & (B - 1))], 1);
  __syncthreads();
  if (t == 0) {
    int run = 0;
    for (int b = 0; b < B; ++b) { off[b] = run; run += cnt[b]; }
    off[B] = run;
  }
  __syncthreads();
  for (int b = t; b <= B; b += 1024) goff[b] = off[b];
  for (int j = t; j < s; j += 1024) {
    const int64_t r = rows[j];
    const int pos = atomicAdd(&off[(int)(r & (B - 1))], 1);
    galpha[pos] = (int)(r >> logB);
    gslot[pos] = j;
  }
}

// Level 1: length-B Walsh-Hadamard transform of every block of B rows, in
// LDS, for a chunk of CW columns.  Rows past n are zero (the padding).
template <class T, class Acc>
__global__ void __launch_bounds__(256) k_srht_level1(const T* __restrict__ A, int64_t n, int d, int B, int logB,
                                                     int CW, uint64_t seedD, Acc* __restrict__ Tbuf) {
  extern __shared__ unsigned char smem_raw[];
  Acc* tile = reinterpret_cast<Acc*>(smem_raw);
  const int a = blockIdx.y;          // column chunks of one row block run side by side
  const int c0 = blockIdx.x * CW;
  const int cw = min(CW, d - c0);
  const int tot = B * CW;
  for (int e = threadIdx.x; e < tot; e += 256) {
    const int r = e / CW, c = e % CW;
    const int64_t row = (int64_t)a * B + r;
    Acc v = Acc(0);
    if (c < cw && row < n) {
      const uint64_t w = splitmix64(seedD, (uint64_t)row);
      v = load_as<Acc>(A + row * d + c0 + c);
      if (w & 1ull) v = -v;
    }
    tile[e] = v;
  }
  __syncthreads();
  const int pairs = tot / 2;
  for (int lh = 0; lh < logB; ++lh) {
    const int h = 1 << lh;
    for (int q = threadIdx.x; q < pairs; q += 256) {
      const int rp = q / CW, c = q % CW;
      const int lo = ((rp >> lh) << (lh + 1)) | (rp & (h - 1));
      const int i0 = lo * CW + c, i1 = (lo + h) * CW + c;
      const Acc x = tile[i0], y = tile[i1];
      tile[i0] = x + y;
      tile[i1] = x - y;
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < tot; e += 256) {
    const int r = e / CW, c = e % CW;
    if (c < cw) Tbuf[((int64_t)a * B + r) * d + c0 + c] = tile[e];
  }
}

// Level 1 for B >= 64, in registers: a workgroup transforms block a for
// CW = 16384 / B columns.  Thread (c, g) of G = 256 / CW row groups first
// holds rows g + G i (i < 64) of column c: the butterflies over the six high
// row bits run in registers; one LDS exchange then gives thread (c, h) the
// rows lo + G (h 64/G + k), lo < G, k < 64/G, and the butterflies over the
// low log2 G row bits run in registers too.  One barrier per block.
template <class T, class Acc>
__global__ void __launch_bounds__(256) k_srht_level1_reg(const T* __restrict__ A, int64_t n, int d, int logB,
                                                         uint64_t seedD, Acc* __restrict__ Tbuf) {
  extern __shared__ unsigned char smem_raw[];
  Acc* tile = reinterpret_cast<Acc*>(smem_raw);   // [B][CW]
  const int B = 1 << logB;
  const int logCW = 14 - logB, CW = 1 << logCW;
  const int logG = 8 - logCW, G = 1 << logG;
  // the column chunks of one row block are consecutive workgroups, so the
  // rows they read and write stream through HBM together
  const int a = blockIdx.y;
  const int c0 = blockIdx.x * CW;
  const int c = threadIdx.x & (CW - 1), g = threadIdx.x >> logCW;
  const bool col_ok = c0 + c < d;
  // the block's signs D_i, one hash per row (after the tile)
  Acc* sgn = tile + 16384;
  for (int r = threadIdx.x; r < B; r += 256)
    sgn[r] = (splitmix64(seedD, (uint64_t)((int64_t)a * B + r)) & 1ull) ? Acc(-1) : Acc(1);
  __syncthreads();
  // one buffer resource for the block's rows: rows past n lie past it and
  // read zero, columns past d take an offset past it; every load issues
  // unconditionally, so all 64 of a thread are in flight together
  const int64_t row0 = (int64_t)a * B;
  const int64_t rows_here = n - row0 < B ? n - row0 : B;
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(A + row0 * d, rows_here * d * (int64_t)sizeof(T));
  Acc v[64];
#pragma unroll
  for (int i = 0; i < 64; ++i) {
    const int r = g + G * i;
    const int off = col_ok ? (r * d + c0 + c) * (int)sizeof(T) : kOob;
    v[i] = buf_load_as<Acc, T>(rs, off) * sgn[r];
  }
#pragma unroll
  for (int h = 1; h < 64; h <<= 1)
#pragma unroll
    for (int i = 0; i < 64; ++i)
      if ((i & h) == 0) {
        const Acc x = v[i], y = v[i + h];
        v[i] = x + y;
        v[i + h] = x - y;
      }
#pragma unroll
  for (int i = 0; i < 64; ++i) tile[(g + G * i) * CW + c] = v[i];
  __syncthreads();
  const int K = 64 >> logG;   // rows per low-bit group held by a thread
#pragma unroll
  for (int i = 0; i < 64; ++i) {
    const int lo = i & (G - 1), k = i >> logG;
    v[i] = tile[(lo + G * (g * K + k)) * CW + c];
  }
#pragma unroll
  for (int lh = 0; lh < 4; ++lh) {   // G <= 16
    if (lh < logG) {
      const int h = 1 << lh;
#pragma unroll
      for (int i = 0; i < 64; ++i)
        if ((i & h) == 0) {
          const Acc x = v[i], y = v[i + h];
          v[i] = x + y;
          v[i + h] = x - y;
        }
    }
  }
  if (col_ok) {
#pragma unroll
    for (int i = 0; i < 64; ++i) {
      const int lo = i & (G - 1), k = i >> logG;
      const int r = lo + G * (g * K + k);
      Tbuf[((int64_t)a * B + r) * d + c0 + c] = v[i];
    }
  }
}

// Level 1 for 2^LR <= B <= 1024 without an LDS tile: lane (c, g) of a wave
// holds rows g + G i (i < R = 2^LR) of column c, G = B / R row groups and
// 64 / G columns per wave (256 / G per block).  The butterflies over the
// LR high row bits run in registers, those over the log2 G low bits
// between lanes (lane shuffles); LDS holds only the block's signs, so
// occupancy is set by registers.  Rows past n read zero through the
// buffer resource, columns past d take an offset past it.
template <class T, class Acc, int LR>
__global__ void __launch_bounds__(256) k_srht_level1_lane(const T* __restrict__ A, int64_t n, int d, int logB,
                                                          uint64_t seedD, Acc* __restrict__ Tbuf) {
  constexpr int R = 1 << LR;
  __shared__ Acc sgn[1024];
  const int B = 1 << logB;
  const int logG = logB - LR, G = 1 << logG;
  const int logCW = 6 - logG, CW = 1 << logCW;          // columns per wave
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int a = blockIdx.y;
  const int c = (blockIdx.x * 4 + w) * CW + (lane & (CW - 1));
  const int g = lane >> logCW;
  for (int r = threadIdx.x; r < B; r += 256)
    sgn[r] = (splitmix64(seedD, (uint64_t)((int64_t)a * B + r)) & 1ull) ? Acc(-1) : Acc(1);
  __syncthreads();
  const bool col_ok = c < d;
  const int64_t row0 = (int64_t)a * B;
  const int64_t rows_here = n - row0 < B ? n - row0 : B;
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(A + row0 * d, rows_here * d * (int64_t)sizeof(T));
  Acc v[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int r = g + G * i;
    const int off = col_ok ? (r * d + c) * (int)sizeof(T) : kOob;
    v[i] = buf_load_as<Acc, T>(rs, off) * sgn[r];
  }
#pragma unroll
  for (int h = 1; h < R; h <<= 1)
#pragma unroll
    for (int i = 0; i < R; ++i)
      if ((i & h) == 0) {
        const Acc x = v[i], y = v[i + h];
        v[i] = x + y;
        v[i + h] = x - y;
      }
  for (int lb = 0; lb < logG; ++lb) {
    const int sh = CW << lb;
    const bool hi = (g >> lb) & 1;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const Acc p = __shfl_xor(v[i], sh, 64);
      v[i] = hi ? p - v[i] : v[i] + p;
    }
  }
  if (col_ok) {
#pragma unroll
    for (int i = 0; i < R; ++i) Tbuf[(row0 + g + G * i) * d + c] = v[i];
  }
}

// Level 2: out[slot] = s^-1/2 * sum_a (-1)^popcount(alpha & a) T[a B + beta].
template <class Acc>
__global__ void __launch_bounds__(256) k_srht_level2(const Acc* __restrict__ Tbuf, int d, int B, int A_eff,
                                                     const int* __restrict__ goff, const int* __restrict__ galpha,
                                                     const int* __restrict__ gslot, Acc scale, Acc* __restrict__ out) {
  constexpr int G = 16;
  const int beta = blockIdx.y;   // the column chunks of one beta are consecutive workgroups
  const int c = blockIdx.x * 256 + threadIdx.x;
  const int beg = goff[beta], cnt = goff[beta + 1] - beg;
  for (int g0 = 0; g0 < cnt; g0 += G) {
    const int gn = min(G, cnt - g0);
    int alpha[G];
    Acc acc[G];
#pragma unroll
    for (int j = 0; j < G; ++j) {
      alpha[j] = (j < gn) ? galpha[beg + g0 + j] : 0;
      acc[j] = Acc(0);
    }
    if (c < d) {
      // eight blocks' loads in flight at a time
#pragma unroll 8
      for (int a = 0; a < A_eff; ++a) {
        const Acc v = Tbuf[((int64_t)a * B + beta) * d + c];
#pragma unroll
        for (int j = 0; j < G; ++j) acc[j] += (__popc(alpha[j] & a) & 1) ? -v : v;
      }
      for (int j = 0; j < gn; ++j) out[(int64_t)gslot[beg + g0 + j] * d + c] = acc[j] * scale;
    }
  }
}

// Level 2 on FP32 matrix cores: for the sampled rows whose low bits are
// beta, out_beta = S T_beta with S[j][a] = (-1)^popcount(alpha_j & a) (the
// rows of H_A the samples pick) and T_beta the rows a B + beta of the
// level-1 output.  Up to NG groups of 16 sampled rows are the A operands
// of one pass over T_beta (each lane forms its +-1 entries from alpha_j and
// a; padding rows are 0); four rows a of T per step are the B operand.  A
// wave owns NT 16-column tiles (the block four waves side by side) and
// walks the a range in runs of four steps (16 rows of T), the next run's
// loads in flight during this run's products.  Each element of T is read
// once (a beta with more than 16 NG samples takes further passes).
template <int NT, int NG>
__global__ void __launch_bounds__(256) k_srht_level2_mfma(const float* __restrict__ Tbuf, int d, int B, int A_eff,
                                                          const int* __restrict__ goff,
                                                          const int* __restrict__ galpha,
                                                          const int* __restrict__ gslot, float scale,
                                                          float* __restrict__ out) {
  const int beta = blockIdx.y;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m = lane & 15, kq = lane >> 4;
  const int c0 = (blockIdx.x * 4 + w) * NT * 16;
  if (c0 >= d) return;
  const int beg = goff[beta], cnt = goff[beta + 1] - beg;
  const float* __restrict__ Tb = Tbuf + (int64_t)beta * d;
  const int64_t rstride = (int64_t)B * d;
  const int nss = (A_eff + 15) / 16;
  for (int g0 = 0; g0 < cnt; g0 += 16 * NG) {
    bool jok[NG];
    int alpha[NG];
    f32x4 acc[NG][NT];
#pragma unroll
    for (int q = 0; q < NG; ++q) {
      jok[q] = g0 + 16 * q + m < cnt;
      alpha[q] = jok[q] ? galpha[beg + g0 + 16 * q + m] : 0;
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[q][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    const int ng = min(NG, (cnt - g0 + 15) / 16);   // groups with samples in this pass
    auto load = [&](int ss, float (&bv)[4][NT]) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int a = 16 * ss + 4 * u + kq;
        const bool aok = a < A_eff;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const int col = c0 + 16 * t + m;
          bv[u][t] = (aok && col < d) ? Tb[(int64_t)a * rstride + col] : 0.f;
        }
      }
    };
    float cur[4][NT], nxt[4][NT];
    load(0, cur);
    for (int ss = 0; ss < nss; ++ss) {
      load(ss + 1, nxt);
#pragma unroll
      for (int q = 0; q < NG; ++q) {
        if (q < ng) {
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int a = 16 * ss + 4 * u + kq;
            const float sg = (jok[q] && a < A_eff) ? ((__popc(alpha[q] & a) & 1) ? -1.f : 1.f) : 0.f;
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[q][t] = mfma16x16x4(sg, cur[u][t], acc[q][t]);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int t = 0; t < NT; ++t) cur[u][t] = nxt[u][t];
    }
#pragma unroll
    for (int q = 0; q < NG; ++q)
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int col = c0 + 16 * t + m;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int j = g0 + 16 * q + 4 * kq + r;   // accumulator row
          if (j < cnt && col < d) out[(int64_t)gslot[beg + j] * d + col] = acc[q][t][r] * scale;
        }
      }
  }
}

// ------------------------------------------------------ fused SRHT (FP32)
// Both levels in one read of FP32 data, for B = 2^LB rows per block with
// LB = 6 or 7 (s from 1024 to 4095).  A workgroup owns 16 columns, one half
// of the low parts beta (the top bit of beta) and a run of steps of four
// consecutive blocks.  The step's rows stream into an LDS ring four steps
// deep (buffer loads to LDS, 16 B per lane; three steps in flight).  Four
// producer waves (one per SIMD) take one block of a step each: the signs D
// from the plan's bit table, the block's two halves combined for the
// workgroup's beta half ((-1)^popcount(beta & b) splits into the top bits'
// sign and the low bits'), then the remaining B/2-point Walsh-Hadamard
// transform, the register bits in registers and the two lane bits by DPP
// exchanges.  Twelve consumer waves each own up to 14 accumulator tiles,
// one per group of at most 16 sampled rows with the same beta:
// out_group += S T_beta on 16x16x4 FP32 matrix cores, the A operand the
// signs (-1)^popcount(alpha_j & a) of the group's rows for the step's four
// blocks a, the B operand the four blocks' level-1 row beta from the LDS
// buffer T.  A step has two barriers: the producers transform step i in
// registers while the consumers multiply step i - 1 out of T, then write
// T.  Workgroups that read the same bytes (both beta halves of four
// neighbouring column slices) get block indexes equal mod 8: they run on
// one XCD and share its L2.  With several row ranges per column slice
// each range writes a partial sketch and a second kernel adds them in
// range order.
constexpr int kFuWaves = 16;
constexpr int kFuThreads = 64 * kFuWaves;
constexpr int kFuProd = 4;                     // producer waves: 12 .. 15, one per SIMD
constexpr int kFuCons = kFuWaves - kFuProd;    // consumer waves: 0 .. 11
constexpr int kFuSlots = 14;                   // accumulator tiles per consumer wave and pass (168 groups)
constexpr int kFuRing = 4;                     // steps of rows held in LDS (three in flight)
constexpr int kFuCSG = 4;                      // column slices sharing an XCD
constexpr int kFuMaxGroups = 320;              // 16-row groups of one beta half

template <int LB>
struct FuShape {
  static constexpr int B = 1 << LB;
  static constexpr int HB = B / 2;                              // betas per workgroup
  static constexpr int R = B / 4;                               // rows per producer lane
  static constexpr int STEP_ROWS = 4 * B;
  static constexpr int STEP_F = STEP_ROWS * 16;                 // floats per step (16 columns)
  static constexpr int DMA_W = STEP_ROWS / (16 * kFuWaves);     // 16-row loads per wave and step
  static constexpr int TP = HB * 16 + 16;                       // T block pitch: the 4 blocks on distinct banks
  static constexpr size_t lds_bytes() {
    return (size_t)(kFuRing * STEP_F + 4 * TP + 3 * kFuMaxGroups + 4) * 4;
  }
};

// s_waitcnt on the vector-memory counter only (gfx9 encoding: expcnt and
// lgkmcnt at their maxima).
template <int N>
__device__ __forceinline__ void fu_wait_vm() {
  static_assert(N >= 0 && N < 16, "vmcnt field");
  __builtin_amdgcn_s_waitcnt(N | (0x7 << 4) | (0xF << 8));
}

// Rows row0 .. row0 + 4B - 1 (past n: zero), columns c0 .. c0 + 15 (past d:
// zero) into the ring slot dst, as [row][16 columns]: each 16-row load moves
// 1 KB, lane l the 16 B of row l / 4, columns 4 (l % 4) .. + 3.
template <int LB>
__device__ __forceinline__ void fu_issue(const float* A, int64_t n, int d, int64_t row0, int c0, float* dst, int w,
                                         int lane) {
  using S = FuShape<LB>;
  const int64_t left = n - row0;
  const int64_t rows = left < S::STEP_ROWS ? (left > 0 ? left : 0) : S::STEP_ROWS;
  const __amdgpu_buffer_rsrc_t r = make_rsrc(A + (rows > 0 ? row0 * d : 0), rows * d * 4);
  const int col = c0 + 4 * (lane & 3);
#pragma unroll
  for (int j = 0; j < S::DMA_W; ++j) {
    const int ins = w * S::DMA_W + j;
    const int row = 16 * ins + (lane >> 2);
    const int voff = col < d ? (row * d + col) * 4 : kOob;
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (__attribute__((address_space(3))) void*)(dst + 256 * ins), 16,
                                             voff, 0, 0, 0);
  }
}

__device__ __forceinline__ void fu_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// The end of a step: this wave's rows of the next step have landed (npend
// later steps, 0 to 2, stay in flight), then the workgroup barrier.
template <int LB>
__device__ __forceinline__ void fu_end(int npend) {
  constexpr int W = FuShape<LB>::DMA_W;
  if (npend >= 2) fu_wait_vm<2 * W>();
  else if (npend == 1) fu_wait_vm<W>();
  else fu_wait_vm<0>();
  fu_barrier();
}

template <int CTRL>
__device__ __forceinline__ float fu_dpp(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, 0xF, 0xF, false));
}

// Producer step it: the DMA of step it + 3 into rdma, level 1 of block a
// (slot p of ring step rcur) for this workgroup's beta half q in registers
// while the consumers use T; after the first barrier the result goes to T.
// Lane (g = lane % 4, c = lane / 4) holds rows b = g + 4 i of column c;
// after the transform it holds T[beta_lo = g + 4 i], i < R / 2.  The LDS
// regions come in as separate restrict pointers, so the compiler's wait
// insertion sees these reads and writes as disjoint from the DMA in flight.
template <int LB>
__device__ __forceinline__ void fu_produce(const float* __restrict__ rcur, float* __restrict__ rdma,
                                           float* __restrict__ tw, const float* A, int64_t n, int d, int c0,
                                           int64_t dma_row0, bool issue, bool work, int npend,
                                           const uint32_t* __restrict__ dbits, int64_t a, int q, int p, int w,
                                           int lane) {
  using S = FuShape<LB>;
  constexpr int R = S::R, H = R / 2, NW = S::B / 32;
  if (issue) fu_issue<LB>(A, n, d, dma_row0, c0, rdma, w, lane);
  const int g = lane & 3, c = lane >> 2;
  float v[R];
  if (work) {
    uint32_t wv[NW];
#pragma unroll
    for (int k = 0; k < NW; ++k) wv[k] = dbits[a * NW + k] >> g;   // bit b of the block: row b negated
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const uint32_t x = __builtin_bit_cast(uint32_t, rcur[(p * S::B + g + 4 * i) * 16 + c]);
      const uint32_t f = (wv[i >> 3] << (31 - 4 * (i & 7))) & 0x80000000u;
      v[i] = __builtin_bit_cast(float, x ^ f);
    }
    // top bit of b against the top bit of beta (q)
    const float sq = q ? -1.f : 1.f;
#pragma unroll
    for (int i = 0; i < H; ++i) v[i] = fmaf(sq, v[i + H], v[i]);
#pragma unroll
    for (int h = 1; h < H; h <<= 1)
#pragma unroll
      for (int i = 0; i < H; ++i)
        if ((i & h) == 0) {
          const float x = v[i], y = v[i + h];
          v[i] = x + y;
          v[i + h] = x - y;
        }
    // lane bits 0 and 1 of b: partner lanes g ^ 1 and g ^ 2 (quad permutes)
    const float s1 = (g & 1) ? -1.f : 1.f, s2 = (g & 2) ? -1.f : 1.f;
#pragma unroll
    for (int i = 0; i < H; ++i) v[i] = fmaf(s1, v[i], fu_dpp<0xB1>(v[i]));
#pragma unroll
    for (int i = 0; i < H; ++i) v[i] = fmaf(s2, v[i], fu_dpp<0x4E>(v[i]));
  }
  fu_barrier();   // the consumers are done with T
  if (work) {
#pragma unroll
    for (int i = 0; i < H; ++i) tw[p * S::TP + (g + 4 * i) * 16 + c] = v[i];
  }
  fu_end<LB>(npend);
}

// Consumer step it: the DMA of step it + 3 into rdma, then the products of
// step it - 1 from tr (ak: the block of this lane's contraction index).
template <int LB>
__device__ __forceinline__ void fu_consume(float* __restrict__ rdma, const float* __restrict__ tr, const float* A,
                                           int64_t n, int d, int c0, int64_t dma_row0, bool issue, bool work,
                                           int npend, int ak, int nsl, const int (&alpha)[kFuSlots],
                                           const int (&bl16)[kFuSlots], int lb, f32x4 (&acc)[kFuSlots], int w,
                                           int lane) {
  if (issue) fu_issue<LB>(A, n, d, dma_row0, c0, rdma, w, lane);
  if (work) {
    // T operands eight slots at a time, all loads in flight before the
    // products (slots past nsl read a valid, unused address)
#pragma unroll
    for (int j0 = 0; j0 < kFuSlots; j0 += 8) {
      float tv[8];
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (j0 + j < kFuSlots) tv[j] = tr[lb + bl16[j0 + j]];
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (j0 + j < kFuSlots && j0 + j < nsl) {
          const float sg = __builtin_bit_cast(float, 0x3f800000u | ((uint32_t)__popc(alpha[j0 + j] & ak) << 31));
          acc[j0 + j] = mfma16x16x4(sg, tv[j], acc[j0 + j]);
        }
    }
  }
  fu_barrier();   // T is free for the producers
  fu_end<LB>(npend);
}

template <int LB>
__global__ void __launch_bounds__(kFuThreads) k_srht_fused(const float* __restrict__ A, int64_t n, int d, int ncs,
                                                          int ngrp, int rsp, int nsteps,
                                                          const uint32_t* __restrict__ dbits,
                                                          const int* __restrict__ goff,
                                                          const int* __restrict__ galpha,
                                                          const int* __restrict__ gslot, int s, float scale,
                                                          float* __restrict__ out) {
  using S = FuShape<LB>;
  extern __shared__ float fsm[];
  float* ring = fsm;
  float* tbuf = ring + kFuRing * S::STEP_F;
  int* gtab = reinterpret_cast<int*>(tbuf + 4 * S::TP);   // [group][beta_local, start, count]
  int* gcount = gtab + 3 * kFuMaxGroups;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  // block index -> (sharing group, member); members share blockIdx % 8
  const int u = blockIdx.x, rest = u >> 3;
  const int member = rest % (2 * kFuCSG);
  const int grp = (rest / (2 * kFuCSG)) * 8 + (u & 7);
  if (grp >= ngrp) return;
  const int q = member & 1;
  const int ncsg = (ncs + kFuCSG - 1) / kFuCSG;
  const int rs = grp / ncsg;
  const int cs = (grp - rs * ncsg) * kFuCSG + (member >> 1);
  if (cs >= ncs) return;
  const int c0 = 16 * cs;
  const int st_beg = (int)((int64_t)rs * nsteps / rsp);
  const int nst = (int)((int64_t)(rs + 1) * nsteps / rsp) - st_beg;
  // the groups of this beta half: beta = q HB + lane, ceil(count / 16) each
  if (w == 0) {
    int start = 0, cnt = 0, ngb = 0;
    if (lane < S::HB) {
      const int beta = q * S::HB + lane;
      start = goff[beta];
      cnt = goff[beta + 1] - start;
      ngb = (cnt + 15) >> 4;
    }
    int incl = ngb;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(incl, o, 64);
      if (lane >= o) incl += t;
    }
    const int excl = incl - ngb;
    for (int j = 0; j < ngb; ++j) {
      const int gi = excl + j;
      if (gi < kFuMaxGroups) {
        gtab[3 * gi] = lane;
        gtab[3 * gi + 1] = start + 16 * j;
        gtab[3 * gi + 2] = min(16, cnt - 16 * j);
      }
    }
    if (lane == 63) *gcount = min(incl, kFuMaxGroups);
  }
  __syncthreads();
  const int ng = *gcount;
  float* dst = out + (rsp > 1 ? (int64_t)rs * s * d : 0);
  const float sc = rsp > 1 ? 1.f : scale;
  for (int pbase = 0; pbase < ng; pbase += kFuCons * kFuSlots) {
    if (w >= kFuCons) {
      const int p = w - kFuCons;
      __builtin_amdgcn_s_waitcnt(0);   // nothing of an earlier pass in flight
      for (int j = 0; j < 3 && j < nst; ++j)
        fu_issue<LB>(A, n, d, (int64_t)(st_beg + j) * S::STEP_ROWS, c0, ring + j * S::STEP_F, w, lane);
      fu_end<LB>(min(nst, 3) - 1);
      for (int it = 0; it <= nst; ++it) {
        fu_produce<LB>(ring + (it % kFuRing) * S::STEP_F, ring + ((it + 3) % kFuRing) * S::STEP_F, tbuf, A, n, d,
                       c0, (int64_t)(st_beg + it + 3) * S::STEP_ROWS, it + 3 < nst, it < nst,
                       (it + 2 < nst) + (it + 3 < nst), dbits, 4 * (int64_t)(st_beg + it) + p, q, p, w, lane);
      }
    } else {
      int alpha[kFuSlots], bl16[kFuSlots];
      f32x4 acc[kFuSlots];
      const int left = ng - pbase - w;
      const int nsl = left > 0 ? min(kFuSlots, (left + kFuCons - 1) / kFuCons) : 0;
      const int m = lane & 15, lb = (lane >> 4) * S::TP + m;
#pragma unroll
      for (int j = 0; j < kFuSlots; ++j) {
        acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
        alpha[j] = 0;
        bl16[j] = 0;
        if (j < nsl) {
          const int gi = pbase + w + kFuCons * j;
          const int cn = gtab[3 * gi + 2];
          // rows past the group's count are never stored: any alpha serves
          alpha[j] = m < cn ? galpha[gtab[3 * gi + 1] + m] : 0;
          bl16[j] = __builtin_amdgcn_readfirstlane(16 * gtab[3 * gi]);
        }
      }
      __builtin_amdgcn_s_waitcnt(0);   // the alpha loads have landed before the row stream starts
      for (int j = 0; j < 3 && j < nst; ++j)
        fu_issue<LB>(A, n, d, (int64_t)(st_beg + j) * S::STEP_ROWS, c0, ring + j * S::STEP_F, w, lane);
      fu_end<LB>(min(nst, 3) - 1);
      for (int it = 0; it <= nst; ++it) {
        fu_consume<LB>(ring + ((it + 3) % kFuRing) * S::STEP_F, tbuf, A, n, d, c0,
                       (int64_t)(st_beg + it + 3) * S::STEP_ROWS, it + 3 < nst, it > 0,
                       (it + 2 < nst) + (it + 3 < nst), 4 * (st_beg + it - 1) + (lane >> 4), nsl, alpha, bl16, lb,
                       acc, w, lane);
      }
      const int col = c0 + (lane & 15);
#pragma unroll
      for (int j = 0; j < kFuSlots; ++j)
        if (j < nsl) {
          const int gi = pbase + w + kFuCons * j;
          const int start = gtab[3 * gi + 1], cn = gtab[3 * gi + 2];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = acc_row<float>(lane, r);
            if (row < cn && col < d) dst[(int64_t)gslot[start + row] * d + col] = acc[j][r] * sc;
          }
        }
    }
    __syncthreads();   // the ring and T are reused by the next pass
  }
}

// out = scale * (sum of the row-range partials, in range order)
__global__ void __launch_bounds__(256) k_srht_fused_sum(const float* __restrict__ part, int rsp, int64_t count,
                                                        float scale, float* __restrict__ out) {
  const int64_t e = blockIdx.x * 256ll + threadIdx.x;
  if (e >= count) return;
  float v = 0.f;
  for (int r = 0; r < rsp; ++r) v += part[r * count + e];
  out[e] = v * scale;
}

// Sign bits of D: bit i % 32 of word i / 32 set when row i is negated.
__global__ void __launch_bounds__(256) k_srht_sign_bits(int64_t nwords, uint64_t seedD, uint32_t* __restrict__ bits) {
  const int64_t r = blockIdx.x * 256ll + threadIdx.x;
  const bool neg = r < nwords * 32 && (splitmix64(seedD, (uint64_t)r) & 1ull);
  const uint64_t m = __ballot(neg);
  const int lane = threadIdx.x & 63;
  const int64_t word = (r - lane) / 32;
  if (lane == 0 && word < nwords) bits[word] = (uint32_t)m;
  if (lane == 32 && word + 1 < nwords) bits[word + 1] = (uint32_t)(m >> 32);
}

static int64_t srht_sign_words(const SrhtGeom& g) {
  // four-block steps past the last block read signs too (their rows are zero)
  const int64_t rows = (int64_t)((g.A_eff + 3) / 4) * 4 * g.B;
  return ((rows + 63) / 64) * 2;
}

// Whether the fused kernel takes this FP32 view.
static bool srht_fused_ok(const SrhtGeom& g, int s, int d, const void* A) {
  return (g.logB == 6 || g.logB == 7) && d % 4 == 0 && d > 0 && (reinterpret_cast<uintptr_t>(A) & 15) == 0 &&
         s + 15 * (g.B / 2) <= 16 * kFuMaxGroups;
}

// The step loop counts its own loads (s_waitcnt on the vector-memory
// counter): a register spill would add scratch loads to that count, so a
// build whose kernel uses scratch memory keeps the two-level kernels.
template <int LB>
static bool srht_fused_clean() {
  static const bool clean = [] {
    hipFuncAttributes attr{};
    return hipFuncGetAttributes(&attr, (const void*)k_srht_fused<LB>) == hipSuccess && attr.localSizeBytes == 0;
  }();
  return clean;
}

template <int LB>
static int srht_fused_launch(const float* A, int64_t n, int d, int s, const SrhtGeom& g, const uint32_t* dbits,
                             const int* goff, const int* galpha, const int* gslot, float* part, size_t part_floats,
                             float* out, hipStream_t st) {
  using S = FuShape<LB>;
  const int ncs = (d + 15) / 16;
  const int ncsg = (ncs + kFuCSG - 1) / kFuCSG;
  const int nsteps = (g.A_eff + 3) / 4;
  // about 256 workgroups: split the rows when the column slices are few
  int rsp = std::max(1, 32 / ncsg);
  rsp = std::min(rsp, nsteps);
  while (rsp > 1 && (size_t)rsp * s * d > part_floats) --rsp;
  const int ngrp = ncsg * rsp;
  const unsigned grid = (unsigned)((ngrp + 7) / 8) * 8 * 2 * kFuCSG;
  const float scale = (float)(1.0 / std::sqrt((double)s));
  SRP_TRY(allow_dynamic_lds((const void*)k_srht_fused<LB>, S::lds_bytes()));
  hipLaunchKernelGGL((k_srht_fused<LB>), dim3(grid), dim3(kFuThreads), S::lds_bytes(), st, A, n, d, ncs, ngrp, rsp,
                     nsteps, dbits, goff, galpha, gslot, s, scale, rsp > 1 ? part : out);
  SRP_LAUNCH_CHECK();
  if (rsp > 1) {
    const int64_t count = (int64_t)s * d;
    hipLaunchKernelGGL(k_srht_fused_sum, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, part, rsp, count,
                       scale, out);
    SRP_LAUNCH_CHECK();
  }
  return SRP_OK;
}

static int srht_chunk_cols(int B, int acc_bytes) {
  // LDS tile of B x CW elements, at most 64 KiB.
  int cw = (64 * 1024) / (B * acc_bytes);
  if (cw > 128) cw = 128;
  if (cw < 1) cw = 1;
  return cw;
}

size_t srht_ws_bytes(int64_t n, int d, int s, int dtype) {
  SrhtGeom g = srht_geom(n, s);
  const size_t acc = dtype == SRP_F64 ? 8 : 4;
  const int chunks = (int)((g.n_pad + kSelChunk - 1) / kSelChunk);
  return bytes_of<int>(65536) + bytes_of<SelectState>(1) + 2 * bytes_of<int>(chunks + 1) +
         bytes_of<int64_t>(s) + bytes_of<int>(g.B + 1) + 2 * bytes_of<int>(s) +
         bytes_of<uint32_t>((size_t)srht_sign_words(g)) + (((size_t)g.A_eff * g.B * d * acc + 255) & ~size_t(255));
}

int srht_rows_run(int64_t n, int s, uint64_t seed, int64_t* rows, Arena& ws, hipStream_t st) {
  SrhtGeom g = srht_geom(n);
  if ((int64_t)s > g.n_pad || g.m > 20) {
    set_error("srht: need s <= n' <= 2^20 (n=%lld, s=%d)", (long long)n, s);
    return SRP_EINVAL;
  }
  return srht_select_rows(g.n_pad, s, seed, rows, ws, st);
}

template <class T, class Acc>
static int srht_levels(const T* A, int64_t n, int d, int s, uint64_t seed, const SrhtGeom& g,
                       const int* goff, const int* galpha, const int* gslot, const uint32_t* dbits, Acc* Tbuf,
                       size_t tcount, Acc* out, hipStream_t st) {
  const int logB = g.logB;
  if constexpr (std::is_same<T, float>::value) {
    if (dbits && srht_fused_ok(g, s, d, A) && (logB == 6 ? srht_fused_clean<6>() : srht_fused_clean<7>())) {
      // one read of the data, no level-1 intermediate (Tbuf holds the
      // row-range partials)
      if (logB == 6)
        return srht_fused_launch<6>(A, n, d, s, g, dbits, goff, galpha, gslot, Tbuf, tcount, out, st);
      return srht_fused_launch<7>(A, n, d, s, g, dbits, goff, galpha, gslot, Tbuf, tcount, out, st);
    }
  }
  if constexpr (sizeof(Acc) == 4) {
    if (logB >= 6 && logB <= 10) {
      // FP32: level 1 in registers and lane shuffles, level 2 on matrix
      // cores.  Groups of 16 per pass: the expected
      // samples per class plus four standard deviations, so that nearly
      // every class reads its rows once.
      const int CWB = 256 >> (logB - 6);   // columns per block
      dim3 grid1((d + CWB - 1) / CWB, g.A_eff);
      hipLaunchKernelGGL((k_srht_level1_lane<T, Acc, 6>), grid1, dim3(256), 0, st, A, n, d, logB,
                         seed ^ kSrhtSignSalt, Tbuf);
      SRP_LAUNCH_CHECK();
      constexpr int NT = 2;
      const double mean = (double)s / g.B;
      const int want = (int)std::ceil((mean + 4.0 * std::sqrt(mean) + 1.0) / 16.0);
      dim3 grid2((d + 4 * NT * 16 - 1) / (4 * NT * 16), g.B);
      const float sc = (float)(1.0 / std::sqrt((double)s));
      const float* Tf = (const float*)Tbuf;
      float* of = (float*)out;
      if (want <= 2)
        hipLaunchKernelGGL((k_srht_level2_mfma<NT, 2>), grid2, dim3(256), 0, st, Tf, d, g.B, g.A_eff, goff, galpha,
                           gslot, sc, of);
      else if (want <= 4)
        hipLaunchKernelGGL((k_srht_level2_mfma<NT, 4>), grid2, dim3(256), 0, st, Tf, d, g.B, g.A_eff, goff, galpha,
                           gslot, sc, of);
      else
        hipLaunchKernelGGL((k_srht_level2_mfma<NT, 6>), grid2, dim3(256), 0, st, Tf, d, g.B, g.A_eff, goff, galpha,
                           gslot, sc, of);
      SRP_LAUNCH_CHECK();
      return SRP_OK;
    }
  }
  // FP64, and blocks outside 2^6 .. 2^10: level 1 through an LDS tile
  // (registers for the 64 high row bits when B >= 64), block-major output;
  // level 2 on the vector units.
  if (logB >= 6 && logB <= 10) {
    const int CW = 16384 >> logB;
    dim3 grid1((d + CW - 1) / CW, g.A_eff);
    const size_t lds = (size_t)(16384 + 1024) * sizeof(Acc);
    SRP_TRY(allow_dynamic_lds((const void*)k_srht_level1_reg<T, Acc>, lds));
    hipLaunchKernelGGL((k_srht_level1_reg<T, Acc>), grid1, dim3(256), lds, st, A, n, d, logB,
                       seed ^ kSrhtSignSalt, Tbuf);
  } else {
    const int CW = srht_chunk_cols(g.B, (int)sizeof(Acc));
    dim3 grid1((d + CW - 1) / CW, g.A_eff);
    const size_t lds = (size_t)g.B * CW * sizeof(Acc);
    hipLaunchKernelGGL((k_srht_level1<T, Acc>), grid1, dim3(256), lds, st, A, n, d, g.B, logB, CW,
                       seed ^ kSrhtSignSalt, Tbuf);
  }
  SRP_LAUNCH_CHECK();
  dim3 grid2((d + 255) / 256, g.B);
  hipLaunchKernelGGL((k_srht_level2<Acc>), grid2, dim3(256), 0, st, Tbuf, d, g.B, g.A_eff, goff, galpha,
                     gslot, (Acc)(1.0 / std::sqrt((double)s)), out);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

size_t srht_plan_bytes(int64_t n, int s) {
  const SrhtGeom g = srht_geom(n, s);
  return bytes_of<int64_t>(s) + bytes_of<int>(g.B + 1) + 2 * bytes_of<int>(s) +
         bytes_of<uint32_t>((size_t)srht_sign_words(g));
}

int srht_plan_run(int64_t n, int s, uint64_t seed, SrhtPlan* plan, Arena& keep, Arena& scratch, hipStream_t st) {
  SrhtGeom g = srht_geom(n, s);
  if ((int64_t)s > g.n_pad || g.m > 20) {
    set_error("srht: need s <= n' <= 2^20 (n=%lld, s=%d)", (long long)n, s);
    return SRP_EINVAL;
  }
  plan->n = n;
  plan->s = s;
  plan->seed = seed;
  plan->rows = keep.take<int64_t>(s);
  plan->goff = keep.take<int>(g.B + 1);
  plan->galpha = keep.take<int>(s);
  plan->gslot = keep.take<int>(s);
  const int64_t words = srht_sign_words(g);
  plan->dbits = keep.take<uint32_t>((size_t)words);
  if (!plan->gslot || !plan->dbits) { set_error("srht: workspace too small"); return SRP_ENOMEM; }
  hipLaunchKernelGGL(k_srht_sign_bits, dim3((unsigned)((words * 32 + 255) / 256)), dim3(256), 0, st, words,
                     seed ^ kSrhtSignSalt, plan->dbits);
  SRP_LAUNCH_CHECK();
  SRP_TRY(srht_select_rows(g.n_pad, s, seed, plan->rows, scratch, st));
  hipLaunchKernelGGL(k_srht_group, dim3(1), dim3(1024), 0, st, plan->rows, s, g.B, g.logB, plan->goff,
                     plan->galpha, plan->gslot);
  SRP_LAUNCH_CHECK();
  return SRP_OK;
}

int srht_apply_run(const SrhtPlan& plan, const void* A, int dtype, int d, void* out, Arena& ws, hipStream_t st) {
  const int64_t n = plan.n;
  const int s = plan.s;
  const uint64_t seed = plan.seed;
  SrhtGeom g = srht_geom(n, s);
  const size_t tcount = (size_t)g.A_eff * g.B * d;
  if (dtype == SRP_F64) {
    double* Tbuf = ws.take<double>(tcount);
    if (!Tbuf) { set_error("srht: workspace too small"); return SRP_ENOMEM; }
    return srht_levels((const double*)A, n, d, s, seed, g, plan.goff, plan.galpha, plan.gslot, plan.dbits, Tbuf,
                       tcount, (double*)out, st);
  }
  float* Tbuf = ws.take<float>(tcount);
  if (!Tbuf) { set_error("srht: workspace too small"); return SRP_ENOMEM; }
  if (dtype == SRP_F32)
    return srht_levels((const float*)A, n, d, s, seed, g, plan.goff, plan.galpha, plan.gslot, plan.dbits, Tbuf,
                       tcount, (float*)out, st);
  if (dtype == SRP_BF16)
    return srht_levels((const bf16*)A, n, d, s, seed, g, plan.goff, plan.galpha, plan.gslot, plan.dbits, Tbuf,
                       tcount, (float*)out, st);
  if (dtype == SRP_FP8E4M3)
    return srht_levels((const fp8e4m3*)A, n, d, s, seed, g, plan.goff, plan.galpha, plan.gslot, plan.dbits, Tbuf,
                       tcount, (float*)out, st);
  set_error("srht: bad dtype %d", dtype);
  return SRP_EINVAL;
}

int srht_run(const void* A, int dtype, int64_t n, int d, int s, uint64_t seed, void* out, Arena& ws,
             hipStream_t st) {
  SrhtPlan plan;
  SRP_TRY(srht_plan_run(n, s, seed, &plan, ws, ws, st));
  return srht_apply_run(plan, A, dtype, d, out, ws, st);
}

}  // namespace srp
