// HIP kernels of the SpGEMM pipeline for gfx950 (CDNA4, wave64).
//
// C = A * B on CSR FP64 operands, row by row as in the paper's row-major
// (Gustavson) algorithm, Section IV-A: row r of C accumulates a(r,c) * b(c,x)
// over the stored entries of row r of A (in stored order) and of row c of B.
// Output rows are sorted by column (Section IV-B append contract).
//
// Pipeline: features -> sizing/tiering -> scan of tile costs -> tile bounds
// -> tile kernel (symbolic, numeric, or one pass into a padded buffer that
// k_compact moves into C) and k_big for the workgroup-tier rows; products
// whose rows all take the row-per-thread merge run k_wave_merge instead
// (its one pass: a decoupled look-back over waves).
#include <algorithm>
#include <mutex>

#include "device_common.h"
#include "spgemm_kernels.h"
#include "spgemm_internal.h"

namespace spg {

// ------------------------------------------------------------------ fills
__global__ void k_fill_i64(int64_t *p, int64_t v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
    p[i] = v;
}
__global__ void k_fill_u64(uint64_t *p, uint64_t v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
    p[i] = v;
}

// Zeroes the counters whose bits are set in `mask` (one launch for the
// per-run counters instead of one fill each).
__global__ void k_clear_ctrs(int64_t *c, uint32_t mask) {
  const int t = threadIdx.x;
  if (t < 32 && ((mask >> t) & 1u)) c[t] = 0;
}

hipError_t launch_clear_counters(int64_t *counters, uint32_t mask, hipStream_t s) {
  hipLaunchKernelGGL(k_clear_ctrs, dim3(1), dim3(kWave), 0, s, counters, mask);
  return hipGetLastError();
}

static int grid_for(int64_t n, int cap = 65536) {
  int64_t g = (n + kBlock - 1) / kBlock;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

hipError_t launch_fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i64, dim3(grid_for(n, 4096)), dim3(kBlock), 0, s, p, v, n);
  return hipGetLastError();
}
hipError_t launch_fill_u64(uint64_t *p, uint64_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 4096)), dim3(kBlock), 0, s, p, v, n);
  return hipGetLastError();
}

// --------------------------------------------------------------- validate
// Canonical CSR: row_ptr[0] == 0, non-decreasing, row_ptr[rows] == nnz,
// columns in [0, cols) and strictly increasing inside a row.
__global__ void k_validate(const int64_t *rp, const int32_t *col, int64_t rows, int64_t cols,
                           int64_t nnz, int64_t *counters) {
  int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  bool bad = false;
  if (i == 0) bad |= (rp[0] != 0) || (rp[rows] != nnz);
  if (i < rows) {
    int64_t s = rp[i], e = rp[i + 1];
    if (e < s || s < 0 || e > nnz) {
      bad = true;
    } else {
      int64_t prev = -1;
      for (int64_t q = s; q < e; ++q) {
        int64_t c = col[q];
        if (c <= prev || c >= cols) { bad = true; break; }
        prev = c;
      }
    }
  }
  if (bad) atomicOr((unsigned long long *)&counters[kCtrError], (unsigned long long)kErrNotCanonical);
}

hipError_t launch_validate(const int64_t *rp, const int32_t *col, int64_t rows, int64_t cols,
                           int64_t nnz, int64_t *counters, hipStream_t s) {
  int64_t n = rows > 0 ? rows : 1;
  hipLaunchKernelGGL(k_validate, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                     rp, col, rows, cols, nnz, counters);
  return hipGetLastError();
}

// --------------------------------------------------------------- features
// Per row i of A: entries of the row, multiplication count (the paper's
// estimate of Section IV-B taken per row; it never underestimates nnz(C_i)),
// the longest selected B row (a lower bound: those columns all appear in
// C_i), and the smallest/largest column any selected B row touches (the
// "MinMax" region of Section IV-B).  The exact int64 sum of the counts is
// the paper's multiplication count of Section III.
// The B row that stored entry e of A selects: its start and length.
__device__ __forceinline__ void b_row_of(const Operands &op, int64_t e, int64_t &bs, int32_t &bl) {
  const int32_t k = op.a_col[e];
  bs = op.b_rp[k];
  bl = (int32_t)(op.b_rp[k + 1] - bs);
}

// The slice of that B row whose columns lie in [c0, c1) (c1 < 0: all of
// it), found by binary search (B's rows are sorted).
__device__ __forceinline__ void b_row_part(const Operands &op, int64_t e, int32_t c0, int32_t c1, int64_t &bs,
                                           int32_t &bl) {
  b_row_of(op, e, bs, bl);
  if (c1 < 0) return;
  int64_t s[2];
  const int32_t x[2] = {c0, c1};
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    int64_t l = bs, h = bs + bl;
    while (l < h) {
      const int64_t m = (l + h) >> 1;
      if (op.b_col[m] < x[k]) l = m + 1;
      else h = m;
    }
    s[k] = l;
  }
  bs = s[0];
  bl = (int32_t)(s[1] - s[0]);
}

// Partials per workgroup: multiplication count, longest row of A, empty
// rows, largest multiplication count summed over 64 consecutive rows.
// MODE 0: partial sums only.  MODE 2: also the per-row plan arrays
// (entries, saturated count, longest B row, column span) for tiled passes.
// gate (MODE 0, may be null): the longest row of A, already summed; when it
// exceeds gate_max the product takes the tiled path, whose plan computes
// these sums again, and every workgroup only passes the longest row on.
template <int MODE>
__global__ void __launch_bounds__(kBlock) k_features(Operands op, Features f, int64_t *partials, int64_t *err,
                                                     const int64_t *gate, int64_t gate_max) {
  __shared__ int64_t s_sum[4][kWavesPerBlock];
  if (MODE == 0 && gate && *gate > gate_max) {
    if (threadIdx.x < 4) partials[blockIdx.x * 4 + threadIdx.x] = threadIdx.x == 1 ? *gate : 0;
    return;
  }
  const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  // arrays sized by the descriptors' nnz rely on it
  if (i == 0 && (op.a_rp[op.rows] != op.a_nnz || op.b_rp[op.b_rows] != op.b_nnz))
    atomicOr((unsigned long long *)err, (unsigned long long)kErrDescriptor);
  int64_t ub = 0, m = 0, empty = 0;
  int32_t mx, lo, hi;
  wave_row_features<MODE == 2>(op, i, i < op.rows, m, ub, mx, lo, hi, f.brow);
  if (i < op.rows) {
    if (MODE == 2) {
      f.nnz_a[i] = (int32_t)m;
      f.ub[i] = (int32_t)min(ub, (int64_t)op.b_cols);
      f.maxb[i] = mx;
      f.lo[i] = lo;
      f.hi[i] = hi;
    }
    empty = ub == 0 ? 1 : 0;
  }
  // each wave's 64 rows are a merge wave's rows: its summed counts is the
  // staging the bound sizer gives that wave
  const int64_t ws = wave_sum(ub), we = wave_sum(empty), wm = wave_max64(m);
  if (lane_id() == 0) {
    s_sum[0][threadIdx.x / kWave] = ws;
    s_sum[1][threadIdx.x / kWave] = wm;
    s_sum[2][threadIdx.x / kWave] = we;
    s_sum[3][threadIdx.x / kWave] = ws;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    const int q = threadIdx.x;
    const bool is_max = q == 1 || q == 3;
    int64_t t = 0;
    for (int j = 0; j < kWavesPerBlock; ++j) t = is_max ? max(t, s_sum[q][j]) : t + s_sum[q][j];
    partials[blockIdx.x * 4 + q] = t;
  }
}

// Length, first and last column of every row of B in one 16-byte record
// (the span pass gathers one record per stored entry of A).
__global__ void __launch_bounds__(kBlock) k_brow_ends(const int64_t *b_rp, const int32_t *b_col, int64_t b_rows,
                                                      int4 *brow) {
  for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < b_rows; k += (int64_t)gridDim.x * kBlock) {
    const int64_t s = b_rp[k], e = b_rp[k + 1];
    brow[k] = e > s ? make_int4((int32_t)(e - s), b_col[s], b_col[e - 1], 0) : make_int4(0, 0x7fffffff, -1, 0);
  }
}

hipError_t launch_brow_ends(const Operands &op, Features f, hipStream_t s) {
  if (op.b_rows <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((op.b_rows + kBlock - 1) / kBlock, 1 << 16);
  hipLaunchKernelGGL(k_brow_ends, dim3((unsigned)blocks), dim3(kBlock), 0, s, op.b_rp, op.b_col, op.b_rows,
                     reinterpret_cast<int4 *>(f.brow));
  return hipGetLastError();
}

// Longest row of A (row pointers only); also checks that the descriptors'
// entry counts equal row_ptr[rows] (arrays sized by nnz rely on it).
__global__ void __launch_bounds__(kBlock) k_row_max(Operands op, int64_t *partials, int64_t *err) {
  const int64_t *rp = op.a_rp;
  const int64_t rows = op.rows;
  if (blockIdx.x == 0 && threadIdx.x == 0 && (op.a_rp[op.rows] != op.a_nnz || op.b_rp[op.b_rows] != op.b_nnz))
    atomicOr((unsigned long long *)err, (unsigned long long)kErrDescriptor);
  int64_t m = 0;
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < rows; i += (int64_t)gridDim.x * kBlock)
    m = max(m, rp[i + 1] - rp[i]);
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) m = max(m, __shfl_xor(m, d, kWave));
  __shared__ int64_t red[kWavesPerBlock];
  if (lane_id() == 0) red[threadIdx.x / kWave] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int j = 0; j < kWavesPerBlock; ++j) t = max(t, red[j]);
    partials[blockIdx.x] = t;
  }
}

// Adds (or takes the max of) per-workgroup partials in a fixed order and
// stores the results in counters[dst[j]]: one workgroup, no contended
// atomics.  Partial j of workgroup b is partials[b * stride + j].
constexpr int kMaxPartials = 10;
constexpr int kSizeParts = 9;   // partial sums of the sizing kernel per workgroup
struct PartialSpec {
  int32_t n, stride;
  int32_t dst[kMaxPartials];
  int32_t is_max[kMaxPartials];
};

constexpr int kSumThreads = 1024;
constexpr int kSumWaves = kSumThreads / kWave;
__global__ void __launch_bounds__(kSumThreads) k_sum_partials(const int64_t *partials, int64_t nblocks, PartialSpec ps,
                                                              int64_t *counters) {
  __shared__ int64_t red[kMaxPartials][kSumWaves];
  // strides follow the launch's width (at most kSumThreads threads); each
  // sum's records eight at a time, their loads issued together
  const int64_t nt = blockDim.x;
  int64_t acc[kMaxPartials];
#pragma unroll
  for (int j = 0; j < kMaxPartials; ++j) acc[j] = 0;
  for (int64_t b0 = threadIdx.x; b0 < nblocks; b0 += 8 * nt) {
#pragma unroll
    for (int j = 0; j < kMaxPartials; ++j) {
      if (j >= ps.n) continue;
      int64_t v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t b = b0 + (int64_t)u * nt;
        v[u] = b < nblocks ? partials[b * ps.stride + j] : 0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[j] = ps.is_max[j] ? max(acc[j], v[u]) : acc[j] + v[u];
    }
  }
#pragma unroll
  for (int j = 0; j < kMaxPartials; ++j) {
    if (j >= ps.n) continue;
    int64_t a = acc[j];
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
      const int64_t o = __shfl_xor(a, d, kWave);
      a = ps.is_max[j] ? max(a, o) : a + o;
    }
    if (lane_id() == 0) red[j][threadIdx.x / kWave] = a;
  }
  __syncthreads();
  if (threadIdx.x < ps.n) {
    int j = threadIdx.x;
    int64_t acc = 0;
    for (int q = 0; q < (int)(nt / kWave); ++q) acc = ps.is_max[j] ? max(acc, red[j][q]) : acc + red[j][q];
    counters[ps.dst[j]] = acc;
  }
}

// Many partials are first folded kFold to one by as many workgroups (one
// record per thread), into the space after them, so that the final
// single-workgroup sum reads a few hundred records.
constexpr int64_t kFold = kBlock;
constexpr int64_t kFoldAbove = 4096;

__global__ void __launch_bounds__(kBlock) k_fold_partials(const int64_t *partials, int64_t nblocks, PartialSpec ps,
                                                          int64_t *out) {
  __shared__ int64_t red[kMaxPartials][kWavesPerBlock];
  const int64_t b = (int64_t)blockIdx.x * kFold + threadIdx.x;
#pragma unroll
  for (int j = 0; j < kMaxPartials; ++j) {
    if (j >= ps.n) continue;
    int64_t a = b < nblocks ? partials[b * ps.stride + j] : 0;
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
      const int64_t o = __shfl_xor(a, d, kWave);
      a = ps.is_max[j] ? max(a, o) : a + o;
    }
    if (lane_id() == 0) red[j][threadIdx.x / kWave] = a;
  }
  __syncthreads();
  if (threadIdx.x < ps.n) {
    const int j = threadIdx.x;
    int64_t acc = 0;
    for (int q = 0; q < kWavesPerBlock; ++q) acc = ps.is_max[j] ? max(acc, red[j][q]) : acc + red[j][q];
    out[(int64_t)blockIdx.x * ps.stride + j] = acc;
  }
}

// partials: every producer's array has room for the folded records after
// its own (at most 9 words per workgroup in an array of 10 per workgroup).
hipError_t launch_sum_partials(const int64_t *partials, int64_t nblocks, int n, int stride, const int32_t *dst,
                               const int32_t *is_max, int64_t *counters, hipStream_t s) {
  PartialSpec ps{};
  ps.n = n;
  ps.stride = stride;
  for (int j = 0; j < n; ++j) {
    ps.dst[j] = dst[j];
    ps.is_max[j] = is_max ? is_max[j] : 0;
  }
  if (nblocks > kFoldAbove) {
    int64_t *folded = const_cast<int64_t *>(partials) + nblocks * stride;
    const int64_t g = (nblocks + kFold - 1) / kFold;
    hipLaunchKernelGGL(k_fold_partials, dim3((unsigned)g), dim3(kBlock), 0, s, partials, nblocks, ps, folded);
    partials = folded;
    nblocks = g;
  }
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kSumThreads), 0, s, partials, nblocks, ps, counters);
  return hipGetLastError();
}

hipError_t launch_features(const Operands &op, const Features &f, int64_t *counters, int64_t *partials, int mode,
                           hipStream_t s, const int64_t *gate, int64_t gate_max) {
  const int32_t dst[4] = {kCtrMults, kCtrMaxA, kCtrEmpty, kCtrWaveCap};
  const int32_t mx[4] = {0, 1, 0, 1};
  if (op.rows <= 0) {
    for (int q = 0; q < 4; ++q) {
      hipError_t e = launch_fill_i64(counters + dst[q], 0, 1, s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  const int64_t blocks = (op.rows + kBlock - 1) / kBlock;
  int64_t *err = counters + kCtrError;
  if (mode == 2)
    hipLaunchKernelGGL(k_features<2>, dim3((unsigned)blocks), dim3(kBlock), 0, s, op, f, partials, err,
                       (const int64_t *)nullptr, (int64_t)0);
  else
    hipLaunchKernelGGL(k_features<0>, dim3((unsigned)blocks), dim3(kBlock), 0, s, op, f, partials, err, gate,
                       gate_max);
  return launch_sum_partials(partials, blocks, 4, 4, dst, mx, counters, s);
}

hipError_t launch_row_max(const Operands &op, int64_t *counters, int64_t *partials, hipStream_t s) {
  const int64_t rows = op.rows;
  if (rows <= 0) return launch_fill_i64(counters + kCtrMaxA, 0, 1, s);
  const int64_t blocks = std::min<int64_t>(1024, (rows + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_row_max, dim3((unsigned)blocks), dim3(kBlock), 0, s, op, partials, counters + kCtrError);
  const int32_t dst[1] = {kCtrMaxA};
  const int32_t mx[1] = {1};
  return launch_sum_partials(partials, blocks, 1, 1, dst, mx, counters, s);
}

// ------------------------------------------------------------ sizing/tiers
// Device table of a workgroup-tier row: capacity c, load <= 1/2, and c
// slots of probe room so that linear probing can never run off the end; a
// dense window when the column region is at most `ratio` times the capacity
// (the paper's "Combined" rule of Section IV-B: MinMax when the region is
// smaller than twice the row's entries, Sort otherwise; the ratio is a
// tuning parameter, 2 by default).
__device__ __forceinline__ int64_t global_table_alloc(int64_t span, int64_t c, float ratio, bool *dense,
                                                       int64_t *slots) {
  if ((double)span <= (double)ratio * (double)c) {
    *dense = true;
    *slots = span;
    return span;
  }
  *dense = false;
  *slots = max((int64_t)16, 2 * c);
  return *slots + c;
}

// Slots global_table_alloc takes for any capacity up to c (a smaller exact
// count may trade a dense window for a hashed table); a dense window is at
// most `cols` slots.
__device__ __forceinline__ int64_t global_table_bound(int64_t c, float ratio, int64_t cols) {
  const double d = min((double)ratio * (double)c, (double)cols);
  return max(3 * c + 16, (int64_t)ceil(d));
}

constexpr int64_t kSortMax = 1024;   // keys a wave sorts in registers (64 lanes x 16)
constexpr int64_t kEscMax = 1024;   // products of an expand-sort row (64 lanes x 16)
constexpr int64_t kEscMaxSmall = 512;  // ... in launches compiled without the 16-per-lane sort
constexpr int64_t kSortCountMax = 256;  // slots of a row counted by sorting (64 lanes x 4)

// Smallest power of two >= x, at least kMinTable.
__device__ __forceinline__ int64_t table_pow2(int64_t x) {
  int64_t t = kMinTable;
  while (t < x) t <<= 1;
  return t;
}

// Tier, capacity and tile cost of every row for one pass.
//   capacity c: the multiplication count (symbolic, upper-bound sizer), the
//     exact count (numeric pass of the two-pass path) or the learned
//     capacity (learned sizer);
//   EMPTY  when the row has no products;
//   MERGE  when the A row has at most merge_lists entries and c <= merge_max;
//   HASH   when the wave's LDS table holds the row: a dense window of the
//          column region when it is at most dense_ratio * c (and fits), else
//          a power-of-two table with load <= 1/2 (symbolic: 2 * bound;
//          numeric: 2 * exact count; one pass: above the bound and at least
//          2 * capacity, so it can never fill, or just above the bound when
//          that is too large);
//   GLOBAL otherwise (a workgroup per row, table in device memory); these
//          rows are listed in pa.big.
// Tile cost (staged entries) bounds what a wave tile stages in LDS:
// min(c, HT) with HT = stage / 2, at least ceil(HT / 64) so a tile holds at
// most 64 rows.  The symbolic pass stages nothing: cost 1, tiles of 64 rows.
// The numeric pass stages merge rows only (hashed rows know their place in
// C and go there directly).
__global__ void __launch_bounds__(kBlock) k_size_rows(Operands op, PlanArrays pa, SizeParams sp) {
  __shared__ int64_t s_red[kSizeParts][kWavesPerBlock];
  const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  const bool sym = sp.mode == kSymbolic;
  const int64_t HT = sym ? kWave : sp.stage / 2;
  const int64_t mincost = sym ? 1 : (HT + kWave - 1) / kWave;
  int64_t n_tier[4] = {0, 0, 0, 0};
  int64_t capsum = 0, scratch = 0, tmax = 0;
  bool big = false, staged = false, esc_row = false;
  if (i < op.rows) {
    const int32_t m = pa.f.nnz_a[i];
    const int64_t ub = pa.f.ub[i];
    const int64_t mx = pa.f.maxb[i];
    int64_t c;
    if (sp.mode == kNumeric) c = sp.cnt[i];
    else if (sp.mode == kOnePass && sp.sizer == 2) c = learned_capacity(sp.pred[i], (int32_t)ub, (int32_t)mx, sp.margin, sp.slack);
    else c = ub;
    uint32_t tier, info;
    int64_t cost = mincost;
    if (m == 0 || ub == 0 || c == 0) {
      tier = kTierEmpty;
      c = 0;
      info = pack_info(kTierEmpty, false, 0);
    } else if (m <= sp.merge_lists && c <= sp.merge_max) {
      tier = kTierMerge;
      info = pack_info(kTierMerge, false, 0);
      if (!sym) {
        cost = max(min(c, HT), mincost);
        staged = !sp.merge_apart;
      }
    } else {
      const int64_t span = (int64_t)pa.f.hi[i] - (int64_t)pa.f.lo[i] + 1;
      bool dense = false;
      int64_t T;
      if ((double)span <= (double)sp.dense_ratio * (double)c && span <= sp.table_max) {
        dense = true;
        T = span;
      } else {
        // the bound one pass sizes its tables so that they never fill; the
        // learned one sizes them like the numeric pass, by the predicted size
        // (the capacity without its margin), and a row whose table fills is
        // computed again by the exact path
        const bool learned1 = sp.mode == kOnePass && sp.sizer == 2;
        const float pf = learned1 ? sp.pred[i] : 0.0f;
        const int64_t pc = (pf >= 0.0f && pf <= (float)ub) ? (int64_t)ceilf(pf) : ub;
        const int64_t ct = learned1 ? min(max(pc, mx), ub) : c;
        const int64_t need = sym ? 2 * ub : ((sp.mode == kNumeric || learned1) ? 2 * ct : max(ub + 1, 2 * c));
        T = table_pow2(need);
        // one pass: a table just above the bound still never fills (the
        // load is high only where the capacity is close to the bound)
        if (sp.mode == kOnePass && T > sp.table_max) T = table_pow2(ub + 1);
      }
      bool esc = false;
      if (sym && !dense && mx <= kWave) {
        // counting: the row's columns in blocks of pow2(mx) per entry of A,
        // sorted; T slots hold the blocks
        int64_t P = 1;
        while (P < mx) P <<= 1;
        const int64_t te = table_pow2((int64_t)m * P);
        if ((int64_t)m * P <= kSortCountMax && te <= sp.table_max) {
          esc = true;
          T = te;
        }
      }
      // rows whose products rarely share a column (the bound, not
      // saturated, within a quarter of the count or the capacity), whose B
      // rows fit one wave and whose column offsets pack with a product index
      // into one word: expand, sort, combine (T slots hold the products).
      // Rows of more than kEscMaxSmall products only where merge rows run
      // apart: the tile launch is then a variant without the merge code, which
      // has the registers for the 16-per-lane sort
      if (!dense && !sym && mx <= kWave && ub <= (sp.merge_apart ? kEscMax : kEscMaxSmall) && ub < op.b_cols &&
          4 * ub <= 5 * c) {
        const int64_t te = table_pow2(ub);
        if (te <= sp.table_max && (((int64_t)op.b_cols - pa.f.lo[i]) << __builtin_ctzll((uint64_t)te)) < ((int64_t)1 << 31)) {
          esc = true;
          T = te;
        }
      }
      // a hashed (not dense) row's keys are sorted in the wave's registers:
      // at most kSortMax of them (a table holds at most T)
      const int64_t most = sym ? 0 : (sp.mode == kNumeric ? c : min(ub, T));
      if (sp.table_max > 0 && T <= sp.table_max && (dense || most <= kSortMax)) {
        tier = kTierHash;
        info = pack_info(kTierHash, dense, (uint32_t)T, esc);
        esc_row = esc;
        tmax = T;
        // small hashed rows are staged; larger ones and expand-sort rows are
        // written straight to C (or the padded buffer of the one pass)
        if (!sym && !esc && c <= sp.stage_row_max) {
          cost = max(min(c, HT), mincost);
          staged = true;
        }
        // the numeric pass has a smaller (values) table: a row it may send
        // to the workgroup tier gets its device table counted already
        if (sym && (table_pow2(2 * ub) > sp.value_table_max || ub > kSortMax) &&
            !((double)span <= (double)sp.dense_ratio * (double)mx && span <= sp.value_table_max))
          scratch = global_table_bound(ub, sp.dense_ratio, op.b_cols);
      } else {
        tier = kTierGlobal;
        info = pack_info(kTierGlobal, false, 0);
        big = true;
        scratch = global_table_bound(sp.mode == kNumeric ? c : ub, sp.dense_ratio, op.b_cols);
      }
    }
    // learned one pass: any row may outgrow its capacity and be computed by
    // a workgroup with a device table sized by its exact count (<= bound)
    if (sp.mode == kOnePass && sp.sizer == 2 && tier != kTierEmpty)
      scratch = max(scratch, global_table_bound(ub, sp.dense_ratio, op.b_cols));
    pa.info[i] = info;
    pa.cap[i] = (int32_t)c;
    pa.cost[i] = cost;
    n_tier[tier] = 1;
    capsum = c;
  }
  // workgroup-tier rows: rows of many products at the front of the list
  // (their workgroups start first), the others from its end; one atomic per
  // wave and kind
  const uint64_t bm = ballot(big);
  if (bm) {
    const bool huge = big && (int64_t)pa.f.ub[i] >= kHugeWork;
    const uint64_t hb = ballot(huge), rb = bm & ~hb;
    int64_t hbase = 0, rbase = 0;
    if (lane_id() == 0) {
      atomicAdd((unsigned long long *)&pa.counters[kCtrGlobal], (unsigned long long)__popcll(bm));
      if (hb) hbase = (int64_t)atomicAdd((unsigned long long *)&pa.counters[kCtrHuge], (unsigned long long)__popcll(hb));
      if (rb) rbase = (int64_t)atomicAdd((unsigned long long *)&pa.counters[kCtrBigTail], (unsigned long long)__popcll(rb));
    }
    hbase = __shfl(hbase, 0, kWave);
    rbase = __shfl(rbase, 0, kWave);
    if (huge) pa.big[hbase + __popcll(hb & lanemask_lt())] = (int32_t)i;
    else if (big) pa.big[op.rows - 1 - (rbase + __popcll(rb & lanemask_lt()))] = (int32_t)i;
  }
  const int w = threadIdx.x / kWave;
  // workgroups that may want a table: one per row, one per part of a
  // split huge row
  // sums, except the two maxima (scratch, tmax) at 6 and 7
  const int64_t want = scratch > 0 ? ((big && (int64_t)pa.f.ub[i] >= kSplitWork) ? kSplitParts : 1) : 0;
  int64_t v[kSizeParts] = {n_tier[kTierMerge], n_tier[kTierHash], n_tier[kTierEmpty], capsum, want,
                           staged ? 1 : 0, scratch, tmax,
                           esc_row ? 1 + ((int64_t)pa.f.ub[i] > kEscMaxSmall ? ((int64_t)1 << 32) : 0) : 0};
#pragma unroll
  for (int j = 0; j < kSizeParts; ++j) {
    int64_t t = v[j];
    if (j == 6 || j == 7) {
#pragma unroll
      for (int d = kWave / 2; d > 0; d >>= 1) t = max(t, __shfl_xor(t, d, kWave));
    } else {
      t = wave_sum(t);
    }
    if (lane_id() == 0) s_red[j][w] = t;
  }
  __syncthreads();
  // one partial per workgroup; k_sum_partials adds them (no hot atomics)
  if (threadIdx.x < kSizeParts) {
    const int j = threadIdx.x;
    const bool mx_j = j == 6 || j == 7;
    int64_t t = 0;
    for (int q = 0; q < kWavesPerBlock; ++q) t = mx_j ? max(t, s_red[j][q]) : t + s_red[j][q];
    pa.partials[(int64_t)blockIdx.x * kSizeParts + j] = t;
  }
}

hipError_t launch_size_rows(const Operands &op, const PlanArrays &pa, const SizeParams &sp,
                            hipStream_t s) {
  PartialSpec ps{};
  ps.n = kSizeParts;
  ps.stride = kSizeParts;
  const int32_t dst[kSizeParts] = {kCtrMerge,       kCtrHash,   kCtrEmpty,   kCtrCapSum, kCtrScratchRows,
                                   kCtrStaged,      kCtrScratch, kCtrTable,  kCtrEsc};
  for (int j = 0; j < kSizeParts; ++j) {
    ps.dst[j] = dst[j];
    ps.is_max[j] = (j == 6 || j == 7);
  }
  hipError_t e = launch_fill_i64(pa.counters + kCtrGlobal, 0, 1, s);
  if (e == hipSuccess) e = launch_fill_i64(pa.counters + kCtrHuge, 0, 2, s);
  if (e != hipSuccess) return e;
  if (op.rows <= 0) {
    e = launch_fill_i64(pa.partials, 0, kSizeParts, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kSumThreads), 0, s, (const int64_t *)pa.partials, (int64_t)1,
                       ps, pa.counters);
    return hipGetLastError();
  }
  const int64_t blocks = (op.rows + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_size_rows, dim3((unsigned)blocks), dim3(kBlock), 0, s, op, pa, sp);
  hipError_t e2 = hipGetLastError();
  if (e2 != hipSuccess) return e2;
  int32_t mx[kSizeParts];
  for (int j = 0; j < kSizeParts; ++j) mx[j] = ps.is_max[j];
  return launch_sum_partials(pa.partials, blocks, kSizeParts, kSizeParts, ps.dst, mx, pa.counters, s);
}


// ------------------------------------------------------------------- scan
// Single-pass exclusive scan with decoupled look-back: each workgroup takes
// a ticket, loads 8192 items (coalesced, through LDS), scans them,
// publishes its aggregate and looks back for its prefix.  out[n] receives
// the total.  Safe in place (in == out).
constexpr int kScanItems = 32;
constexpr int kScanTile = kBlock * kScanItems;

// group_max (may be null): the largest sum of 64 consecutive items starting
// at a multiple of 64 (a merge wave's output) is raised into it.
template <typename TIn>
__global__ void __launch_bounds__(kBlock) k_scan(const TIn *in, int64_t *out, int64_t n,
                                                  uint64_t *status, int64_t *ticket,
                                                  int64_t *total_dst, int64_t *err, int64_t *group_max) {
  __shared__ int64_t buf[kScanTile];
  __shared__ int64_t s_tile, s_excl;
  __shared__ int64_t s_wtot[kWavesPerBlock + 1];
  if (threadIdx.x == 0) s_tile = (int64_t)__hip_atomic_fetch_add((unsigned long long *)ticket, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  const int64_t t = s_tile;
  const int64_t base = t * kScanTile;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int64_t idx = base + k * kBlock + threadIdx.x;
    buf[k * kBlock + threadIdx.x] = idx < n ? (int64_t)in[idx] : 0;
  }
  __syncthreads();
  int64_t sum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) sum += buf[threadIdx.x * kScanItems + k];
  __shared__ int64_t s_gmax[kWavesPerBlock];
  if (group_max) {
    // threads 2g and 2g+1 hold the 64 items of group g of the tile
    static_assert(kScanItems * 2 == kWave, "a group of 64 items spans two threads");
    int64_t g = sum + __shfl_xor(sum, 1, kWave);
#pragma unroll
    for (int d = kWave / 2; d > 1; d >>= 1) g = max(g, __shfl_xor(g, d, kWave));
    if (lane_id() == 0) s_gmax[threadIdx.x / kWave] = g;
  }
  int64_t agg;
  int64_t excl = block_exclusive_sum(sum, s_wtot, &agg);   // its barriers also order s_gmax
  if (group_max && threadIdx.x == 0) {
    int64_t m = 0;
    for (int w = 0; w < kWavesPerBlock; ++w) m = max(m, s_gmax[w]);
    atomicMax((unsigned long long *)group_max, (unsigned long long)m);
  }
  if (threadIdx.x < kWave) {
    int64_t pre = lookback_exclusive(status, t, agg, err, kErrLookback);
    if (threadIdx.x == 0) s_excl = pre;
  }
  __syncthreads();
  int64_t run = s_excl + excl;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int64_t v = buf[threadIdx.x * kScanItems + k];
    buf[threadIdx.x * kScanItems + k] = run;
    run += v;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int64_t idx = base + k * kBlock + threadIdx.x;
    if (idx < n) out[idx] = buf[k * kBlock + threadIdx.x];
  }
  if (base + kScanTile >= n && threadIdx.x == 0) {
    // the tile holding item n-1 also writes the total
    int64_t tot = s_excl + agg;
    out[n] = tot;
    if (total_dst) *total_dst = tot;
  }
}

// Clears the look-back status words and the ticket in one launch.
__global__ void k_scan_reset(uint64_t *status, int64_t tiles, int64_t *ticket, int64_t *group_max) {
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < tiles; i += (int64_t)gridDim.x * kBlock)
    status[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *ticket = 0;
    if (group_max) *group_max = 0;
  }
}

hipError_t launch_scan_i32(const int32_t *in, int64_t *out, int64_t n, uint64_t *status,
                           int64_t *ticket, int64_t *total_dst, int64_t *err, hipStream_t s,
                           int64_t *group_max) {
  if (n <= 0) {
    if (group_max) {
      hipError_t e = launch_fill_i64(group_max, 0, 1, s);
      if (e != hipSuccess) return e;
    }
    return launch_fill_i64(out, 0, 1, s);
  }
  int64_t tiles = (n + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(k_scan_reset, dim3(grid_for(tiles, 1024)), dim3(kBlock), 0, s, status, tiles, ticket, group_max);
  hipLaunchKernelGGL(k_scan<int32_t>, dim3((unsigned)tiles), dim3(kBlock), 0, s, in, out, n, status,
                     ticket, total_dst, err, group_max);
  return hipGetLastError();
}

hipError_t launch_scan_i64_inplace(int64_t *inout, int64_t n, uint64_t *status, int64_t *ticket,
                                   int64_t *err, hipStream_t s) {
  if (n <= 0) return launch_fill_i64(inout, 0, 1, s);
  int64_t tiles = (n + kScanTile - 1) / kScanTile;
  hipError_t e = launch_fill_u64(status, 0, tiles, s);
  if (e != hipSuccess) return e;
  e = launch_fill_i64(ticket, 0, 1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan<int64_t>, dim3((unsigned)tiles), dim3(kBlock), 0, s, inout, inout, n,
                     status, ticket, (int64_t *)nullptr, err, (int64_t *)nullptr);
  return hipGetLastError();
}

// ------------------------------------------------------------ tile bounds
// Row i belongs to tile floor(prefix_i / HT), prefix_i the exclusive prefix
// of the tile costs.  A row's cost is at most HT, so a tile holds at most
// 2*HT worth of rows; tiles skipped by a large row stay empty.
__global__ void k_tile_bounds(const int64_t *cost, int64_t rows, int64_t HT, int32_t *tile_row,
                              int64_t *counters) {
  int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i >= rows) return;
  int64_t q = cost[i] / HT;
  int64_t qp = i == 0 ? -1 : cost[i - 1] / HT;
  for (int64_t t = qp + 1; t <= q; ++t) tile_row[t] = (int32_t)i;
  if (i == rows - 1) {
    tile_row[q + 1] = (int32_t)rows;
    counters[kCtrTiles] = q + 1;
  }
}

hipError_t launch_tile_bounds(const int64_t *cost, int64_t rows, int64_t HT, int32_t *tile_row,
                              int64_t *counters, hipStream_t s) {
  if (rows <= 0) return launch_fill_i64(counters + kCtrTiles, 0, 1, s);
  hipLaunchKernelGGL(k_tile_bounds, dim3((unsigned)((rows + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                     cost, rows, HT, tile_row, counters);
  return hipGetLastError();
}

// ============================================================ row kernels
// Monotone hash: home slot of column j in a row whose columns lie in
// [lo, lo + span).  Dense window: slot = j - lo.  Hashed: slot =
// floor((j - lo) * scale / 2^32) with scale = floor(T * 2^32 / span), which
// never decreases with j.  With linear probing, keys then sit in column
// order except where a probe pushed a key past larger ones; the extraction
// repairs that within the row's largest probe distance.
struct RowHash {
  int32_t lo;
  uint32_t scale;
  bool dense;
  __device__ __forceinline__ int32_t home(int32_t j) const {
    uint32_t x = (uint32_t)(j - lo);
    return dense ? (int32_t)x : (int32_t)__umulhi(x, scale);
  }
};

__device__ __forceinline__ RowHash make_hash(int32_t lo, int32_t hi, int64_t slots, bool dense) {
  RowHash h;
  h.lo = lo;
  h.dense = dense;
  int64_t span = (int64_t)hi - (int64_t)lo + 1;
  h.scale = dense ? 0u : (uint32_t)(((uint64_t)slots << 32) / (uint64_t)span);
  return h;
}

// --- register merge tier: one thread, up to M stored entries in the A row.
// The row of C is the union of the selected B rows, each sorted by column;
// the thread repeatedly takes the smallest head column and sums the heads
// carrying it in list order, i.e. in A's column order.  Output comes out
// sorted and every entry is accumulated exactly like the dense temporary of
// the row-major kernel.  Writes min(count, lim) entries; returns the count.
template <int M, bool VALUES, bool DBUF = true>
__device__ int64_t merge_row(const Operands &op, int64_t row, int32_t *out_col, double *out_val,
                             int64_t lim, int64_t *ub_out = nullptr, double *maxabs_out = nullptr) {
  const int64_t as = op.a_rp[row];
  const int m = (int)(op.a_rp[row + 1] - as);
  // per list: head (h, v), with DBUF the entry after it (h2, v2), the next
  // position to load and how many entries are left to load; with DBUF the
  // entry after the head is loaded one consumption ahead, so a list rarely
  // waits on a load (more registers: the tile kernel merges without it)
  int32_t h[M], h2[M];
  int64_t pos[M];
  int32_t rem[M];
  double a[M], v[M], v2[M];
#pragma unroll
  for (int l = 0; l < M; ++l) {
    rem[l] = 0;
    pos[l] = 0;
    a[l] = 0.0;
    if (l < m) {
      if (VALUES) a[l] = op.a_val[as + l];
      b_row_of(op, as + l, pos[l], rem[l]);
    }
  }
  if (ub_out) {
    int64_t ub = 0;
#pragma unroll
    for (int l = 0; l < M; ++l) ub += rem[l];
    *ub_out = ub;
  }
#pragma unroll
  for (int l = 0; l < M; ++l) {
    h[l] = rem[l] > 0 ? op.b_col[pos[l]] : kColMax;
    v[l] = (VALUES && rem[l] > 0) ? op.b_val[pos[l]] : 0.0;
    if (DBUF) {
      h2[l] = rem[l] > 1 ? op.b_col[pos[l] + 1] : kColMax;
      v2[l] = (VALUES && rem[l] > 1) ? op.b_val[pos[l] + 1] : 0.0;
      pos[l] += 2;
      rem[l] -= 2;
    } else {
      pos[l] += 1;
      rem[l] -= 1;
    }
  }
  int64_t n = 0;
  while (true) {
    int32_t mn = h[0];
#pragma unroll
    for (int l = 1; l < M; ++l) mn = min(mn, h[l]);
    if (mn == kColMax) break;
    double acc = 0.0;
#pragma unroll
    for (int l = 0; l < M; ++l) {
      if (h[l] == mn) {
        if (VALUES) acc = mul_add_rn(acc, a[l], v[l]);
        if (DBUF) {
          h[l] = h2[l];
          if (VALUES) v[l] = v2[l];
          h2[l] = rem[l] > 0 ? op.b_col[pos[l]] : kColMax;
          if (VALUES) v2[l] = rem[l] > 0 ? op.b_val[pos[l]] : 0.0;
        } else {
          h[l] = rem[l] > 0 ? op.b_col[pos[l]] : kColMax;
          if (VALUES) v[l] = rem[l] > 0 ? op.b_val[pos[l]] : 0.0;
        }
        ++pos[l];
        --rem[l];
      }
    }
    if (n < lim) {
      out_col[n] = mn;
      if (VALUES) out_val[n] = acc;
    }
    if (VALUES && maxabs_out) *maxabs_out = fmax(*maxabs_out, fabs(acc));
    ++n;
  }
  return n;
}

// --- LDS hash tier: G lanes per row.  A entries are taken in stored order;
// for each, the G lanes cover the B row.  Columns of one B row are distinct,
// so within a step no two lanes touch the same slot, and steps run in
// program order inside the wave: every slot is updated in A's column order
// with plain loads and stores (no floating-point atomics).
// Order repair.  With the monotone hash and linear probing, a maximal run
// of occupied slots holds exactly the keys whose home lies in the run, and
// every key of an earlier run is smaller than every key of a later one; only
// inside a run can probing have put a key after a larger one.  Sorting each
// run in place (insertion sort, one lane per run; runs are disjoint) makes
// the whole table sorted in slot order, so a key's rank is the number of
// occupied slots before it.  Tables where no key was displaced are sorted
// already.
// A workgroup's device table is its own (one region of the scratch per
// workgroup): its accesses are atomics at workgroup scope, which keep the
// waves of the workgroup coherent through the CU's L1 instead of going to
// L2 for every access.
__device__ __forceinline__ int32_t gload(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// Two neighbouring keys (8-byte aligned) in one load.
__device__ __forceinline__ uint64_t gload64(const int32_t *p) {
  return __hip_atomic_load(reinterpret_cast<const uint64_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ double gloadd(const double *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void gstored(double *p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void gstore(int32_t *p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ int32_t gcas(int32_t *p, int32_t expected, int32_t desired) {
  __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
  return expected;
}
// The table's writes before the barrier are seen by every wave of the
// workgroup after it.
__device__ __forceinline__ void wg_sync_global() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
}

// Write the sorted row held by an LDS table (G lanes).
struct WgScratch {
  int64_t pref[kBlock + 1];
  int64_t bs[kBlock];
  double av[kBlock];
  int64_t wtot[kWavesPerBlock + 1];
  int32_t cnt, dmax;
  int32_t top;   // numeric: the highest slot a key was inserted at
  int64_t run;
  int32_t first;   // extraction: the end of a chunk
};

// Extraction staging of the workgroup tier (see wg_extract_chunked); free
// while the table is built, when it holds the LDS sets of the ordered
// accumulation.
constexpr int kExtChunk = 2048, kExtPad = 256;
struct ExtLds {
  int32_t k[kExtChunk + kExtPad];
  double v[kExtChunk + kExtPad];
};

// Waits until this wave's outstanding memory operations have completed (no
// cache write-back or invalidation): the device-table updates of one
// sub-step are in L2 before the next sub-step reads them.
__device__ __forceinline__ void wave_mem_wait() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Stores of C, which the product writes once and does not read back:
// non-temporal (streaming) stores.  NT false: plain stores (LDS staging or
// the one pass's padded buffer).  The choice is made at compile time: a
// branch between the two kinds lets the compiler merge the stores and drop
// the non-temporal hint.
template <bool NT = true>
__device__ __forceinline__ void put_c(int32_t *col, double *val, int64_t i, int32_t c, double v) {
  if constexpr (NT) {
    __builtin_nontemporal_store(c, col + i);
    __builtin_nontemporal_store(v, val + i);
  } else {
    col[i] = c;
    val[i] = v;
  }
}

// Orders the LDS accesses of the lanes of one wave (a wave's LDS
// instructions execute in issue order): a fence at wavefront scope keeps the
// compiler from moving memory operations across, without waiting for
// outstanding global loads.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Workgroup-tier passes take the row's products in steps of kWgChunk, in
// A's stored order (entries of A 256 at a time, their B rows enumerated
// flat): thread t holds products q0 + u * kBlock + t for u < kWgProducts, so
// that the gathers and table probes of its kWgProducts products are in
// flight together.
constexpr int kWgProducts = 4;
constexpr int kWgChunk = kBlock * kWgProducts;
constexpr int kDupBits = 11;
constexpr int kDupSlots = 1 << kDupBits;   // LDS set of one step's columns (2 x kWgChunk)
static_assert(kDupSlots == 2 * kWgChunk, "set size");
static_assert(sizeof(ExtLds::v) / 4 >= kDupSlots, "LDS set");

// Stages the next (at most) 256 entries of A from eb: the exclusive sums of
// their B rows' lengths (those of columns in [c0, c1); c1 < 0: all), the B
// row starts and the A values.  Returns the batch's product count.  The
// caller synchronises before restaging.
__device__ __forceinline__ int64_t wg_stage_entries(const Operands &op, int64_t eb, int64_t ae, int32_t c0,
                                                    int32_t c1, WgScratch &ws, bool values) {
  const int64_t e = eb + threadIdx.x;
  int64_t bs = 0, bl = 0;
  double av = 0.0;
  if (e < ae) {
    av = values && op.a_val ? op.a_val[e] : 0.0;
    int32_t l;
    b_row_part(op, e, c0, c1, bs, l);
    bl = l;
  }
  int64_t tot;
  const int64_t ex = block_exclusive_sum(bl, ws.wtot, &tot);
  ws.pref[threadIdx.x] = ex;
  ws.bs[threadIdx.x] = bs;
  ws.av[threadIdx.x] = av;
  __syncthreads();
  return tot;
}

// This thread's products of the step at q0 of a staged batch of tot
// products: B positions and A values (live[u] false past the batch).
__device__ __forceinline__ void wg_step_products(const WgScratch &ws, int64_t q0, int64_t tot, int64_t *bpos,
                                                 double *av, bool *live) {
#pragma unroll
  for (int u = 0; u < kWgProducts; ++u) {
    const int64_t q = q0 + u * kBlock + threadIdx.x;
    live[u] = q < tot;
    bpos[u] = 0;
    av[u] = 0.0;
    if (live[u]) {
      int lo = 0, hi = kBlock - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ws.pref[mid] <= q) lo = mid;
        else hi = mid - 1;
      }
      bpos[u] = ws.bs[lo] + (q - ws.pref[lo]);
      av[u] = ws.av[lo];
    }
  }
}

// Inserts the keys j[u] (where go[u]) into the device table: slot[u] is the
// key's slot, fresh[u] whether this call claimed it.  The first probes of
// the thread's keys are issued together; a key displaced further probes on
// one slot at a time.  The table has room for every product, so no probe
// leaves it; one that would sets *full (reported, never dropped silently).
template <bool GROUP>
__device__ __forceinline__ void global_insert_n(int32_t *keys, int64_t alloc, const RowHash &hs, const int32_t *j,
                                                const bool *go, int64_t *slot, bool *fresh, int32_t &dmax,
                                                bool &full, int32_t *top = nullptr) {
  int32_t old[kWgProducts];
#pragma unroll
  for (int u = 0; u < kWgProducts; ++u) {
    slot[u] = go[u] ? hs.home(j[u]) : 0;
    old[u] = go[u] ? gcas(&keys[slot[u]], kEmpty, j[u]) : kEmpty;
  }
#pragma unroll
  for (int u = 0; u < kWgProducts; ++u) {
    fresh[u] = false;
    if (!go[u]) continue;
    if (old[u] == kEmpty) {
      fresh[u] = true;
      continue;
    }
    if (old[u] == j[u]) continue;
    const int64_t h = slot[u];
    int64_t sl = h + 1;
    bool done = false;
    while (!done && sl < alloc) {
      // the keys from slot sl to the end of its aligned group of four, read
      // at once (a key once set never changes, so a stale read can only show
      // a slot as empty, which the compare-and-swap then settles)
      const int64_t g = GROUP ? sl & ~(int64_t)3 : sl;
      int32_t kv[4];
      if (!GROUP) {
        kv[0] = kEmpty;   // one slot at a time: straight to the compare-and-swap
      } else if (g + 4 <= alloc) {
        const uint64_t w0 = gload64(keys + g), w1 = gload64(keys + g + 2);
        kv[0] = (int32_t)(uint32_t)w0;
        kv[1] = (int32_t)(uint32_t)(w0 >> 32);
        kv[2] = (int32_t)(uint32_t)w1;
        kv[3] = (int32_t)(uint32_t)(w1 >> 32);
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) kv[q] = g + q < alloc ? gload(keys + g + q) : kEmpty;
      }
      for (; sl < g + (GROUP ? 4 : 1) && sl < alloc; ++sl) {
        int32_t kq = kv[sl - g];
        if (kq == kEmpty) {
          kq = gcas(&keys[sl], kEmpty, j[u]);
          if (kq == kEmpty) {
            fresh[u] = true;
            done = true;
            break;
          }
        }
        if (kq == j[u]) {
          done = true;
          break;
        }
      }
    }
    if (sl >= alloc) {
      full = true;
      sl = h;   // never used: the row is reported
    }
    slot[u] = sl;
    dmax = max(dmax, (int32_t)(sl - h));
  }
  if (top) {
#pragma unroll
    for (int u = 0; u < kWgProducts; ++u)
      if (fresh[u]) *top = max(*top, (int32_t)slot[u]);
  }
}

// Publishes a pass's distinct-key count and largest displacement to ws.
__device__ __forceinline__ void wg_publish_keys(WgScratch &ws, int32_t nnew, int32_t dmax, bool full, int64_t *err,
                                                int32_t top = -1) {
  const int32_t wn = (int32_t)wave_sum((int64_t)nnew), wd = wave_max32(dmax), wt = wave_max32(top);
  const bool wf = ballot(full) != 0;
  if (lane_id() == 0) {
    if (wn) atomicAdd(&ws.cnt, wn);
    if (wd) atomicMax(&ws.dmax, wd);
    if (wt >= 0) atomicMax(&ws.top, wt);
    if (wf) atomicOr((unsigned long long *)err, (unsigned long long)kErrInconsistent);
  }
}

// Counting pass of a workgroup-tier row (or of the column range [c0, c1) of
// a split one): builds its key set in the table and returns its size.
__device__ int32_t wg_global_keys(const Operands &op, int64_t row, int32_t c0, int32_t c1, int32_t *keys,
                                  int64_t alloc, const RowHash &hs, WgScratch &ws, int64_t *err) {
  for (int64_t s = threadIdx.x; s < alloc; s += kBlock) gstore(keys + s, kEmpty);
  if (threadIdx.x == 0) {
    ws.cnt = 0;
    ws.dmax = 0;
  }
  wg_sync_global();
  int32_t nnew = 0, dmax = 0;
  bool full = false;
  const int64_t as = op.a_rp[row], ae = op.a_rp[row + 1];
  for (int64_t eb = as; eb < ae; eb += kBlock) {
    const int64_t tot = wg_stage_entries(op, eb, ae, c0, c1, ws, false);
    for (int64_t q0 = 0; q0 < tot; q0 += kWgChunk) {
      int64_t bpos[kWgProducts], slot[kWgProducts];
      double av[kWgProducts];
      bool live[kWgProducts], fresh[kWgProducts];
      int32_t j[kWgProducts];
      wg_step_products(ws, q0, tot, bpos, av, live);
#pragma unroll
      for (int u = 0; u < kWgProducts; ++u) j[u] = live[u] ? op.b_col[bpos[u]] : 0;
      global_insert_n<true>(keys, alloc, hs, j, live, slot, fresh, dmax, full);
#pragma unroll
      for (int u = 0; u < kWgProducts; ++u) nnew += fresh[u] ? 1 : 0;
    }
    __syncthreads();
  }
  wg_publish_keys(ws, nnew, dmax, full, err);
  wg_sync_global();
  return ws.cnt;
}

// One step's products applied in A's order.  `apply(go)` updates the
// targets of the products with go[u] set, whose columns are distinct, and
// waits for its stores; a barrier follows.  Columns that repeat within the
// step are found through the LDS set `dset` (kDupSlots cells, kEmpty between
// steps); such a step applies in rounds, in each of which the lowest-indexed
// pending product of every column applies (the minimum kept in the column's
// cell, INT32_MAX between rounds): as many rounds as the step's largest
// repeat count.  Every target thus receives its products in A's order.
template <typename Apply>
__device__ __forceinline__ void wg_apply_in_order(int32_t *dset, const bool *live, const int32_t *j, Apply apply) {
  const int t = threadIdx.x;
  int32_t cell[kWgProducts], at[kWgProducts];
  bool dup = false;
#pragma unroll
  for (int u = 0; u < kWgProducts; ++u) {
    at[u] = -1;
    cell[u] = 0;
    if (!live[u]) continue;
    uint32_t h = ((uint32_t)j[u] * 0x9E3779B1u) >> (32 - kDupBits);
    while (true) {
      const int32_t o = atomicCAS(&dset[h], kEmpty, j[u]);
      if (o == kEmpty) {
        at[u] = (int32_t)h;
        break;
      }
      if (o == j[u]) {
        dup = true;
        break;
      }
      h = (h + 1) & (kDupSlots - 1);
    }
    cell[u] = (int32_t)h;
  }
  const bool ordered = __syncthreads_or(dup ? 1 : 0) != 0;
  // the set's cells of this step's columns: free again, or (ordered) the
  // columns' round minima
#pragma unroll
  for (int u = 0; u < kWgProducts; ++u)
    if (at[u] >= 0) dset[at[u]] = ordered ? 0x7fffffff : kEmpty;
  if (!ordered) {
    apply(live);
    __syncthreads();
    return;
  }
  bool pend[kWgProducts];
#pragma unroll
  for (int u = 0; u < kWgProducts; ++u) pend[u] = live[u];
  while (true) {
    bool any = false;
#pragma unroll
    for (int u = 0; u < kWgProducts; ++u) any |= pend[u];
    if (!__syncthreads_or(any ? 1 : 0)) break;
#pragma unroll
    for (int u = 0; u < kWgProducts; ++u)
      if (pend[u]) atomicMin(&dset[cell[u]], u * kBlock + t);
    __syncthreads();
    bool go[kWgProducts];
#pragma unroll
    for (int u = 0; u < kWgProducts; ++u) go[u] = pend[u] && dset[cell[u]] == u * kBlock + t;
    apply(go);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kWgProducts; ++u)
      if (go[u]) {
        dset[cell[u]] = 0x7fffffff;
        pend[u] = false;
      }
  }
  // the last round's barrier has passed: free the cells before the next
  // step inserts
#pragma unroll
  for (int u = 0; u < kWgProducts; ++u)
    if (at[u] >= 0) dset[at[u]] = kEmpty;
  __syncthreads();
}

// Numeric pass of a workgroup-tier row (or of a column range): keys and
// values in one sweep over the products, in A's order (wg_apply_in_order):
// a slot claimed by a product starts at +0.0 + a*b, one claimed earlier
// adds a*b to what the earlier products left, so every entry of C sums its
// products in A's column order, as the row-major kernel does (Section
// IV-A).  Fast: every product at once, atomic adds into slots cleared to
// +0.0 (the summation order is then not fixed).  Returns the row's size.
__device__ int32_t wg_global_accumulate(const Operands &op, int64_t row, int32_t c0, int32_t c1, int32_t *keys,
                                        double *vals, int64_t alloc, const RowHash &hs, WgScratch &ws, ExtLds &xl,
                                        bool fast, int64_t *err) {
  const int t = threadIdx.x;
  int32_t *dset = reinterpret_cast<int32_t *>(xl.v);
  for (int64_t s = t; s < alloc; s += kBlock) {
    gstore(keys + s, kEmpty);
    if (fast) gstored(vals + s, 0.0);
  }
  for (int q = t; q < kDupSlots; q += kBlock) dset[q] = kEmpty;
  if (t == 0) {
    ws.cnt = 0;
    ws.dmax = 0;
    ws.top = -1;
  }
  wg_sync_global();
  int32_t nnew = 0, dmax = 0, top = -1;
  bool full = false;
  const int64_t as = op.a_rp[row], ae = op.a_rp[row + 1];
  for (int64_t eb = as; eb < ae; eb += kBlock) {
    const int64_t tot = wg_stage_entries(op, eb, ae, c0, c1, ws, true);
    for (int64_t q0 = 0; q0 < tot; q0 += kWgChunk) {
      int64_t bpos[kWgProducts], slot[kWgProducts];
      double a[kWgProducts], b[kWgProducts];
      bool live[kWgProducts], fresh[kWgProducts];
      int32_t j[kWgProducts];
      wg_step_products(ws, q0, tot, bpos, a, live);
#pragma unroll
      for (int u = 0; u < kWgProducts; ++u) {
        j[u] = live[u] ? op.b_col[bpos[u]] : 0;
        b[u] = live[u] ? op.b_val[bpos[u]] : 0.0;
      }
      if (fast) {
        global_insert_n<false>(keys, alloc, hs, j, live, slot, fresh, dmax, full, &top);
#pragma unroll
        for (int u = 0; u < kWgProducts; ++u) {
          nnew += fresh[u] ? 1 : 0;
          if (live[u] && !full) {
            double pr;
            {
#pragma clang fp contract(off)
              pr = a[u] * b[u];
            }
            atomicAdd(&vals[slot[u]], pr);
          }
        }
        continue;
      }
      wg_apply_in_order(dset, live, j, [&](const bool *go) {
        global_insert_n<false>(keys, alloc, hs, j, go, slot, fresh, dmax, full, &top);
        double old[kWgProducts];
#pragma unroll
        for (int u = 0; u < kWgProducts; ++u) old[u] = (go[u] && !fresh[u] && !full) ? gloadd(vals + slot[u]) : 0.0;
#pragma unroll
        for (int u = 0; u < kWgProducts; ++u) {
          if (!go[u] || full) continue;
          nnew += fresh[u] ? 1 : 0;
          gstored(vals + slot[u], fresh[u] ? first_add_rn(a[u], b[u]) : mul_add_rn(old[u], a[u], b[u]));
        }
        wave_mem_wait();
      });
    }
    __syncthreads();
  }
  wg_publish_keys(ws, nnew, dmax, full, err, top);
  wg_sync_global();
  return ws.cnt;
}

// Run sorting (see lds_sort_runs) on a device table, one thread per run.
__device__ void wg_sort_runs(int32_t *keys, double *vals, int64_t alloc) {
  for (int64_t s = threadIdx.x; s < alloc; s += kBlock) {
    if (gload(keys + s) == kEmpty || (s > 0 && gload(keys + s - 1) != kEmpty)) continue;
    for (int64_t q = s + 1; q < alloc; ++q) {
      const int32_t k = gload(keys + q);
      if (k == kEmpty) break;
      const double v = vals ? gloadd(vals + q) : 0.0;
      int64_t at = q;
      while (at > s) {
        const int32_t prev = gload(keys + at - 1);
        if (prev <= k) break;
        gstore(keys + at, prev);
        if (vals) gstored(vals + at, gloadd(vals + at - 1));
        --at;
      }
      gstore(keys + at, k);
      if (vals) gstored(vals + at, v);
    }
  }
  wg_sync_global();
}

// Sorted write-out through LDS, kExtChunk slots at a time: a chunk is read
// with coalesced loads (with kExtPad slots beyond it) and ends at the first
// empty slot at or after kExtChunk, so no run crosses chunks; its runs are
// sorted in LDS (one thread per run), and its occupied slots are compacted
// to the output.  Returns false, having written nothing final, when a run is
// longer than the pad (the caller then sorts the runs in device memory).

__device__ bool wg_extract_chunked(const int32_t *keys, const double *vals, int64_t alloc, WgScratch &ws,
                                   ExtLds &xl, int32_t *out_col, double *out_val, int64_t lim) {
  const int t = threadIdx.x;
  int64_t c0 = 0, run = 0;
  while (c0 < alloc) {
    const int n = (int)min((int64_t)(kExtChunk + kExtPad), alloc - c0);
    // every load of the chunk in flight before the first is stored
    constexpr int kLoadPer = (kExtChunk + kExtPad) / kBlock;
    static_assert(kLoadPer * kBlock == kExtChunk + kExtPad, "chunk loads");
    int32_t kk[kLoadPer];
    double vv[kLoadPer];
#pragma unroll
    for (int u = 0; u < kLoadPer; ++u) {
      const int i = t + u * kBlock;
      kk[u] = i < n ? gload(keys + c0 + i) : kEmpty;
      vv[u] = (vals && i < n) ? gloadd(vals + c0 + i) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kLoadPer; ++u) {
      const int i = t + u * kBlock;
      if (i < n) {
        xl.k[i] = kk[u];
        xl.v[i] = vv[u];
      }
    }
    if (t == 0) ws.first = n;
    __syncthreads();
    // the chunk ends at the first empty slot from kExtChunk on
    if (n > kExtChunk)
      for (int i = kExtChunk + t; i < n; i += kBlock)
        if (xl.k[i] == kEmpty) atomicMin(&ws.first, i);
    __syncthreads();
    const int end = ws.first;
    if (end == n && c0 + n < alloc) return false;   // uniform: a run longer than the pad
    for (int i = t; i < end; i += kBlock) {
      if (xl.k[i] == kEmpty || (i > 0 && xl.k[i - 1] != kEmpty)) continue;
      for (int q = i + 1; q < end && xl.k[q] != kEmpty; ++q) {
        const int32_t k = xl.k[q];
        const double v = xl.v[q];
        int at = q;
        while (at > i && xl.k[at - 1] > k) {
          xl.k[at] = xl.k[at - 1];
          xl.v[at] = xl.v[at - 1];
          --at;
        }
        xl.k[at] = k;
        xl.v[at] = v;
      }
    }
    __syncthreads();
    // compaction with one scan: thread t takes kExtPer consecutive slots
    constexpr int kExtPer = (kExtChunk + kExtPad + kBlock - 1) / kBlock;
    const int b0 = t * kExtPer, b1 = min(b0 + kExtPer, end);
    int64_t occ = 0;
    for (int i = b0; i < b1; ++i) occ += xl.k[i] != kEmpty ? 1 : 0;
    int64_t tot;
    int64_t o = run + block_exclusive_sum(occ, ws.wtot, &tot);
    for (int i = b0; i < b1; ++i) {
      const int32_t key = xl.k[i];
      if (key == kEmpty) continue;
      if (o < lim) {
        if (out_val) put_c(out_col, out_val, o, key, xl.v[i]);
        else out_col[o] = key;
      }
      ++o;
    }
    run += tot;
    c0 += end;
    __syncthreads();
  }
  return true;
}

// Sorted write-out of a device table by the whole workgroup.
__device__ void wg_global_extract(int32_t *keys, double *vals, int64_t alloc, int32_t dmax, WgScratch &ws,
                                  ExtLds &xl, int32_t *out_col, double *out_val, int64_t lim) {
  if (wg_extract_chunked(keys, vals, alloc, ws, xl, out_col, out_val, lim)) return;
  if (dmax > 0) wg_sort_runs(keys, vals, alloc);
  int64_t run = 0;
  for (int64_t c = 0; c < alloc; c += kBlock) {
    int64_t s = c + threadIdx.x;
    int32_t key = s < alloc ? gload(keys + s) : kEmpty;
    int64_t occ = key != kEmpty ? 1 : 0;
    int64_t tot;
    int64_t ex = block_exclusive_sum(occ, ws.wtot, &tot);
    if (occ) {
      int64_t rank = run + ex;
      if (rank < lim) {
        out_col[rank] = key;
        if (out_val) out_val[rank] = gloadd(vals + s);
      }
    }
    run += tot;
  }
  __syncthreads();
}

// ============================================================ wave tiles
// A wave tile is a run of at most 64 consecutive rows handled by one wave
// (one 64-lane workgroup).  Merge rows take one lane each; hashed rows take
// the whole wave one after another, accumulating in the wave's LDS table;
// workgroup-tier rows are left to k_big.  Numeric and one-pass tiles stage
// their sorted rows in LDS and copy them to C with contiguous, coalesced
// stores once the tile's offset in C is known.

// Home slot of column j.  Dense window: j - lo (the MinMax storing of
// Section IV-B, sorted by construction).  Otherwise a multiplicative
// (Fibonacci) hash into a power-of-two table with linear probing; the keys
// come out unsorted and the extraction sorts them (the Sort storing).
struct WaveTable {
  int32_t *keys;
  double *vals;
  int32_t T;       // slots (power of two unless dense)
  int32_t lo;
  uint32_t shift;  // 32 - log2(T)
  bool dense;
  // hashed tables whose columns minus lo, shifted left by log2(T), stay
  // below 2^31: a key and its slot sort together as one 32-bit word
  bool packs;
  __device__ __forceinline__ int32_t home(int32_t j) const {
    return dense ? j - lo : (int32_t)(((uint32_t)j * 0x9E3779B1u) >> shift);
  }
};

__device__ __forceinline__ WaveTable wave_table(int32_t *keys, double *vals, uint32_t inf, int32_t lo,
                                                int32_t b_cols) {
  WaveTable t;
  t.keys = keys;
  t.vals = vals;
  t.T = (int32_t)info_slots(inf);
  t.dense = info_dense(inf);
  t.lo = lo;
  t.shift = t.dense ? 0u : (uint32_t)(32 - __builtin_ctz((unsigned)t.T));
  t.packs = !t.dense && (((int64_t)b_cols - lo) << (32 - t.shift)) < ((int64_t)1 << 31);
  return t;
}


// Claim or find column j; returns its slot.  A table sized by the rules of
// k_size_rows never fills, so the probe always ends; a probe that would run
// past T (an inconsistent call) raises kErrInconsistent and drops the key.
template <bool VALUES>
__device__ __forceinline__ int32_t wave_probe(const WaveTable &tb, int32_t j, int32_t &cnt, int64_t *err) {
  int32_t h = tb.home(j);
  for (int32_t it = 0;; ++it) {
    const int32_t old = atomicCAS(&tb.keys[h], kEmpty, j);
    if (old == kEmpty) {
      ++cnt;
      if (VALUES) tb.vals[h] = 0.0;
      return h;
    }
    if (old == j) return h;
    if (tb.dense || it >= tb.T) {
      atomicOr((unsigned long long *)err, (unsigned long long)kErrInconsistent);
      return -1;
    }
    h = (h + 1) & (tb.T - 1);
  }
}

// Lanes per A entry: the next power of two >= the longest selected B row,
// at least kMinLanes (so at most 64 / kMinLanes ordered sub-steps) and at
// most 64 (longer B rows loop).
constexpr int kMinLanes = 16;
// Steps of A entries loaded ahead: four for the counting pass; two when
// values come along (fewer registers, more waves resident).
template <bool VALUES>
constexpr int wave_prefetch() {
  return VALUES ? 2 : 4;
}

// log2 of the lanes per A entry for a row whose longest selected B row has
// maxb entries.
__device__ __forceinline__ int lanes_log2(int32_t maxb) {
  int lw = __builtin_ctz((unsigned)kMinLanes);
  while ((1 << lw) < maxb && lw < 6) ++lw;
  return lw;
}

// One batch of a row: 64 / W entries of A per step, wave_prefetch() steps.
// First level: the lane's A entry (column, value) and its B row's bounds.
template <int PF>
struct Batch1 {
  int64_t bs[PF];
  int32_t bl[PF];
  double av[PF];
};
// Second level: the lane's B entry (column, value) of each step.
template <int PF>
struct Batch2 {
  int32_t jj[PF];
  double bb[PF];
};

template <bool VALUES, int PF = wave_prefetch<VALUES>()>
__device__ __forceinline__ void load_batch2(const Operands &op, int lw, const Batch1<PF> &b1, Batch2<PF> &b2) {
  const int bp = (int)threadIdx.x & ((1 << lw) - 1);
#pragma unroll
  for (int u = 0; u < PF; ++u) {
    const bool live = bp < b1.bl[u];
    b2.jj[u] = live ? op.b_col[b1.bs[u] + bp] : kEmpty;
    b2.bb[u] = (VALUES && live) ? op.b_val[b1.bs[u] + bp] : 0.0;
  }
}

// Inserts the products of one batch into the wave's table.  Values: a slot
// starts at +0.0 when claimed, and the entries of one step add their
// products in A's stored order (one sub-step per entry), so every slot is
// accumulated exactly in A's column order, as in the row-major kernel of
// Section IV-A.  cnt counts this lane's new columns.
template <bool VALUES, int PF = wave_prefetch<VALUES>()>
__device__ __forceinline__ void insert_batch(const Operands &op, int64_t e0, int64_t ae, int lw, const Batch1<PF> &b1,
                                             const Batch2<PF> &b2, const WaveTable &tb, int32_t &cnt, int64_t *err) {
  const int lane = threadIdx.x;
  const int per = kWave >> lw, sub = lane >> lw;
#pragma unroll
  for (int u = 0; u < PF; ++u) {
    if (e0 + (int64_t)u * per >= ae) continue;   // uniform: no entries left
    int32_t s = -1;
    if (b2.jj[u] != kEmpty) s = wave_probe<VALUES>(tb, b2.jj[u], cnt, err);
    if (VALUES) {
      for (int q = 0; q < per; ++q) {
        wave_sync();
        if (sub == q && s >= 0) tb.vals[s] = mul_add_rn(tb.vals[s], b1.av[u], b2.bb[u]);
      }
    }
    if (lw == 6 && b1.bl[u] > kWave) {
      // one A entry per step here: the rest of its B row, 64 columns at a time
      for (int32_t f = kWave + lane; f < b1.bl[u]; f += kWave) {
        const int32_t j = op.b_col[b1.bs[u] + f];
        const int32_t sl = wave_probe<VALUES>(tb, j, cnt, err);
        if (VALUES && sl >= 0) tb.vals[sl] = mul_add_rn(tb.vals[sl], b1.av[u], op.b_val[b1.bs[u] + f]);
      }
    }
    wave_sync();
  }
}

// The entries of a row's A part staged in the wave's LDS, 64 at a time: the
// start and length of the B row each selects, and its A value.
struct RowEntries {
  int64_t *bs;
  int32_t *bl;   // expand-sort rows: the length (<= 64) in the low 16 bits,
                 // the index of the entry's first product above
  double *av;
};

template <bool VALUES, int PF>
__device__ __forceinline__ void entries_batch1(const RowEntries &re, int e0, int gn, int lw, Batch1<PF> &b) {
  const int per = kWave >> lw, sub = (int)threadIdx.x >> lw;
#pragma unroll
  for (int u = 0; u < PF; ++u) {
    const int e = e0 + u * per + sub;
    b.bs[u] = 0;
    b.bl[u] = 0;
    b.av[u] = 0.0;
    if (e < gn) {
      b.bs[u] = re.bs[e];
      b.bl[u] = re.bl[e];
      if (VALUES) b.av[u] = re.av[e];
    }
  }
}

// Inserts every product of row [as, ae) (longest selected B row maxb) into
// the wave's table; returns the number of distinct columns (wave-uniform).
// The row's A entries and their B row bounds are loaded once (one per lane)
// into LDS; the B entries of the next batch are requested before the
// current batch is inserted.
template <bool VALUES>
__device__ int32_t wave_insert_row(const Operands &op, int64_t as, int64_t ae, int32_t maxb, const WaveTable &tb,
                                   const RowEntries &re, int64_t *err) {
  const int lane = threadIdx.x;
  const int lw = lanes_log2(maxb);
  constexpr int PF = wave_prefetch<VALUES>();
  const int step = (kWave >> lw) * PF;
  int32_t cnt = 0;
  for (int64_t g0 = as; g0 < ae; g0 += kWave) {
    const int gn = (int)min((int64_t)kWave, ae - g0);
    if (lane < gn) {
      int64_t bs;
      int32_t bl;
      b_row_of(op, g0 + lane, bs, bl);
      re.bs[lane] = bs;
      re.bl[lane] = bl;
      if (VALUES) re.av[lane] = op.a_val[g0 + lane];
    }
    wave_sync();
    Batch2<PF> c2, n2;
    {
      Batch1<PF> b1;
      entries_batch1<VALUES, PF>(re, 0, gn, lw, b1);
      load_batch2<VALUES, PF>(op, lw, b1, c2);
    }
    for (int e0 = 0; e0 < gn; e0 += step) {
      const bool more = e0 + step < gn;
      if (more) {
        Batch1<PF> b1;
        entries_batch1<VALUES, PF>(re, e0 + step, gn, lw, b1);
        load_batch2<VALUES, PF>(op, lw, b1, n2);
      }
      {
        // the A values and B row bounds again from LDS (not held in registers)
        Batch1<PF> b1;
        entries_batch1<VALUES, PF>(re, e0, gn, lw, b1);
        insert_batch<VALUES, PF>(op, e0, gn, lw, b1, c2, tb, cnt, err);
      }
      if (more) c2 = n2;
    }
    wave_sync();
  }
  return (int32_t)wave_sum(cnt);
}

__device__ __forceinline__ void wave_clear(const WaveTable &tb) {
  for (int32_t q = threadIdx.x; q < tb.T; q += kWave) tb.keys[q] = kEmpty;
  wave_sync();
}

// Ascending bitonic sort of 64 * E keys held lane-major (element i = lane *
// E + e), in the form whose every compare-exchange puts the smaller key at
// the lower index: level K (sorted blocks of K/2 become sorted blocks of K)
// first compares i with its mirror i ^ (K - 1) inside the block, then i with
// i ^ J for J = K/4 .. 1.  Partners within a lane are exchanged in
// registers, partners in other lanes through a lane exchange.  One
// instantiation per (level, distance) stage, so every register index is a
// constant.
// The value of the lane whose index is this lane's xor LM: DPP within a row
// of 16 lanes (quad permutations for 1, 2, 3, half-row and row mirrors for
// 7 and 15, a rotation by 8 for 8), a swizzle within 32 lanes for 4, 16 and
// 31, a permute across the halves for 32 and 63.
template <int LM>
__device__ __forceinline__ int32_t xor_lane(int32_t v) {
  if constexpr (LM == 1) return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, true);   // quad (1,0,3,2)
  else if constexpr (LM == 2) return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, true);  // quad (2,3,0,1)
  else if constexpr (LM == 3) return __builtin_amdgcn_update_dpp(0, v, 0x1B, 0xF, 0xF, true);  // quad (3,2,1,0)
  else if constexpr (LM == 7) return __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, true); // half-row mirror
  else if constexpr (LM == 8) return __builtin_amdgcn_update_dpp(0, v, 0x128, 0xF, 0xF, true); // row rotate 8
  else if constexpr (LM == 15) return __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, true); // row mirror
  else if constexpr (LM < 32) return __builtin_amdgcn_ds_swizzle(v, 0x1F | (LM << 10));        // lane ^ LM
  else return __shfl_xor(v, LM, kWave);
}

// The middle of three keys: with c the smallest int the smaller of x and y,
// with c the largest the larger; one instruction for the compare-exchange
// of a lane with its partner lane.
__device__ __forceinline__ int32_t med3_i32(int32_t x, int32_t y, int32_t c) {
  int32_t r;
  asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(y), "v"(c));
  return r;
}
// c for a stage whose lower lanes (bit B of the lane clear) keep the smaller
// key: the smallest int there, the largest elsewhere.  Made where it is used
// (not hoisted: one register instead of one per stage).
template <int B>
__device__ __forceinline__ int32_t lane_side(int lane) {
  int32_t c;
  asm volatile("v_bfe_i32 %0, %1, %2, 1\n\tv_xor_b32 %0, 0x80000000, %0" : "=&v"(c) : "v"(lane), "i"(B));
  return c;
}

// Stage (K, J) of the sort: J == K / 2 is the mirror stage of level K.
template <int E, int K, int J>
__device__ __forceinline__ void wave_bitonic_stage(int32_t (&x)[E]) {
  const int lane = threadIdx.x;
  if constexpr (J == K / 2 && K > E) {
    // mirror partner: lane ^ (K/E - 1), element E - 1 - e
    constexpr int lm = K / E - 1;
    const int32_t c = lane_side<__builtin_ctz(K / (2 * E))>(lane);
    // elements e and E - 1 - e trade partners: two values in flight
#pragma unroll
    for (int e = 0; e < (E + 1) / 2; ++e) {
      const int32_t ya = xor_lane<lm>(x[E - 1 - e]);
      const int32_t yb = xor_lane<lm>(x[e]);
      x[e] = med3_i32(x[e], ya, c);
      if (E - 1 - e != e) x[E - 1 - e] = med3_i32(x[E - 1 - e], yb, c);
    }
  } else if constexpr (J == K / 2) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if ((e & J) == 0) {
        const int32_t a = x[e], b = x[e ^ (K - 1)];
        x[e] = min(a, b);
        x[e ^ (K - 1)] = max(a, b);
      }
    }
  } else if constexpr (J >= E) {
    constexpr int lm = J / E;
    const int32_t c = lane_side<__builtin_ctz(lm)>(lane);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int32_t y = xor_lane<lm>(x[e]);
      x[e] = med3_i32(x[e], y, c);
    }
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if ((e & J) == 0) {
        const int32_t a = x[e], b = x[e ^ J];
        x[e] = min(a, b);
        x[e ^ J] = max(a, b);
      }
    }
  }
  if constexpr (J > 1) wave_bitonic_stage<E, K, J / 2>(x);
}

// Levels K .. 64 E; levels below `from` are skipped (their blocks of
// from / 2 keys are sorted already).
template <int E, int K>
__device__ __forceinline__ void wave_bitonic_levels(int32_t (&x)[E], int32_t from) {
  if (K >= from) wave_bitonic_stage<E, K, K / 2>(x);
  if constexpr (K < kWave * E) wave_bitonic_levels<E, 2 * K>(x, from);
}

template <int E>
__device__ __forceinline__ void wave_bitonic(int32_t (&x)[E], int32_t from = 2) {
  wave_bitonic_levels<E, 2>(x, from);
}

// Sorted write-out of a hashed row whose n keys were compacted (in slot
// order) to buf[0..n) in LDS: sort them there, then take every key's value
// from the slot its sorted word carries (or, where key and slot do not pack
// into one word, look the key up again) and write (column, value) at
// positions 0..n-1 of ocol/oval (at most lim), and empty the table.  ocol
// may be buf itself.
template <int E, bool NT>
__device__ void wave_sort_out(const WaveTable &tb, int32_t n, int32_t *buf, int32_t *ocol, double *oval,
                              int64_t lim) {
  const int lane = threadIdx.x;
  int32_t x[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int32_t pos = lane * E + e;
    x[e] = pos < n ? buf[pos] : kColMax;
  }
  wave_sync();
  wave_bitonic<E>(x);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int32_t pos = lane * E + e;
    if (pos < n) buf[pos] = x[e];
  }
  wave_sync();
  const int32_t m = (int32_t)min((int64_t)n, lim);
  if (tb.packs) {
    // the sorted words carry each key's slot: no second probe
    const int l2 = 32 - (int)tb.shift;
    for (int32_t pos = lane; pos < m; pos += kWave) {
      const int32_t w = buf[pos];
      put_c<NT>(ocol, oval, pos, (w >> l2) + tb.lo, tb.vals[w & (tb.T - 1)]);
    }
  } else {
    for (int32_t pos = lane; pos < m; pos += kWave) {
      const int32_t key = buf[pos];
      int32_t h = tb.home(key);
      for (int32_t it = 0; it < tb.T && tb.keys[h] != key; ++it) h = (h + 1) & (tb.T - 1);
      put_c<NT>(ocol, oval, pos, key, tb.vals[h]);
    }
  }
  wave_sync();
  wave_clear(tb);
}

// Sorts buf[0..nload) (nload <= 64 E) ascending in the wave's registers,
// where each aligned block of from / 2 keys is sorted already, and writes
// back the n smallest.
template <int E>
__device__ __forceinline__ void wave_sort_buf(int32_t *buf, int32_t nload, int32_t n, int32_t from) {
  const int lane = threadIdx.x;
  int32_t x[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int32_t pos = lane * E + e;
    x[e] = pos < nload ? buf[pos] : kColMax;
  }
  wave_sync();
  wave_bitonic<E>(x, from);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int32_t pos = lane * E + e;
    if (pos < n) buf[pos] = x[e];
  }
  wave_sync();
}

constexpr int kEscSteps = 2;

// Expand, sort, combine: the numeric row [as, ae) (every selected B row at
// most 64 long, at most kEscMax products) without a hash table.  Each
// product is stored at its index pi (A's stored order, then B's) as the
// rounded product a*b in pv[pi] and the word ((column - lo) << log2 T) | pi
// in buf[pi]; sorting the words orders the products by column and, within a
// column, by pi, i.e. in A's order.  Each run of one column sums its
// products from +0.0 in that order, exactly the row-major kernel's
// accumulation (Section IV-A).
// wave_esc_sort: expands and sorts; returns the number of products.
template <bool BIG>
__device__ int32_t wave_esc_sort(const Operands &op, int64_t as, int64_t ae, int32_t maxb, int32_t lo, int32_t T,
                                 const RowEntries &re, int32_t *buf, double *pv) {
  const int lane = threadIdx.x;
  const int bits = __builtin_ctz((unsigned)T);
  const int lw = lanes_log2(maxb);
  const int per = kWave >> lw, sub = lane >> lw, bp = lane & ((1 << lw) - 1);
  // every B row is sorted: where one block of P = pow2(maxb) indices per
  // entry of A fits the T slots, entry j's products take indices j P + bp
  // (the rest of its block a sentinel above every word), and the sort
  // starts from sorted blocks of P
  int32_t P = 1;
  while (P < maxb) P <<= 1;
  const bool blocks = (ae - as) * P <= T;
  int32_t pbase = 0;
  for (int64_t g0 = as; g0 < ae; g0 += kWave) {
    const int gn = (int)min((int64_t)kWave, ae - g0);
    int32_t bl = 0;
    int64_t bs = 0;
    if (lane < gn) b_row_of(op, g0 + lane, bs, bl);
    const int32_t inc = wave_inclusive_sum32(bl);
    if (lane < gn) {
      re.bs[lane] = bs;
      re.bl[lane] = bl | ((pbase + inc - bl) << 16);
      re.av[lane] = op.a_val[g0 + lane];
    }
    pbase += __shfl(inc, kWave - 1, kWave);
    wave_sync();
    // kEscSteps steps of `per` entries at a time, their loads in flight
    // together
    for (int e0 = 0; e0 < gn; e0 += kEscSteps * per) {
      int32_t jj[kEscSteps], pi[kEscSteps];
      double ab[kEscSteps], bb[kEscSteps];
#pragma unroll
      for (int u = 0; u < kEscSteps; ++u) {
        const int e = e0 + u * per + sub;
        pi[u] = -1;
        const int32_t w = e < gn ? re.bl[e] : 0;
        const int32_t at_pi = blocks ? (int32_t)(g0 - as + e) * P + bp : (w >> 16) + bp;
        if (bp < (w & 0xffff)) {
          const int64_t at = re.bs[e] + bp;
          jj[u] = op.b_col[at];
          bb[u] = op.b_val[at];
          ab[u] = re.av[e];
          pi[u] = at_pi;
        } else if (blocks && e < gn && bp < P) {
          buf[at_pi] = kColMax;
        }
      }
#pragma unroll
      for (int u = 0; u < kEscSteps; ++u) {
        if (pi[u] < 0) continue;
        buf[pi[u]] = ((jj[u] - lo) << bits) | pi[u];
        double p;
        {
#pragma clang fp contract(off)
          p = ab[u] * bb[u];
        }
        pv[pi[u]] = p;
      }
    }
    wave_sync();
  }
  const int32_t n = pbase;
  const int32_t nl = blocks ? (int32_t)(ae - as) * P : n, from = blocks ? 2 * P : 2;
  if (nl <= 64) wave_sort_buf<1>(buf, nl, n, from);
  else if (nl <= 128) wave_sort_buf<2>(buf, nl, n, from);
  else if (nl <= 256) wave_sort_buf<4>(buf, nl, n, from);
  else if (!BIG || nl <= 512) wave_sort_buf<8>(buf, nl, n, from);   // !BIG: nl <= kEscMaxSmall
  else wave_sort_buf<16>(buf, nl, n, from);   // nl <= T <= kEscMax
  return n;
}

// Counting pass by sorting: the columns of row [as, ae) go to buf in one
// block of P = pow2(maxb) slots per entry of A (each block sorted, as B's
// rows are, the rest of it a sentinel above every column; at most
// kSortCountMax slots), are sorted from those blocks, and the row's size is
// the number of runs.  buf (the wave's table) is left empty.
__device__ int32_t wave_sort_count(const Operands &op, int64_t as, int64_t ae, int32_t maxb, const RowEntries &re,
                                   int32_t *buf) {
  const int lane = threadIdx.x;
  const int lw = lanes_log2(maxb);
  const int per = kWave >> lw, sub = lane >> lw, bp = lane & ((1 << lw) - 1);
  int32_t P = 1;
  while (P < maxb) P <<= 1;
  int32_t tot = 0;
  for (int64_t g0 = as; g0 < ae; g0 += kWave) {
    const int gn = (int)min((int64_t)kWave, ae - g0);
    if (lane < gn) {
      int64_t bs;
      int32_t bl;
      b_row_of(op, g0 + lane, bs, bl);
      re.bs[lane] = bs;
      re.bl[lane] = bl;
      tot += bl;
    }
    wave_sync();
    for (int e0 = 0; e0 < gn; e0 += 4 * per) {
      int32_t jj[4], at[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + u * per + sub;
        at[u] = -1;
        jj[u] = kColMax;
        if (e < gn && bp < P) {
          at[u] = (int32_t)(g0 - as + e) * P + bp;
          if (bp < re.bl[e]) jj[u] = op.b_col[re.bs[e] + bp];
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (at[u] >= 0) buf[at[u]] = jj[u];
    }
    wave_sync();
  }
  const int32_t n = (int32_t)wave_sum((int64_t)tot);
  const int32_t nl = (int32_t)(ae - as) * P;
  if (nl <= 64) wave_sort_buf<1>(buf, nl, n, 2 * P);
  else if (nl <= 128) wave_sort_buf<2>(buf, nl, n, 2 * P);
  else wave_sort_buf<4>(buf, nl, n, 2 * P);   // nl <= kSortCountMax
  int32_t runs = 0;
  for (int32_t q0 = 0; q0 < n; q0 += kWave) {
    const int32_t q = q0 + lane;
    const bool head = q < n && (q == 0 || buf[q - 1] != buf[q]);
    runs += __popcll(ballot(head));
  }
  wave_sync();
  for (int32_t q = lane; q < nl; q += kWave) buf[q] = kEmpty;
  wave_sync();
  return runs;
}

// wave_esc_emit: combines the runs of one column of the n sorted products;
// the rank of a run's head is its place.  WRITE: writes the row (at most lim
// entries) to ocol/oval in column order.  Returns the row's size.
template <bool WRITE, bool NT>
__device__ int32_t wave_esc_emit(const int32_t *buf, const double *pv, int32_t n, int32_t lo, int32_t T,
                                 int32_t *ocol, double *oval, int64_t lim) {
  const int lane = threadIdx.x;
  const int bits = __builtin_ctz((unsigned)T);
  const uint64_t lt = lanemask_lt();
  int32_t run = 0;
  for (int32_t q0 = 0; q0 < n; q0 += kWave) {
    const int32_t q = q0 + lane;
    int32_t w = 0;
    bool head = false;
    if (q < n) {
      w = buf[q];
      head = q == 0 || (buf[q - 1] >> bits) != (w >> bits);
    }
    const uint64_t hb = ballot(head);
    if (WRITE && head) {
      const int32_t key = w >> bits;
      double v;
      {
#pragma clang fp contract(off)
        v = 0.0 + pv[w & (T - 1)];
        for (int32_t t = q + 1; t < n; ++t) {
          const int32_t w2 = buf[t];
          if ((w2 >> bits) != key) break;
          v = v + pv[w2 & (T - 1)];
        }
      }
      const int32_t rank = run + __popcll(hb & lt);
      if (rank < lim) put_c<NT>(ocol, oval, rank, key + lo, v);
    }
    run += __popcll(hb);
  }
  wave_sync();
  return run;
}

// Expand, sort, combine and write (the numeric pass); returns the row's size.
template <bool NT, bool BIG>
__device__ __forceinline__ int32_t wave_esc_row(const Operands &op, int64_t as, int64_t ae, int32_t maxb, int32_t lo,
                                                int32_t T, const RowEntries &re, int32_t *buf, double *pv,
                                                int32_t *ocol, double *oval, int64_t lim) {
  const int32_t n = wave_esc_sort<BIG>(op, as, ae, maxb, lo, T, re, buf, pv);
  return wave_esc_emit<true, NT>(buf, pv, n, lo, T, ocol, oval, lim);
}

// Writes the row held by the table in column order to ocol/oval (at most
// lim entries) and leaves the table empty.  buf: LDS room for n keys (may be
// ocol itself when that is in LDS).
template <bool NT>
__device__ void wave_extract(const WaveTable &tb, int32_t n, int32_t *buf, int32_t *ocol, double *oval,
                             int64_t lim) {
  const int lane = threadIdx.x;
  const uint64_t lt = lanemask_lt();
  int32_t run = 0;
  if (tb.dense) {
    // slot order is column order
    for (int32_t c0 = 0; c0 < tb.T; c0 += kWave) {
      const int32_t q = c0 + lane;
      const int32_t key = q < tb.T ? tb.keys[q] : kEmpty;
      const bool occ = key != kEmpty;
      const uint64_t bal = ballot(occ);
      if (occ) {
        const int32_t rank = run + __popcll(bal & lt);
        if (rank < lim) put_c<NT>(ocol, oval, rank, key, tb.vals[q]);
        tb.keys[q] = kEmpty;
      }
      run += __popcll(bal);
    }
    wave_sync();
    return;
  }
  for (int32_t c0 = 0; c0 < tb.T; c0 += kWave) {
    const int32_t q = c0 + lane;
    const int32_t key = q < tb.T ? tb.keys[q] : kEmpty;
    const bool occ = key != kEmpty;
    const uint64_t bal = ballot(occ);
    if (occ) buf[run + __popcll(bal & lt)] = tb.packs ? ((key - tb.lo) << (32 - tb.shift)) | q : key;
    run += __popcll(bal);
  }
  wave_sync();
  // n <= kSortMax (k_size_rows sends larger hashed rows to the workgroup tier)
  if (n <= 64) wave_sort_out<1, NT>(tb, n, buf, ocol, oval, lim);
  else if (n <= 128) wave_sort_out<2, NT>(tb, n, buf, ocol, oval, lim);
  else if (n <= 256) wave_sort_out<4, NT>(tb, n, buf, ocol, oval, lim);
  else if (n <= 512) wave_sort_out<8, NT>(tb, n, buf, ocol, oval, lim);
  else wave_sort_out<16, NT>(tb, n, buf, ocol, oval, lim);
}

// Tile kernel.  A tile is a run of at most 64 consecutive rows; its merge
// rows take one lane each, its hashed rows the whole wave one after another,
// and its workgroup-tier rows are left to k_big.
//   kSymbolic: per-row counts (cnt_out).
//   kNumeric:  c_rp holds the exact row offsets; every row is written there.
//   kOnePass:  c_rp holds padded offsets (the scan of the rows' capacities,
//              learned or bound).  A tile's rows share its padded range and
//              are laid out in it by their exact counts; every row's count
//              goes to cnt_out and its place to pad_src, and a row the range
//              has no room for takes a place in the spill arena (after the
//              padded range) or, with the arena full, is listed in ovf_list
//              (counted in counters[kCtrOverflow]) for the exact path.
// Merge rows and small hashed rows (capacity <= stage_row_max) are staged in
// LDS at offsets that follow their capacities and copied out with
// contiguous stores; larger hashed rows are written by their wave directly.
// LDS of a wave tile: table keys, table values, the compaction buffer of a
// hashed row (kSortMax keys at most), stage columns, stage values.
struct WaveLds {
  size_t ent, vals, buf, scol, sval, total;
};
__host__ __device__ inline WaveLds wave_lds_layout(bool values, int table_slots, int stage_slots) {
  auto a16 = [](size_t x) { return (x + 15) & ~(size_t)15; };
  WaveLds L;
  // row entries (64 x (int64 + int32 + double)) first, a flag word (16
  // bytes), then the table
  L.ent = (size_t)kWave * 20 + 16;
  L.vals = L.ent + a16((size_t)table_slots * 4);
  if (!values) {
    L.buf = L.scol = L.sval = L.total = L.vals;
    return L;
  }
  const size_t nbuf = (size_t)(table_slots < kSortMax ? table_slots : kSortMax);
  L.buf = L.vals + (size_t)table_slots * 8;
  L.scol = a16(L.buf + nbuf * 4);
  L.sval = a16(L.scol + (size_t)stage_slots * 4);
  L.total = L.sval + (size_t)stage_slots * 8;
  return L;
}

// ESCO: every hashed row of the launch is an expand-sort row (numeric or
// one pass) or, counting, a sort-count row (no merge rows): the table path
// is not compiled, which frees registers.
// Resident waves per SIMD: seven for the counting pass (no values: it fits
// 72 registers with few spills), eight when it only sorts; for expand-sort
// launches seven in the
// numeric pass and six in the one pass (their spills, outside the sort,
// cost less than the extra waves gain in hiding the gathers' latency), five
// with the 16-per-lane sort (no spills); four for the table launches (the
// one pass spills a few registers there, which costs less than the fourth
// wave gains: 24.0 -> 19.7 ms on the 27-point product), fewer where the
// merge lists take registers.
// BIG: expand-sort rows of up to kEscMax products (sorted 16 per lane);
// launches without it take rows of at most kEscMaxSmall (fewer registers).
template <int MODE, int M, bool MERGE, bool ESCO = false, bool BIG = false>
__global__ void __launch_bounds__(kWave, ESCO ? (BIG ? 5 : (MODE == kOnePass ? 6 : (MODE == kNumeric ? 7 : 8)))
                                         : MODE == kSymbolic ? 7
                                         : (MODE == kOnePass ? (MERGE ? 2 : 4) : (MERGE && M == 8 ? 3 : 4)))
k_wt(WaveTileParams p) {
  constexpr bool VALUES = (MODE != kSymbolic);
  extern __shared__ __align__(16) unsigned char lds[];
  const int lane = threadIdx.x;
  const Operands &op = p.op;
  int64_t *err = p.counters + kCtrError;
  const WaveLds L = wave_lds_layout(VALUES, p.table_slots, p.stage_slots);
  const RowEntries re{reinterpret_cast<int64_t *>(lds), reinterpret_cast<int32_t *>(lds + kWave * 8),
                      reinterpret_cast<double *>(lds + kWave * 12)};
  int32_t *tkeys = reinterpret_cast<int32_t *>(lds + L.ent);
  double *tvals = reinterpret_cast<double *>(lds + L.vals);
  int32_t *buf = reinterpret_cast<int32_t *>(lds + L.buf);
  int32_t *scol = reinterpret_cast<int32_t *>(lds + L.scol);
  double *sval = reinterpret_cast<double *>(lds + L.sval);
  // one pass: set by a probe that found its row's table full
  int64_t *full_flag = reinterpret_cast<int64_t *>(lds + kWave * 20);
  for (int32_t q = lane; q < p.table_slots; q += kWave) tkeys[q] = kEmpty;
  if (lane == 0) *full_flag = 0;
  wave_sync();

  for (int64_t t = blockIdx.x; t < p.ntiles; t += gridDim.x) {
    const int64_t r0 = p.tile_row ? (int64_t)p.tile_row[t] : t * kWave;
    const int64_t r1 = p.tile_row ? (int64_t)p.tile_row[t + 1] : min(r0 + kWave, op.rows);
    const int nr = (int)(r1 - r0);
    const bool valid = lane < nr;
    const int64_t row = r0 + lane;
    const uint32_t inf = valid ? p.info[row] : 0u;
    const uint32_t tier = valid ? info_tier(inf) : (uint32_t)kTierEmpty;
    const int32_t capr = valid ? p.cap[row] : 0;
    int64_t n = 0;

    // staged rows and their stage offsets (by capacity, in row order)
    const bool staged = VALUES && ((MERGE && tier == kTierMerge) ||
                                   (tier == kTierHash && capr <= p.stage_row_max && !info_esc(inf)));
    const int32_t res = staged ? capr : 0;
    const int32_t sinc = wave_inclusive_sum32(res);
    const int32_t soff = sinc - res;
    int64_t base = 0, pos = 0, tile_len = 0;
    if (VALUES) {
      base = p.c_rp[r0];
      pos = valid ? p.c_rp[row] - base : 0;
      tile_len = p.c_rp[r1] - base;
    }
    bool fits = true;   // kOnePass: the row keeps its place in the tile's range

    // merge rows, one lane each
    if (VALUES && MERGE) {
      if (tier == kTierMerge) {
        n = merge_row<M, true, false>(op, row, scol + soff, sval + soff, capr);
        fits = n <= capr;
      }
    } else if (MERGE && tier == kTierMerge) {
      n = merge_row<M, false, false>(op, row, nullptr, nullptr, 0);
    }
    wave_sync();

    // one pass: the tile's rows share its padded range (the sum of their
    // capacities) and are laid out there by their exact counts, in row
    // order.  The merge rows that fit their staging keep their places; then
    // every hashed row, in row order, takes the next place if the range
    // still holds it.  hb: entries of the kept hashed rows before a row.  A
    // row with no room claims a place in the spill arena; only when that is
    // full is the row left to the exact path.
    int32_t mexcl = 0, mtot = 0, hb = 0;
    int64_t hsum = 0, spos = -1;
    if (MODE == kOnePass) {
      const int32_t mk = (tier == kTierMerge && fits) ? (int32_t)n : 0;
      const int32_t minc = wave_inclusive_sum32(mk);
      mexcl = minc - mk;
      mtot = __shfl(minc, kWave - 1, kWave);
    }

    // hashed rows, the whole wave on one row at a time
    uint64_t hm = ballot(tier == kTierHash);
    while (hm) {
      const int r = __ffsll((unsigned long long)hm) - 1;
      hm &= hm - 1;
      const int64_t hrow = r0 + r;
      if (MODE != kSymbolic && (ESCO || info_esc(__shfl(inf, r, kWave)))) {
        // expand, sort, combine: no table; the row (never staged) goes
        // straight to its place
        const int32_t cap_r = __shfl(capr, r, kWave);
        const int32_t T = (int32_t)info_slots(__shfl(inf, r, kWave));
        if (MODE == kNumeric) {
          const int64_t o = base + __shfl(pos, r, kWave);
          const int64_t lim = max((int64_t)0, min((int64_t)cap_r, p.c_capacity - o));
          const int32_t c = wave_esc_row<true, BIG>(op, op.a_rp[hrow], op.a_rp[hrow + 1], p.maxb[hrow], p.lo[hrow], T,
                                               re, buf, tvals, p.c_col + o, p.c_val + o, lim);
          if (lane == r) {
            n = c;
            fits = c <= cap_r;
          }
          continue;
        }
        // one pass: count first, then the place (the tile's range or the
        // spill arena, as for a hashed row), then write
        const int32_t np = wave_esc_sort<false>(op, op.a_rp[hrow], op.a_rp[hrow + 1], p.maxb[hrow], p.lo[hrow], T, re, buf,
                                         tvals);
        const int32_t c = wave_esc_emit<false, false>(buf, tvals, np, p.lo[hrow], T, nullptr, nullptr, 0);
        bool keep = (int64_t)mtot + hsum + c <= tile_len, spill = false;
        int64_t o = base + __shfl(mexcl, r, kWave) + hsum;
        if (!keep) {
          int64_t at = 0;
          if (lane == 0) at = (int64_t)atomicAdd((unsigned long long *)&p.counters[kCtrSpill], (unsigned long long)c);
          at = __shfl(at, 0, kWave);
          spill = at + c <= p.spill_cap;
          o = p.spill_base + at;
        }
        if (keep || spill) {
          const int64_t rl = max((int64_t)0, min((int64_t)c, p.c_capacity - o));
          wave_esc_emit<true, false>(buf, tvals, np, p.lo[hrow], T, p.c_col + o, p.c_val + o, rl);
        }
        if (keep) {
          if (lane > r) hb += c;
          hsum += c;
        }
        if (lane == r) {
          n = c;
          fits = keep;
          if (spill) spos = o;
        }
        continue;
      }
      if (MODE == kSymbolic && (ESCO || info_esc(__shfl(inf, r, kWave)))) {
        const int32_t c = wave_sort_count(op, op.a_rp[hrow], op.a_rp[hrow + 1], p.maxb[hrow], re, tkeys);
        if (lane == r) n = c;
        continue;
      }
      const WaveTable tb = wave_table(tkeys, tvals, __shfl(inf, r, kWave), p.lo[hrow], op.b_cols);
      const int32_t c = wave_insert_row<VALUES>(op, op.a_rp[hrow], op.a_rp[hrow + 1], p.maxb[hrow], tb, re,
                                                MODE == kOnePass ? full_flag : err);
      const int32_t cap_r = __shfl(capr, r, kWave);
      bool keep, spill = false, full = false;
      int64_t o;   // the row's place when written straight out
      if (MODE == kOnePass) {
        // a table sized by a learned capacity may have filled: keys were
        // dropped, and the row goes to the exact path
        wave_sync();
        full = *full_flag != 0;
        wave_sync();
        if (full && lane == 0) *full_flag = 0;
        keep = !full && (int64_t)mtot + hsum + c <= tile_len;
        o = base + __shfl(mexcl, r, kWave) + hsum;
        if (!keep && !full) {
          int64_t at = 0;
          if (lane == 0) at = (int64_t)atomicAdd((unsigned long long *)&p.counters[kCtrSpill], (unsigned long long)c);
          at = __shfl(at, 0, kWave);
          spill = at + c <= p.spill_cap;
          o = p.spill_base + at;
        }
      } else {
        keep = VALUES && c <= cap_r;
        o = base + __shfl(pos, r, kWave);
      }
      if (!keep && !spill) {
        // counted only, or no room (one pass: computed again by the exact path)
        wave_clear(tb);
      } else if (keep && __shfl(staged ? 1 : 0, r, kWave) && c <= cap_r) {
        const int32_t so = __shfl(soff, r, kWave);
        wave_extract<false>(tb, c, buf, scol + so, sval + so, c);
      } else {
        // straight to the row's place in C (or in the padded buffer)
        const int64_t rl = max((int64_t)0, min((int64_t)c, p.c_capacity - o));
        wave_extract<MODE == kNumeric>(tb, c, buf, p.c_col + o, p.c_val + o, rl);
      }
      if (MODE == kOnePass && keep) {
        if (lane > r) hb += c;
        hsum += c;
      }
      if (lane == r) {
        n = c;
        fits = keep;
        if (spill) spos = o;
      }
    }

    // without MERGE, merge-tier rows are the row-per-thread kernel's
    const bool own = valid && tier != kTierGlobal && (MERGE || tier != kTierMerge);
    if (MODE == kSymbolic) {
      if (own) p.cnt_out[row] = (int32_t)n;
      continue;
    }
    if (MODE == kNumeric && own && n != capr)
      atomicOr((unsigned long long *)err, (unsigned long long)kErrInconsistent);
    if (lane == 0 && base + tile_len > p.c_capacity)
      atomicOr((unsigned long long *)err, (unsigned long long)kErrCapacity);

    if (MODE == kOnePass) {
      // merge rows longer than their staging: merged again into the arena
      const bool mspill = MERGE && valid && tier == kTierMerge && !fits;
      if (ballot(mspill)) {
        const int64_t want = mspill ? n : 0;
        const int32_t winc = wave_inclusive_sum32((int32_t)want);
        int64_t at = 0;
        if (lane == kWave - 1 && winc > 0)
          at = (int64_t)atomicAdd((unsigned long long *)&p.counters[kCtrSpill], (unsigned long long)winc);
        at = __shfl(at, kWave - 1, kWave) + (winc - want);
        if (mspill && at + want <= p.spill_cap) {
          spos = p.spill_base + at;
          merge_row<M, true, false>(op, row, p.c_col + spos, p.c_val + spos, want);
        }
      }
      const bool row_out = valid && tier != kTierGlobal;
      const bool kept = row_out && fits;
      const int32_t ppos = mexcl + hb;   // place in the tile's range (kept rows)
      // every row of the tile gets its place (-1: written straight into C,
      // as the workgroup-tier rows and the rows with no room are)
      if (row_out) p.cnt_out[row] = (int32_t)n;
      if (valid) p.pad_src[row] = kept ? base + ppos : (row_out ? spos : (int64_t)-1);
      const uint64_t sb = ballot(row_out && !fits && spos >= 0);
      if (sb && lane == 0) atomicAdd((unsigned long long *)&p.counters[kCtrSpillRows], (unsigned long long)__popcll(sb));
      // rows with no room anywhere go to the exact path
      const bool ov = row_out && !fits && spos < 0;
      const uint64_t ob = ballot(ov);
      if (ob) {
        int64_t at = 0;
        if (lane == 0)
          at = (int64_t)atomicAdd((unsigned long long *)&p.counters[kCtrOverflow], (unsigned long long)__popcll(ob));
        at = __shfl(at, 0, kWave);
        if (ov) p.ovf_list[at + __popcll(ob & lanemask_lt())] = (int32_t)row;
      }
      // staged kept rows move from their staging (laid out by capacity) to
      // their places (laid out by count): every entry of the kept range
      // finds its row by a search over the places in LDS (the row-entry
      // area, free here)
      int32_t *s_pos = reinterpret_cast<int32_t *>(lds);
      int32_t *s_so = s_pos + kWave;
      s_pos[lane] = ppos;
      s_so[lane] = (kept && staged && n <= capr) ? soff : -1;
      wave_sync();
      const int64_t ktot = (int64_t)mtot + hsum;
      const int64_t lim = max((int64_t)0, min(ktot, p.c_capacity - base));
      for (int64_t q = lane; q < lim; q += kWave) {
        int lo = 0, hi = kWave - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_pos[mid] <= q) lo = mid;
          else hi = mid - 1;
        }
        const int32_t so = s_so[lo];
        if (so >= 0) {
          const int32_t from = so + (int32_t)(q - s_pos[lo]);
          p.c_col[base + q] = scol[from];
          p.c_val[base + q] = sval[from];
        }
      }
      wave_sync();
      continue;
    }

    // copy-out of the staged rows: one contiguous copy of the tile's range
    // when every row with room is staged at its place, else row by row
    const bool in_order = ballot(valid && capr > 0 && !(staged && fits && soff == pos)) == 0ull;
    if (in_order) {
      const int64_t lim = max((int64_t)0, min(tile_len, p.c_capacity - base));
      for (int64_t q = lane; q < lim; q += kWave) put_c(p.c_col, p.c_val, base + q, scol[q], sval[q]);
    } else {
      uint64_t sm = ballot(valid && staged && fits && n > 0);
      while (sm) {
        const int r = __ffsll((unsigned long long)sm) - 1;
        sm &= sm - 1;
        const int32_t so = __shfl(soff, r, kWave);
        const int64_t o = base + __shfl(pos, r, kWave);
        const int64_t lim = max((int64_t)0, min(__shfl(n, r, kWave), p.c_capacity - o));
        for (int64_t q = lane; q < lim; q += kWave) put_c(p.c_col, p.c_val, o + q, scol[so + q], sval[so + q]);
      }
    }
    wave_sync();
  }
}

// Moves the one-pass rows from the padded buffer to their exact places:
// 64 rows per wave, their entries copied as one contiguous range of C (rows
// written elsewhere, workgroup-tier and overflow rows, are skipped).
__global__ void __launch_bounds__(kBlock) k_compact(CompactParams p) {
  // the wave's row offsets live in LDS: the search below runs in divergent
  // lanes, where a cross-lane read from an inactive lane would return 0
  __shared__ int64_t s_dst[kWavesPerBlock][kWave + 1];
  __shared__ int64_t s_src[kWavesPerBlock][kWave];
  const int l = lane_id();
  const int w = threadIdx.x / kWave;
  const int64_t r0 = ((int64_t)blockIdx.x * kWavesPerBlock + w) * kWave;
  if (r0 >= p.rows) return;
  const int64_t row = r0 + l;
  const int nr = (int)min((int64_t)kWave, p.rows - r0);
  const int64_t base = p.c_rp[r0];
  if (l < nr) {
    s_dst[w][l] = p.c_rp[row] - base;
    // rows written straight into C (workgroup tier, no room) are marked -1
    s_src[w][l] = info_tier(p.info[row]) == kTierGlobal ? (int64_t)-1 : p.pad_src[row];
  }
  if (l == 0) s_dst[w][nr] = p.c_rp[r0 + nr] - base;
  wave_sync();
  const int64_t lim = min(base + s_dst[w][nr], p.c_capacity) - base;
  if (s_dst[w][nr] >= 32 * (int64_t)nr) {
    // rows of 32 or more entries on average: row by row, the whole wave on
    // each row's contiguous range (no search per entry)
    for (int r = 0; r < nr; ++r) {
      const int64_t from = s_src[w][r];
      const int64_t d0 = s_dst[w][r], d1 = min(s_dst[w][r + 1], lim);
      if (from < 0) continue;
      for (int64_t q = d0 + l; q < d1; q += kWave)
        put_c<false>(p.c_col, p.c_val, base + q, p.pad_col[from + (q - d0)], p.pad_val[from + (q - d0)]);
    }
    return;
  }
  for (int64_t q = l; q < lim; q += kWave) {
    // the row holding entry base + q: the last row whose start is <= q
    int lo = 0, hi = nr - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_dst[w][mid] <= q) lo = mid;
      else hi = mid - 1;
    }
    const int64_t from = s_src[w][lo];
    if (from >= 0) {
      // plain stores here: streaming ones measured slower for this copy
      put_c<false>(p.c_col, p.c_val, base + q, p.pad_col[from + (q - s_dst[w][lo])],
                   p.pad_val[from + (q - s_dst[w][lo])]);
    }
  }
}

hipError_t launch_compact(const CompactParams &cp, hipStream_t s) {
  if (cp.rows <= 0) return hipSuccess;
  const int64_t waves = (cp.rows + kWave - 1) / kWave;
  const int64_t blocks = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
  hipLaunchKernelGGL(k_compact, dim3((unsigned)blocks), dim3(kBlock), 0, s, cp);
  return hipGetLastError();
}

// Workgroup-tier rows: one workgroup per listed row, the table in the
// workgroup's slice of device scratch (sized by the plan).
// Part words of a split row: done flag above the part's size.
constexpr int64_t kPartDone = 1ll << 40;
constexpr int64_t kPartSize = kPartDone - 1;

// Workgroup-tier rows from an atomic ticket.  The first kMaxSplitRows rows of
// the list's huge front are taken as kSplitParts items each: a row of at
// least kSplitWork products as one item per column range (B row slices
// found by binary search; every column is still accumulated by one
// workgroup in A's order), a smaller one whole by its first item (the
// others end at once).  Counting pass: each part
// publishes its size and the last part of the row to finish writes the row's
// count.  Numeric pass: a part publishes its size after its key pass and
// writes its columns after those of the earlier parts, whose sizes it waits
// for; those parts hold earlier tickets, so their workgroups are running and
// wait on nothing later (a wait that exceeds kSpinLimit polls raises
// kErrLookback instead of hanging).
template <int MODE>
__global__ void __launch_bounds__(kBlock) k_big(BigParams p) {
  __shared__ WgScratch ws;
  __shared__ ExtLds xl;
  const Operands &op = p.op;
  const int64_t nbig = p.counters[p.count_ctr];
  int32_t *gkeys = reinterpret_cast<int32_t *>(p.scratch + (size_t)blockIdx.x * (size_t)p.scratch_slots * 12);
  double *gvals = reinterpret_cast<double *>(p.scratch + (size_t)blockIdx.x * (size_t)p.scratch_slots * 12 +
                                             (size_t)p.scratch_slots * 4);
  int64_t *err = p.counters + kCtrError;
  const int64_t nh = p.huge_ctr >= 0 ? p.counters[p.huge_ctr] : nbig;
  const int64_t ns = p.split ? min(nh, kMaxSplitRows) : 0;
  const int64_t nitems = nbig + ns * (kSplitParts - 1);
  __shared__ int64_t s_i, s_off;
  while (true) {
    // the next item from the ticket: workgroups that finish early take more
    if (threadIdx.x == 0)
      s_i = (int64_t)atomicAdd((unsigned long long *)&p.counters[kCtrBigTicket], 1ull);
    __syncthreads();
    const int64_t i = s_i;
    __syncthreads();
    if (i >= nitems) break;
    int64_t row, slot = -1;
    int g = 0;
    if (i < ns * kSplitParts) {
      slot = i / kSplitParts;
      g = (int)(i % kSplitParts);
      row = p.list[slot];
      if ((int64_t)p.ub[row] < kSplitWork) {
        if (g > 0) continue;   // uniform: the row is its first item's
        slot = -1;
      }
    } else {
      const int64_t j = i - ns * (kSplitParts - 1);
      row = j < nh ? p.list[j] : p.list[p.list_len - 1 - (j - nh)];
    }
    // the row's (or the part's) column range and its table
    const int64_t c = (MODE == kNumeric) ? (int64_t)p.cnt[row] : (int64_t)p.ub[row];
    int32_t lo = p.lo[row], hi = p.hi[row], c0 = 0, c1 = -1;
    if (slot >= 0) {
      const int64_t span = (int64_t)hi - lo + 1;
      c0 = (int32_t)(lo + span * g / kSplitParts);
      c1 = (int32_t)(lo + span * (g + 1) / kSplitParts);
      lo = c0;
      hi = c1 - 1;
    }
    bool work = slot < 0 || c1 > c0;
    bool dense = false;
    int64_t slots = 0, alloc = 0;
    if (work) {
      alloc = global_table_alloc((int64_t)hi - lo + 1, c, p.dense_ratio, &dense, &slots);
      if (alloc > p.scratch_slots) {
        if (threadIdx.x == 0) atomicOr((unsigned long long *)err, (unsigned long long)kErrScratch);
        work = false;
      }
    }
    RowHash hs{};
    if (work) hs = make_hash(lo, hi, slots, dense);
    int32_t n = 0;
    if (work)
      n = MODE == kNumeric ? wg_global_accumulate(op, row, c0, c1, gkeys, gvals, alloc, hs, ws, xl, p.fast != 0, err)
                           : wg_global_keys(op, row, c0, c1, gkeys, alloc, hs, ws, err);
    int64_t *pp = slot >= 0 ? p.parts + slot * (kSplitParts + 1) : nullptr;
    if (MODE == kSymbolic) {
      if (threadIdx.x == 0) {
        if (!pp) {
          p.cnt[row] = n;
        } else {
          // one word counts the finished parts (above kPartSize) and sums
          // their sizes: the part that finishes last holds the row's size in
          // what its own add returns.  Relaxed atomics: the payload is the
          // word itself (an agent-scope release would write back the XCD's
          // whole L2, which holds the tables of every other workgroup).
          const int64_t before =
              __hip_atomic_fetch_add(pp + kSplitParts, kPartDone + (int64_t)n, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
          if ((before >> 40) == kSplitParts - 1) p.cnt[row] = (int32_t)((before & kPartSize) + n);
        }
      }
    } else {
      // the size travels in the flag word itself: relaxed atomics suffice
      if (threadIdx.x == 0 && pp)
        __hip_atomic_store(pp + g, kPartDone | (int64_t)n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (threadIdx.x == 0) {
        int64_t pre = 0;
        if (pp) {
          for (int k = 0; k < g; ++k) {
            int64_t v = 0;
            for (int64_t polls = 0;; ++polls) {
              v = __hip_atomic_load(pp + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              if (v & kPartDone) break;
              if (polls > kSpinLimit) {
                atomicOr((unsigned long long *)err, (unsigned long long)kErrLookback);
                break;
              }
              __builtin_amdgcn_s_sleep(2);
            }
            pre += v & kPartSize;
          }
          if (g == kSplitParts - 1 && pre + n != c)
            atomicOr((unsigned long long *)err, (unsigned long long)kErrInconsistent);
        } else if (n != c) {
          atomicOr((unsigned long long *)err, (unsigned long long)kErrInconsistent);
        }
        s_off = pre;
      }
      __syncthreads();
      const int64_t o = p.c_rp[row] + s_off;
      const int64_t lim = max((int64_t)0, min((int64_t)n, p.c_capacity - o));
      if (threadIdx.x == 0 && lim < n) atomicOr((unsigned long long *)err, (unsigned long long)kErrCapacity);
      // the table holds no key above the highest slot one was inserted at
      if (work) wg_global_extract(gkeys, gvals, min(alloc, (int64_t)ws.top + 1), ws.dmax, ws, xl, p.c_col + o,
                                  p.c_val + o, lim);
    }
    __syncthreads();
  }
}


// ============================================ workgroup tier: bitmap window
// The paper's MinMax store keeps a dense temporary row over the column
// region [lo, hi] of the row (Section IV-B).  On the GPU that region lives
// in a workgroup's LDS as one bit per column (a 2^20-column region is
// 128 KB), with a running count per group of kBitmapGroup words.
//   counting pass: every product sets its column's bit; the row's size is
//     the number of bits it set first.
//   numeric pass: the bits are set again and their ranks (the count of set
//     bits before each) summed per group; the row's columns are written to C
//     in order, its values cleared to +0.0, and every product adds a*b into
//     the value at its column's rank, the products in A's order
//     (wg_apply_in_order), i.e. exactly the accumulation of the row-major
//     kernel (Section IV-A) into C itself: no table, no sort.
// Dynamic LDS: the window's words, then (numeric) the group counts and the
// step set.
__host__ __device__ inline int32_t bitmap_groups(int32_t words) { return (words + kBitmapGroup - 1) / kBitmapGroup; }
size_t bitmap_lds_bytes(int32_t words, int mode) {
  size_t b = (size_t)words * 4;
  if (mode == kNumeric) b += (size_t)bitmap_groups(words) * 4 + (size_t)kDupSlots * 4;
  return b;
}

// Rank of window position x: set bits before it.
__device__ __forceinline__ int32_t bm_rank(const uint32_t *bm, const int32_t *pre, int32_t x) {
  const int32_t w = x >> 5;
  int32_t r = pre[w / kBitmapGroup];
  for (int32_t k = w & ~(kBitmapGroup - 1); k < w; ++k) r += __popc(bm[k]);
  return r + __popc(bm[w] & ((1u << (x & 31)) - 1u));
}

// Sets the bits of the row's products' columns; returns (through ws.cnt
// after the closing barrier) the number of bits set first.
__device__ int32_t wg_bitmap_fill(const Operands &op, int64_t row, int32_t lo, int32_t nw, uint32_t *bm,
                                  WgScratch &ws) {
  for (int32_t w = threadIdx.x; w < nw; w += kBlock) bm[w] = 0u;
  if (threadIdx.x == 0) ws.cnt = 0;
  __syncthreads();
  int32_t nnew = 0;
  const int64_t as = op.a_rp[row], ae = op.a_rp[row + 1];
  for (int64_t eb = as; eb < ae; eb += kBlock) {
    const int64_t tot = wg_stage_entries(op, eb, ae, 0, -1, ws, false);
    for (int64_t q0 = 0; q0 < tot; q0 += kWgChunk) {
      int64_t bpos[kWgProducts];
      double av[kWgProducts];
      bool live[kWgProducts];
      int32_t j[kWgProducts];
      wg_step_products(ws, q0, tot, bpos, av, live);
#pragma unroll
      for (int u = 0; u < kWgProducts; ++u) j[u] = live[u] ? op.b_col[bpos[u]] - lo : 0;
#pragma unroll
      for (int u = 0; u < kWgProducts; ++u) {
        if (!live[u]) continue;
        const uint32_t bit = 1u << (j[u] & 31);
        nnew += (atomicOr(&bm[j[u] >> 5], bit) & bit) ? 0 : 1;
      }
    }
    __syncthreads();
  }
  const int32_t wn = (int32_t)wave_sum((int64_t)nnew);
  if (lane_id() == 0 && wn) atomicAdd(&ws.cnt, wn);
  __syncthreads();
  return ws.cnt;
}

template <int MODE>
__global__ void __launch_bounds__(kBlock) k_bitmap(BigParams p);

// Windows above 64 KB of dynamic LDS: raises both kernels' limit to the
// largest window (within a compute unit's 160 KB with the static part), once
// per device, outside any stream capture (the plan calls it).
hipError_t bitmap_kernels_prepare() {
  static std::mutex mu;
  static bool raised[64] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  if (dev >= 0 && dev < 64 && raised[dev]) return hipSuccess;
  const int most = (int)bitmap_lds_bytes(kBitmapMaxCols / 32, kNumeric);
  e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_bitmap<kSymbolic>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, most);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_bitmap<kNumeric>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, most);
  if (e == hipSuccess && dev >= 0 && dev < 64) raised[dev] = true;
  return e;
}

template <int MODE>
__global__ void __launch_bounds__(kBlock) k_bitmap(BigParams p) {
  __shared__ WgScratch ws;
  extern __shared__ uint32_t bm_lds[];
  const int32_t W = p.bitmap_words;
  uint32_t *bm = bm_lds;
  int32_t *pre = reinterpret_cast<int32_t *>(bm_lds + W);
  int32_t *dset = pre + bitmap_groups(W);
  const Operands &op = p.op;
  const int t = threadIdx.x;
  const int64_t nbig = p.counters[p.count_ctr];
  const int64_t nh = p.huge_ctr >= 0 ? p.counters[p.huge_ctr] : nbig;
  int64_t *err = p.counters + kCtrError;
  if (MODE == kNumeric)
    for (int q = t; q < kDupSlots; q += kBlock) dset[q] = kEmpty;
  __shared__ int64_t s_i;
  while (true) {
    if (t == 0) s_i = (int64_t)atomicAdd((unsigned long long *)&p.counters[kCtrBigTicket], 1ull);
    __syncthreads();
    const int64_t i = s_i;
    __syncthreads();
    if (i >= nbig) break;
    const int64_t row = i < nh ? p.list[i] : p.list[p.list_len - 1 - (i - nh)];
    const int32_t lo = p.lo[row];
    const int64_t nw64 = (((int64_t)p.hi[row] - lo) >> 5) + 1;
    if (p.hi[row] < lo || nw64 > W) {
      // not a window this launch holds (the host sizes it by B's columns)
      if (t == 0) atomicOr((unsigned long long *)err, (unsigned long long)kErrScratch);
      continue;
    }
    const int32_t nw = (int32_t)nw64;
    const int32_t n = wg_bitmap_fill(op, row, lo, nw, bm, ws);
    if (MODE == kSymbolic) {
      if (t == 0) p.cnt[row] = n;
      continue;
    }
    const int64_t c = p.cnt[row];
    const int64_t o = p.c_rp[row];
    const int64_t lim = max((int64_t)0, min((int64_t)n, p.c_capacity - o));
    if (t == 0 && n != c) atomicOr((unsigned long long *)err, (unsigned long long)kErrInconsistent);
    if (t == 0 && lim < n) atomicOr((unsigned long long *)err, (unsigned long long)kErrCapacity);
    // group counts, then their exclusive sums: thread t takes a run of groups
    const int32_t ng = bitmap_groups(nw);
    const int32_t per = (ng + kBlock - 1) / kBlock, g0 = min(t * per, ng), g1 = min(g0 + per, ng);
    int64_t mine = 0;
    for (int32_t g = g0; g < g1; ++g) {
      int32_t sg = 0;
      for (int32_t w = g * kBitmapGroup; w < min((g + 1) * kBitmapGroup, nw); ++w) sg += __popc(bm[w]);
      pre[g] = sg;
      mine += sg;
    }
    int64_t tot;
    int64_t run = block_exclusive_sum(mine, ws.wtot, &tot);
    for (int32_t g = g0; g < g1; ++g) {
      const int32_t sg = pre[g];
      pre[g] = (int32_t)run;
      run += sg;
    }
    __syncthreads();
    // the row's columns into C in order, their values cleared to +0.0
    int32_t *ccol = p.c_col + o;
    double *cval = p.c_val + o;
    for (int32_t w = t; w < nw; w += kBlock) {
      uint32_t x = bm[w];
      if (!x) continue;
      int32_t r = bm_rank(bm, pre, w << 5);
      while (x) {
        const int b = __builtin_ctz(x);
        x &= x - 1;
        if (r < lim) {
          ccol[r] = lo + (w << 5) + b;
          gstored(cval + r, 0.0);
        }
        ++r;
      }
    }
    wave_mem_wait();
    wg_sync_global();
    // values in A's order into the value at each column's rank
    const int64_t as = op.a_rp[row], ae = op.a_rp[row + 1];
    for (int64_t eb = as; eb < ae; eb += kBlock) {
      const int64_t tot2 = wg_stage_entries(op, eb, ae, 0, -1, ws, true);
      for (int64_t q0 = 0; q0 < tot2; q0 += kWgChunk) {
        int64_t bpos[kWgProducts];
        double a[kWgProducts], b[kWgProducts];
        bool live[kWgProducts];
        int32_t j[kWgProducts], r[kWgProducts];
        wg_step_products(ws, q0, tot2, bpos, a, live);
#pragma unroll
        for (int u = 0; u < kWgProducts; ++u) {
          j[u] = live[u] ? op.b_col[bpos[u]] : 0;
          b[u] = live[u] ? op.b_val[bpos[u]] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kWgProducts; ++u) r[u] = live[u] ? bm_rank(bm, pre, j[u] - lo) : 0;
        if (p.fast) {
#pragma unroll
          for (int u = 0; u < kWgProducts; ++u) {
            if (!live[u] || r[u] >= lim) continue;
            double pr;
            {
#pragma clang fp contract(off)
              pr = a[u] * b[u];
            }
            atomicAdd(cval + r[u], pr);
          }
          continue;
        }
        wg_apply_in_order(dset, live, j, [&](const bool *go) {
          double old[kWgProducts];
#pragma unroll
          for (int u = 0; u < kWgProducts; ++u) old[u] = (go[u] && r[u] < lim) ? gloadd(cval + r[u]) : 0.0;
#pragma unroll
          for (int u = 0; u < kWgProducts; ++u)
            if (go[u] && r[u] < lim) gstored(cval + r[u], mul_add_rn(old[u], a[u], b[u]));
          wave_mem_wait();
        });
      }
      __syncthreads();
    }
    wave_mem_wait();
    __syncthreads();
  }
}

// ===================================================== register-merge rows
// Matrices whose every row is a register-merge row need no tiles and no
// workgroup barriers: one thread per row, 64 consecutive rows per wave.
//   symbolic: merge without values, write the count; per-workgroup partial
//             sums of the multiplication counts and empty rows;
//   numeric:  merge with values into the wave's LDS staging at the row's
//             offset inside the wave's output (known from row_ptr), then
//             copy the wave's contiguous output to C with all 64 lanes
//             (coalesced stores; one store per lane per row would scatter
//             over many cache lines; staging decides how many waves a
//             compute unit holds, so it is sized by the largest wave output).
// The one pass of such matrices runs the two, with the scan between them,
// back to back on the device (no host round trip): a single merge that
// publishes its count only once its values are staged holds every later
// wave in the look-back, and one that counts first merges twice.
__host__ __device__ inline size_t wave_merge_vals_offset(int stage) {
  return (((size_t)kWavesPerBlock * stage * 4) + 15) & ~(size_t)15;
}
__host__ __device__ inline size_t wave_merge_lds(int mode, int stage) {
  if (mode != kNumeric) return 0;
  return wave_merge_vals_offset(stage) + (size_t)kWavesPerBlock * stage * 8;
}

// tiers (not null): only the rows whose tier is the register merge are
// merged (the other rows of a tiled pass are the tile and workgroup kernels';
// a numeric wave that stages copies its whole range, and those kernels,
// launched after it, write their rows over it); no partial sums.
template <int M, int MODE>
__global__ void __launch_bounds__(kBlock, M == 10 ? 3 : (M <= 8 ? 4 : 1))
k_wave_merge(Operands op, int64_t *counters, int32_t *cnt_out, int64_t *partials, const int64_t *c_rp,
             int32_t *c_col, double *c_val, int64_t c_capacity, int stage, const uint32_t *tiers) {
  extern __shared__ __align__(16) unsigned char wm_lds[];
  const int l = lane_id();
  const int w = threadIdx.x / kWave;
  if (MODE == kSymbolic) {
    // counts, and the workgroup's sums of multiplication counts and empty rows
    __shared__ int64_t s_part[2][kWavesPerBlock];
    const int64_t row = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int64_t n = 0, ub = 0;
    if (row < op.rows && (!tiers || info_tier(tiers[row]) == kTierMerge)) {
      n = merge_row<M, false>(op, row, nullptr, nullptr, 0, &ub);
      cnt_out[row] = (int32_t)n;
    }
    if (tiers) return;
    const int64_t wu = wave_sum(ub), we = wave_sum(row < op.rows && ub == 0 ? 1 : 0);
    if (l == 0) {
      s_part[0][w] = wu;
      s_part[1][w] = we;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t a = 0, b = 0;
      for (int q = 0; q < kWavesPerBlock; ++q) {
        a += s_part[0][q];
        b += s_part[1][q];
      }
      partials[2 * blockIdx.x] = a;
      partials[2 * blockIdx.x + 1] = b;
    }
    return;
  }
  if (MODE == kComputeOnly) {
    // every entry accumulated as in the numeric pass, none stored: the
    // row's count and largest magnitude are all that leave the chip
    const int64_t row = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (row < op.rows) {
      double mx = 0.0;
      const int64_t n = merge_row<M, true>(op, row, nullptr, nullptr, 0, nullptr, &mx);
      cnt_out[row] = (int32_t)n;
      c_val[row] = mx;
    }
    return;
  }
  // numeric: this wave's staging, `stage` columns, then `stage` values
  int32_t *scw = reinterpret_cast<int32_t *>(wm_lds) + (size_t)w * stage;
  double *svw = reinterpret_cast<double *>(wm_lds + wave_merge_vals_offset(stage)) + (size_t)w * stage;
  const int64_t row0 = ((int64_t)blockIdx.x * kWavesPerBlock + w) * kWave;
  if (row0 >= op.rows) return;   // whole wave past the end
  const int64_t row = row0 + l;
  const bool valid = row < op.rows;
  const int64_t base = c_rp[row0];
  const int64_t tot = c_rp[min(row0 + kWave, op.rows)] - base;
  const int64_t o = valid ? c_rp[row] - base : 0;
  const int64_t n = valid ? c_rp[row + 1] - c_rp[row] : 0;
  const bool staged = tot <= stage;
  const bool mine = valid && (!tiers || info_tier(tiers[row]) == kTierMerge);
  if (staged && mine) {
    const int64_t got = merge_row<M, true>(op, row, scw + o, svw + o, n);
    if (got != n) atomicOr((unsigned long long *)&counters[kCtrError], (unsigned long long)kErrInconsistent);
  }
  const int64_t lim = max((int64_t)0, min(tot, c_capacity - base));
  if (lim < tot && l == 0) atomicOr((unsigned long long *)&counters[kCtrError], (unsigned long long)kErrCapacity);
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  if (staged) {
    for (int64_t q = l; q < lim; q += kWave) put_c(c_col, c_val, base + q, scw[q], svw[q]);
  } else if (!staged && mine) {
    // the wave's output does not fit the staging: rows write their own entries
    const int64_t rl = max((int64_t)0, min(n, lim - o));
    const int64_t got = merge_row<M, true>(op, row, c_col + base + o, c_val + base + o, rl);
    if (got != n) atomicOr((unsigned long long *)&counters[kCtrError], (unsigned long long)kErrInconsistent);
  }
}

template <int M, int MODE>
static hipError_t launch_wave_merge_mm(const Operands &op, int stage, int64_t *counters, int32_t *cnt_out,
                                       int64_t *partials, const int64_t *c_rp, int32_t *c_col, double *c_val,
                                       int64_t c_capacity, hipStream_t s, const uint32_t *tiers = nullptr) {
  const size_t lds = wave_merge_lds(MODE, stage);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_wave_merge<M, MODE>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const int64_t blocks = (op.rows + kBlock - 1) / kBlock;
  hipLaunchKernelGGL((k_wave_merge<M, MODE>), dim3((unsigned)blocks), dim3(kBlock), lds, s, op, counters, cnt_out,
                     partials, c_rp, c_col, c_val, c_capacity, stage, tiers);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || MODE != kSymbolic || tiers) return e;
  const int32_t dst[2] = {kCtrMults, kCtrEmpty};
  return launch_sum_partials(partials, blocks, 2, 2, dst, nullptr, counters, s);
}

template <int M>
static hipError_t launch_wave_merge_m(const Operands &op, int mode, int stage, int64_t *counters, int32_t *cnt_out,
                                      int64_t *partials, const int64_t *c_rp, int32_t *c_col, double *c_val,
                                      int64_t c_capacity, hipStream_t s) {
  if (mode == kSymbolic)
    return launch_wave_merge_mm<M, kSymbolic>(op, stage, counters, cnt_out, partials, c_rp, c_col, c_val, c_capacity,
                                              s);
  if (mode == kNumeric)
    return launch_wave_merge_mm<M, kNumeric>(op, stage, counters, cnt_out, partials, c_rp, c_col, c_val, c_capacity,
                                             s);
  if (mode == kComputeOnly)
    return launch_wave_merge_mm<M, kComputeOnly>(op, 0, counters, cnt_out, partials, c_rp, c_col, c_val, c_capacity,
                                                 s);
  return hipErrorInvalidValue;
}

hipError_t launch_wave_merge(const Operands &op, int mode, int merge_lists, int stage, int64_t *counters,
                             int32_t *cnt_out, int64_t *partials, const int64_t *c_rp, int32_t *c_col,
                             double *c_val, int64_t c_capacity, hipStream_t s) {
  if (op.rows <= 0) return hipSuccess;
  switch (merge_lists) {
    case 4: return launch_wave_merge_m<4>(op, mode, stage, counters, cnt_out, partials, c_rp, c_col, c_val, c_capacity, s);
    case 6: return launch_wave_merge_m<6>(op, mode, stage, counters, cnt_out, partials, c_rp, c_col, c_val, c_capacity, s);
    case 8: return launch_wave_merge_m<8>(op, mode, stage, counters, cnt_out, partials, c_rp, c_col, c_val, c_capacity, s);
    case 10: return launch_wave_merge_m<10>(op, mode, stage, counters, cnt_out, partials, c_rp, c_col, c_val, c_capacity, s);
    case 16: return launch_wave_merge_m<16>(op, mode, stage, counters, cnt_out, partials, c_rp, c_col, c_val, c_capacity, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_wave_merge_tiered(const Operands &op, int mode, int merge_lists, int stage, const uint32_t *tiers,
                                    int64_t *counters, int32_t *cnt_out, const int64_t *c_rp, int32_t *c_col,
                                    double *c_val, int64_t c_capacity, hipStream_t s) {
  if (op.rows <= 0) return hipSuccess;
  if (mode != kSymbolic && mode != kNumeric) return hipErrorInvalidValue;
  const bool sym = mode == kSymbolic;
  switch (merge_lists) {
    case 4:
      return sym ? launch_wave_merge_mm<4, kSymbolic>(op, 0, counters, cnt_out, nullptr, c_rp, c_col, c_val,
                                                       c_capacity, s, tiers)
                 : launch_wave_merge_mm<4, kNumeric>(op, stage, counters, cnt_out, nullptr, c_rp, c_col, c_val,
                                                      c_capacity, s, tiers);
    case 8:
      return sym ? launch_wave_merge_mm<8, kSymbolic>(op, 0, counters, cnt_out, nullptr, c_rp, c_col, c_val,
                                                       c_capacity, s, tiers)
                 : launch_wave_merge_mm<8, kNumeric>(op, stage, counters, cnt_out, nullptr, c_rp, c_col, c_val,
                                                      c_capacity, s, tiers);
    default: return hipErrorInvalidValue;
  }
}

size_t wave_tile_lds(int mode, int table_slots, int stage_slots) {
  return wave_lds_layout(mode != kSymbolic, table_slots, stage_slots).total;
}

template <int MODE, int M, bool MERGE, bool ESCO = false, bool BIG = false>
static hipError_t launch_wt_mm(const WaveTileParams &wp, size_t lds, hipStream_t s) {
  const void *fn = reinterpret_cast<const void *>(&k_wt<MODE, M, MERGE, ESCO, BIG>);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const int64_t grid = std::min<int64_t>(wp.ntiles, 0x7fffffff);
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_wt<MODE, M, MERGE, ESCO, BIG>), dim3((unsigned)grid), dim3(kWave), lds, s, wp);
  return hipGetLastError();
}

template <int M, bool MERGE>
static hipError_t launch_wt_m(const WaveTileParams &wp, int mode, size_t lds, hipStream_t s) {
  switch (mode) {
    case kSymbolic: return launch_wt_mm<kSymbolic, M, MERGE>(wp, lds, s);
    case kNumeric: return launch_wt_mm<kNumeric, M, MERGE>(wp, lds, s);
    default: return launch_wt_mm<kOnePass, M, MERGE>(wp, lds, s);
  }
}

hipError_t launch_wave_tiles(const WaveTileParams &wp, int mode, int merge_lists, bool has_merge, bool esc_only,
                             bool esc_big, hipStream_t s) {
  const size_t lds = wave_tile_lds(mode, wp.table_slots, wp.stage_slots);
  if (esc_big && (mode != kNumeric || has_merge)) return hipErrorInvalidValue;   // sizing never asks for it
  if (esc_big)
    return esc_only ? launch_wt_mm<kNumeric, 4, false, true, true>(wp, lds, s)
                    : launch_wt_mm<kNumeric, 4, false, false, true>(wp, lds, s);
  if (esc_only && !has_merge) {
    if (mode == kSymbolic) return launch_wt_mm<kSymbolic, 4, false, true>(wp, lds, s);
    return mode == kNumeric ? launch_wt_mm<kNumeric, 4, false, true>(wp, lds, s)
                            : launch_wt_mm<kOnePass, 4, false, true>(wp, lds, s);
  }
  if (!has_merge) return launch_wt_m<4, false>(wp, mode, lds, s);
  switch (merge_lists) {
    case 4: return launch_wt_m<4, true>(wp, mode, lds, s);
    case 8: return launch_wt_m<8, true>(wp, mode, lds, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_big_rows(const BigParams &bp, int mode, int grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  hipError_t e = launch_fill_i64(bp.counters + kCtrBigTicket, 0, 1, s);
  if (e != hipSuccess) return e;
  if (bp.split) {
    e = launch_fill_i64(bp.parts, 0, kMaxSplitRows * (kSplitParts + 1), s);
    if (e != hipSuccess) return e;
  }
  if (bp.bitmap_words > 0) {
    const size_t lds = bitmap_lds_bytes(bp.bitmap_words, mode == kSymbolic ? kSymbolic : kNumeric);

    if (mode == kSymbolic)
      hipLaunchKernelGGL(k_bitmap<kSymbolic>, dim3(bp.grid_bitmap), dim3(kBlock), lds, s, bp);
    else
      hipLaunchKernelGGL(k_bitmap<kNumeric>, dim3(bp.grid_bitmap), dim3(kBlock), lds, s, bp);
    return hipGetLastError();
  }
  if (mode == kSymbolic) hipLaunchKernelGGL(k_big<kSymbolic>, dim3(grid), dim3(kBlock), 0, s, bp);
  else hipLaunchKernelGGL(k_big<kNumeric>, dim3(grid), dim3(kBlock), 0, s, bp);
  return hipGetLastError();
}

}  // namespace spg

