// HIP kernels of the SpGEMM pipeline for gfx950 (CDNA4, wave64).
//
// C = A * B on CSR FP64 operands, row by row as in the paper's row-major
// (Gustavson) algorithm, Section IV-A: row r of C accumulates a(r,c) * b(c,x)
// over the stored entries of row r of A (in stored order) and of row c of B.
// Output rows are sorted by column (Section IV-B append contract).
//
// Pipeline: features -> sizing/tiering -> scan of tile costs -> tile bounds
// -> tile kernel (symbolic, numeric, or one pass with decoupled look-back).
#include <algorithm>

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
// Features of row i (see above); rows of at most 8 stored entries issue
// all their loads at once (two dependent gather rounds per row).
template <bool SPAN>
__device__ __forceinline__ void row_features(const Operands &op, int64_t i, int64_t &m, int64_t &ub, int32_t &mx,
                                             int32_t &lo, int32_t &hi) {
  const int64_t s = op.a_rp[i], e = op.a_rp[i + 1];
  m = e - s;
  ub = 0;
  mx = 0;
  lo = 0x7fffffff;
  hi = -1;
  if (m <= 8) {
    int32_t k[8];
    int64_t bs[8], be[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) k[q] = q < m ? op.a_col[s + q] : 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      bs[q] = q < m ? op.b_rp[k[q]] : 0;
      be[q] = q < m ? op.b_rp[k[q] + 1] : 0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int32_t len = (int32_t)(be[q] - bs[q]);
      ub += len;
      mx = max(mx, len);
      if (SPAN && len > 0) {
        lo = min(lo, op.b_col[bs[q]]);
        hi = max(hi, op.b_col[be[q] - 1]);
      }
    }
  } else {
    for (int64_t q = s; q < e; ++q) {
      const int32_t k = op.a_col[q];
      const int64_t bs = op.b_rp[k], be = op.b_rp[k + 1];
      const int32_t len = (int32_t)(be - bs);
      ub += len;
      mx = max(mx, len);
      if (SPAN && len > 0) {
        lo = min(lo, op.b_col[bs]);
        hi = max(hi, op.b_col[be - 1]);
      }
    }
  }
}

// Packed feature triple of a row (the learned sizer's input): entries of the
// A row (21 bits), multiplication count saturated at B.cols (22 bits),
// longest selected B row (20 bits); all ones when a field does not fit.
__device__ __forceinline__ uint64_t pack_triple(int64_t m, int64_t ub, int32_t mx, int32_t b_cols) {
  const int64_t u = min(ub, (int64_t)b_cols);
  if (m >= (1 << 21) || u >= (1 << 22) || mx >= (1 << 20)) return ~0ull;
  return (uint64_t)m | ((uint64_t)u << 21) | ((uint64_t)mx << 43);
}

// MODE 0: partial sums only.  MODE 1: also the packed triple of every row.
// MODE 2: also the per-row plan arrays (entries, saturated count, longest
// B row, column span) for tiled passes.
template <int MODE>
__global__ void __launch_bounds__(kBlock) k_features(Operands op, Features f, uint64_t *keys, int64_t *partials) {
  __shared__ int64_t s_sum[4][kWavesPerBlock];
  const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  int64_t ub = 0, m = 0, empty = 0, unpacked = 0;
  if (i < op.rows) {
    int32_t mx, lo, hi;
    row_features<MODE == 2>(op, i, m, ub, mx, lo, hi);
    if (MODE == 1) {
      keys[i] = pack_triple(m, ub, mx, op.b_cols);
      if (keys[i] == ~0ull) unpacked = min(ub, (int64_t)op.b_cols);
    }
    if (MODE == 2) {
      f.nnz_a[i] = (int32_t)m;
      f.ub[i] = (int32_t)min(ub, (int64_t)op.b_cols);
      f.maxb[i] = mx;
      f.lo[i] = lo;
      f.hi[i] = hi;
    }
    empty = ub == 0 ? 1 : 0;
  }
  int64_t ws = wave_sum(ub), we = wave_sum(empty), wu = wave_sum(unpacked), wm = m;
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) wm = max(wm, __shfl_xor(wm, d, kWave));
  if (lane_id() == 0) {
    s_sum[0][threadIdx.x / kWave] = ws;
    s_sum[1][threadIdx.x / kWave] = wm;
    s_sum[2][threadIdx.x / kWave] = we;
    s_sum[3][threadIdx.x / kWave] = wu;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t t = 0, tm = 0, te = 0, tu = 0;
    for (int j = 0; j < kWavesPerBlock; ++j) {
      t += s_sum[0][j];
      tm = max(tm, s_sum[1][j]);
      te += s_sum[2][j];
      tu += s_sum[3][j];
    }
    partials[blockIdx.x * 4 + 0] = t;
    partials[blockIdx.x * 4 + 1] = tm;
    partials[blockIdx.x * 4 + 2] = te;
    partials[blockIdx.x * 4 + 3] = tu;
  }
}

// Longest row of A (row pointers only).
__global__ void __launch_bounds__(kBlock) k_row_max(const int64_t *rp, int64_t rows, int64_t *partials) {
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
struct PartialSpec {
  int32_t n, stride;
  int32_t dst[8];
  int32_t is_max[8];
};

__global__ void __launch_bounds__(kBlock) k_sum_partials(const int64_t *partials, int64_t nblocks, PartialSpec ps,
                                                         int64_t *counters) {
  __shared__ int64_t red[8][kWavesPerBlock];
  for (int j = 0; j < ps.n; ++j) {
    int64_t acc = 0;
    for (int64_t b = threadIdx.x; b < nblocks; b += kBlock) {
      int64_t v = partials[b * ps.stride + j];
      acc = ps.is_max[j] ? max(acc, v) : acc + v;
    }
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
      int64_t o = __shfl_xor(acc, d, kWave);
      acc = ps.is_max[j] ? max(acc, o) : acc + o;
    }
    if (lane_id() == 0) red[j][threadIdx.x / kWave] = acc;
  }
  __syncthreads();
  if (threadIdx.x < ps.n) {
    int j = threadIdx.x;
    int64_t acc = 0;
    for (int q = 0; q < kWavesPerBlock; ++q) acc = ps.is_max[j] ? max(acc, red[j][q]) : acc + red[j][q];
    counters[ps.dst[j]] = acc;
  }
}

hipError_t launch_sum_partials(const int64_t *partials, int64_t nblocks, int n, int stride, const int32_t *dst,
                               const int32_t *is_max, int64_t *counters, hipStream_t s) {
  PartialSpec ps{};
  ps.n = n;
  ps.stride = stride;
  for (int j = 0; j < n; ++j) {
    ps.dst[j] = dst[j];
    ps.is_max[j] = is_max ? is_max[j] : 0;
  }
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBlock), 0, s, partials, nblocks, ps, counters);
  return hipGetLastError();
}

hipError_t launch_features(const Operands &op, const Features &f, uint64_t *keys, int64_t *counters,
                           int64_t *partials, int mode, hipStream_t s) {
  if (op.rows <= 0) return launch_fill_i64(counters + kCtrMults, 0, 1, s);
  const int64_t blocks = (op.rows + kBlock - 1) / kBlock;
  if (mode == 2) hipLaunchKernelGGL(k_features<2>, dim3((unsigned)blocks), dim3(kBlock), 0, s, op, f, keys, partials);
  else if (mode == 1) hipLaunchKernelGGL(k_features<1>, dim3((unsigned)blocks), dim3(kBlock), 0, s, op, f, keys, partials);
  else hipLaunchKernelGGL(k_features<0>, dim3((unsigned)blocks), dim3(kBlock), 0, s, op, f, keys, partials);
  const int32_t dst[4] = {kCtrMults, kCtrMaxA, kCtrEmpty, kCtrUnpacked};
  const int32_t mx[4] = {0, 1, 0, 0};
  return launch_sum_partials(partials, blocks, 4, 4, dst, mx, counters, s);
}

hipError_t launch_row_max(const int64_t *rp, int64_t rows, int64_t *counters, int64_t *partials, hipStream_t s) {
  if (rows <= 0) return launch_fill_i64(counters + kCtrMaxA, 0, 1, s);
  const int64_t blocks = std::min<int64_t>(1024, (rows + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_row_max, dim3((unsigned)blocks), dim3(kBlock), 0, s, rp, rows, partials);
  const int32_t dst[1] = {kCtrMaxA};
  const int32_t mx[1] = {1};
  return launch_sum_partials(partials, blocks, 1, 1, dst, mx, counters, s);
}

// ------------------------------------------------------------ sizing/tiers
// Table of a hashed row: T slots for capacity c (load <= 1/2) plus `pad`
// slots of probe room; a dense window when the column region is at most
// dense_ratio * c (the paper's "Combined" rule of Section IV-B: MinMax when
// the region is smaller than twice the row's entries, Sort otherwise).
__device__ __forceinline__ void table_shape(int64_t span, int64_t c, float dense_ratio, int pad,
                                            bool *dense, int64_t *slots, int64_t *alloc) {
  if ((double)span <= (double)dense_ratio * (double)c) {
    *dense = true;
    *slots = span;
    *alloc = span;
  } else {
    *dense = false;
    *slots = max((int64_t)16, 2 * c);
    *alloc = *slots + pad;
  }
}

// Device table of a workgroup-level row: capacity c, load <= 1/2, and c
// slots of probe room so that linear probing can never run off the end.
__device__ __forceinline__ int64_t global_table_alloc(int64_t span, int64_t c, bool *dense,
                                                       int64_t *slots) {
  if (span <= 2 * c) {
    *dense = true;
    *slots = span;
    return span;
  }
  *dense = false;
  *slots = max((int64_t)16, 2 * c);
  return *slots + c;
}

__global__ void __launch_bounds__(kBlock) k_size_rows(Operands op, PlanArrays pa, SizeParams sp) {
  __shared__ int64_t s_red[7][kWavesPerBlock];
  int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  // Tile budget HT (cost units): half the LDS pool when there is one, so a
  // tile's hashed rows always fit the pool; every row costs at least
  // ceil(HT / tile_rows), so a tile holds at most tile_rows rows.
  const int64_t H = sp.pool_slots / 2;
  const int64_t HT = tile_budget(sp.pool_slots, sp.tile_rows);
  const int64_t mincost = H > 0 ? (H + sp.tile_rows - 1) / sp.tile_rows : 1;
  int64_t n_tier[4] = {0, 0, 0, 0};
  int64_t capsum = 0, scratch = 0, pool_rows = 0;
  if (i < op.rows) {
    int32_t m = pa.f.nnz_a[i];
    int64_t ub = pa.f.ub[i];
    int64_t mx = pa.f.maxb[i];
    int64_t c;
    if (sp.mode == kNumeric) {
      c = sp.cnt[i];
    } else if (sp.mode == kOnePass && sp.sizer == 2) {
      c = learned_capacity(sp.pred[i], (int32_t)ub, (int32_t)mx, sp.margin, sp.slack);
    } else {
      c = ub;
    }
    uint32_t tier, info;
    int64_t use = 0, cost;
    if (m == 0 || ub == 0 || c == 0) {
      tier = kTierEmpty;
      c = 0;
      info = pack_info(kTierEmpty, false, 0);
      cost = mincost;
    } else if (m <= sp.merge_lists && c <= sp.merge_max && (sp.mode == kSymbolic || c <= H)) {
      // register merge; the passes that write values stage the row in LDS
      tier = kTierMerge;
      info = pack_info(kTierMerge, false, 0);
      use = (sp.mode == kSymbolic) ? 0 : c;
      cost = max(use, mincost);
    } else {
      int64_t span = (int64_t)pa.f.hi[i] - (int64_t)pa.f.lo[i] + 1;
      bool dense;
      int64_t slots, alloc;
      table_shape(span, c, sp.dense_ratio, sp.pad, &dense, &slots, &alloc);
      if (alloc <= H) {
        tier = kTierHash;
        info = pack_info(kTierHash, dense, (uint32_t)slots);
        use = alloc;
        cost = max(use, mincost);
      } else {
        tier = kTierGlobal;
        info = pack_info(kTierGlobal, false, 0);
        cost = HT;
      }
      // device table for a workgroup-level pass over this row (a global row,
      // or a hashed row whose probes ran past its LDS slice)
      if (tier == kTierGlobal || !dense) {
        int64_t cg = (sp.mode == kNumeric) ? c : ub;
        bool dg;
        int64_t sg;
        scratch = global_table_alloc(span, cg, &dg, &sg);
      }
    }
    pa.info[i] = info;
    pa.cap[i] = (int32_t)c;
    pa.cost[i] = cost;
    pool_rows = use > 0 ? 1 : 0;
    n_tier[tier] = 1;
    capsum = c;
  }
  int w = threadIdx.x / kWave;
  int64_t v[7] = {n_tier[1], n_tier[2], n_tier[3], n_tier[0], capsum, pool_rows, scratch};
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    int64_t t = wave_sum(v[j]);
    if (lane_id() == 0) s_red[j][w] = t;
  }
  {
    int64_t t = v[6];
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) t = max(t, __shfl_xor(t, d, kWave));
    if (lane_id() == 0) s_red[6][w] = t;
  }
  __syncthreads();
  // one partial per workgroup; k_sum_partials adds them (no hot atomics)
  if (threadIdx.x < 7) {
    int j = threadIdx.x;
    int64_t t = 0;
    for (int q = 0; q < kWavesPerBlock; ++q) t = (j == 6) ? max(t, s_red[j][q]) : t + s_red[j][q];
    pa.partials[(int64_t)blockIdx.x * 8 + j] = t;
  }
}

hipError_t launch_size_rows(const Operands &op, const PlanArrays &pa, const SizeParams &sp,
                            hipStream_t s) {
  PartialSpec ps{};
  ps.n = 7;
  ps.stride = 8;
  const int32_t dst[7] = {kCtrMerge, kCtrHash, kCtrGlobal, kCtrEmpty, kCtrCapSum, kCtrPoolRows, kCtrScratch};
  for (int j = 0; j < 7; ++j) {
    ps.dst[j] = dst[j];
    ps.is_max[j] = (j == 6);
  }
  if (op.rows <= 0) {
    hipError_t e = launch_fill_i64(pa.partials, 0, 8, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBlock), 0, s, (const int64_t *)pa.partials, (int64_t)1, ps,
                       pa.counters);
    return hipGetLastError();
  }
  const int64_t blocks = (op.rows + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_size_rows, dim3((unsigned)blocks), dim3(kBlock), 0, s, op, pa, sp);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBlock), 0, s, (const int64_t *)pa.partials, blocks, ps,
                     pa.counters);
  return hipGetLastError();
}

// ------------------------------------------------------------------- scan
// Single-pass exclusive scan with decoupled look-back: each workgroup takes
// a ticket, loads 8192 items (coalesced, through LDS), scans them,
// publishes its aggregate and looks back for its prefix.  out[n] receives
// the total.  Safe in place (in == out).
constexpr int kScanItems = 32;
constexpr int kScanTile = kBlock * kScanItems;

template <typename TIn>
__global__ void __launch_bounds__(kBlock) k_scan(const TIn *in, int64_t *out, int64_t n,
                                                  uint64_t *status, int64_t *ticket,
                                                  int64_t *total_dst, int64_t *err) {
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
  int64_t agg;
  int64_t excl = block_exclusive_sum(sum, s_wtot, &agg);
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

hipError_t launch_scan_i32(const int32_t *in, int64_t *out, int64_t n, uint64_t *status,
                           int64_t *ticket, int64_t *total_dst, int64_t *err, hipStream_t s) {
  if (n <= 0) return launch_fill_i64(out, 0, 1, s);
  int64_t tiles = (n + kScanTile - 1) / kScanTile;
  hipError_t e = launch_fill_u64(status, 0, tiles, s);
  if (e != hipSuccess) return e;
  e = launch_fill_i64(ticket, 0, 1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan<int32_t>, dim3((unsigned)tiles), dim3(kBlock), 0, s, in, out, n, status,
                     ticket, total_dst, err);
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
                     status, ticket, (int64_t *)nullptr, err);
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

// ============================================================ tile kernel
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
template <int M, bool VALUES>
__device__ int64_t merge_row(const Operands &op, int64_t row, int32_t *out_col, double *out_val,
                             int64_t lim) {
  const int64_t as = op.a_rp[row];
  const int m = (int)(op.a_rp[row + 1] - as);
  int32_t h[M];
  int64_t pos[M];
  int32_t rem[M];
  double a[M], v[M];
#pragma unroll
  for (int l = 0; l < M; ++l) {
    rem[l] = 0;
    pos[l] = 0;
    a[l] = 0.0;
    if (l < m) {
      int32_t k = op.a_col[as + l];
      if (VALUES) a[l] = op.a_val[as + l];
      int64_t bs = op.b_rp[k];
      pos[l] = bs;
      rem[l] = (int32_t)(op.b_rp[k + 1] - bs);
    }
  }
#pragma unroll
  for (int l = 0; l < M; ++l) {
    h[l] = rem[l] > 0 ? op.b_col[pos[l]] : kColMax;
    v[l] = (VALUES && rem[l] > 0) ? op.b_val[pos[l]] : 0.0;
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
        ++pos[l];
        --rem[l];
        h[l] = rem[l] > 0 ? op.b_col[pos[l]] : kColMax;
        if (VALUES) v[l] = rem[l] > 0 ? op.b_val[pos[l]] : 0.0;
      }
    }
    if (n < lim) {
      out_col[n] = mn;
      if (VALUES) out_val[n] = acc;
    }
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
template <int G, bool VALUES>
__device__ void lds_sort_runs(int32_t *keys, double *vals, int32_t alloc) {
  const int gl = lane_id() & (G - 1);
  for (int32_t s = gl; s < alloc; s += G) {
    if (keys[s] == kEmpty || (s > 0 && keys[s - 1] != kEmpty)) continue;
    for (int32_t q = s + 1; q < alloc; ++q) {
      const int32_t k = keys[q];
      if (k == kEmpty) break;
      const double v = VALUES ? vals[q] : 0.0;
      int32_t at = q;
      while (at > s && keys[at - 1] > k) {
        keys[at] = keys[at - 1];
        if (VALUES) vals[at] = vals[at - 1];
        --at;
      }
      keys[at] = k;
      if (VALUES) vals[at] = v;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// Insert column j with the product a*b into an LDS table (G-lane tier).
template <bool VALUES>
__device__ __forceinline__ void lds_insert(int32_t *keys, double *vals, int32_t alloc, const RowHash &hs,
                                           int32_t j, double a, double b, int32_t &cnt, int32_t &dmax,
                                           bool &ovf) {
  const int32_t h = hs.home(j);
  int32_t s = h;
  while (true) {
    if (s >= alloc) {
      ovf = true;
      break;
    }
    int32_t old = atomicCAS(&keys[s], kEmpty, j);
    if (old == kEmpty) {
      ++cnt;
      if (VALUES) vals[s] = first_add_rn(a, b);
      break;
    }
    if (old == j) {
      if (VALUES) vals[s] = mul_add_rn(vals[s], a, b);
      break;
    }
    ++s;
  }
  dmax = max(dmax, s - h);
}

// --- LDS hash tier: G lanes per row.  A entries are taken in stored order;
// for each, the G lanes cover the B row.  Columns of one B row are distinct,
// so within a step no two lanes touch the same slot, and steps run in
// program order inside the wave: every slot is updated in A's column order
// with plain loads and stores (no floating-point atomics).  The first G
// entries of the next kPrefetch B rows are loaded before any of them is
// inserted, so a row waits for one gather round trip per kPrefetch entries
// of A instead of one per entry.
constexpr int kPrefetch = 8;

template <int G, bool VALUES>
__device__ void hash_row(const Operands &op, int64_t row, int32_t *keys, double *vals, int32_t alloc,
                         const RowHash &hs, int32_t *cnt_out, int32_t *dmax_out, int32_t *ovf_out) {
  const int gl = lane_id() & (G - 1);
  const int64_t as = op.a_rp[row], ae = op.a_rp[row + 1];
  int32_t cnt = 0, dmax = 0;
  bool ovf = false;
  for (int64_t eb = as; eb < ae; eb += G) {
    const int64_t e = eb + gl;
    int64_t bs = 0;
    int32_t bl = 0;
    double av = 0.0;
    if (e < ae) {
      int32_t k = op.a_col[e];
      if (VALUES) av = op.a_val[e];
      bs = op.b_rp[k];
      bl = (int32_t)(op.b_rp[k + 1] - bs);
    }
    const int ne = (int)min((int64_t)G, ae - eb);
    for (int i0 = 0; i0 < ne; i0 += kPrefetch) {
      int32_t jj[kPrefetch];
      double bb[kPrefetch];
#pragma unroll
      for (int u = 0; u < kPrefetch; ++u) {
        const int i = i0 + u;
        const int64_t bsi = __shfl(bs, i & (G - 1), G);
        const int32_t bli = __shfl(bl, i & (G - 1), G);
        const bool live = i < ne && gl < bli;
        jj[u] = live ? op.b_col[bsi + gl] : kEmpty;
        bb[u] = (VALUES && live) ? op.b_val[bsi + gl] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kPrefetch; ++u) {
        const int i = i0 + u;
        if (i >= ne) break;
        const double avi = VALUES ? __shfl(av, i & (G - 1), G) : 0.0;
        if (jj[u] != kEmpty)
          lds_insert<VALUES>(keys, vals, alloc, hs, jj[u], avi, bb[u], cnt, dmax, ovf);
        // B rows longer than G: the rest of this row, still before entry i + 1
        const int32_t bli = __shfl(bl, i & (G - 1), G);
        if (bli > G) {
          const int64_t bsi = __shfl(bs, i & (G - 1), G);
          for (int32_t f = G + gl; f < bli; f += G) {
            const int32_t j = op.b_col[bsi + f];
            const double b = VALUES ? op.b_val[bsi + f] : 0.0;
            lds_insert<VALUES>(keys, vals, alloc, hs, j, avi, b, cnt, dmax, ovf);
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      }
    }
  }
  // every lane takes part in every shuffle (no short-circuit around them)
  int32_t of = ovf ? 1 : 0;
#pragma unroll
  for (int d = G / 2; d > 0; d >>= 1) {
    cnt += __shfl_xor(cnt, d, G);
    dmax = max(dmax, __shfl_xor(dmax, d, G));
    of |= __shfl_xor(of, d, G);
  }
  if (gl == 0) {
    *cnt_out = cnt;
    *dmax_out = dmax;
    *ovf_out = of;
  }
  if (VALUES && dmax > 0 && !of) lds_sort_runs<G, VALUES>(keys, vals, alloc);
}

// The per-workgroup tables live in device memory and are written by
// several waves: initial stores, atomic claims (performed in L2) and value
// updates.  Reads go around the L1 cache (agent-scope atomic loads), and
// phases are separated by agent-scope fences on both sides of the barrier,
// so a late initial store can never land on a claimed slot and no wave
// reads a stale L1 line.
__device__ __forceinline__ int32_t gload(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double gloadd(const double *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void gstored(double *p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void wg_sync_global() {
  __threadfence();
  __syncthreads();
  __threadfence();
}

// Write the sorted row held by an LDS table (G lanes).
template <int G, bool VALUES>
__device__ void hash_extract(const int32_t *keys, const double *vals, int32_t alloc, int32_t *out_col,
                             double *out_val, int64_t lim) {
  const int gl = lane_id() & (G - 1);
  const uint64_t gm = group_mask<G>();
  const uint64_t lt = lanemask_lt();
  int64_t run = 0;
  for (int32_t c = 0; c < alloc; c += G) {
    const int32_t s = c + gl;
    const int32_t key = s < alloc ? keys[s] : kEmpty;
    const bool occ = key != kEmpty;
    const uint64_t bal = ballot(occ) & gm;
    if (occ) {
      const int64_t rank = run + __popcll(bal & lt);
      if (rank < lim) {
        out_col[rank] = key;
        if (VALUES) out_val[rank] = vals[s];
      }
    }
    run += __popcll(bal);
  }
}

// --- workgroup-level rows in a per-workgroup device table.
struct WgScratch {
  int64_t pref[kBlock + 1];
  int64_t bs[kBlock];
  double av[kBlock];
  int64_t wtot[kWavesPerBlock + 1];
  int32_t cnt, dmax;
  int64_t run;
};

// Products of the row enumerated flat over the workgroup, 256 A entries at
// a time; fn(q_a_index, b_position, a_value) is called once per product.
template <typename Fn>
__device__ void wg_for_products(const Operands &op, int64_t row, WgScratch &ws, Fn fn) {
  const int64_t as = op.a_rp[row], ae = op.a_rp[row + 1];
  for (int64_t eb = as; eb < ae; eb += kBlock) {
    const int64_t e = eb + threadIdx.x;
    int64_t bs = 0, bl = 0;
    double av = 0.0;
    if (e < ae) {
      int32_t k = op.a_col[e];
      av = op.a_val ? op.a_val[e] : 0.0;
      bs = op.b_rp[k];
      bl = op.b_rp[k + 1] - bs;
    }
    int64_t tot;
    int64_t ex = block_exclusive_sum(bl, ws.wtot, &tot);
    ws.pref[threadIdx.x] = ex;
    ws.bs[threadIdx.x] = bs;
    ws.av[threadIdx.x] = av;
    __syncthreads();
    for (int64_t q = threadIdx.x; q < tot; q += kBlock) {
      int lo = 0, hi = kBlock - 1;
      while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (ws.pref[mid] <= q) lo = mid;
        else hi = mid - 1;
      }
      fn(ws.bs[lo] + (q - ws.pref[lo]), ws.av[lo]);
    }
    __syncthreads();
  }
}

__device__ __forceinline__ int32_t global_probe_insert(int32_t *keys, int64_t alloc, const RowHash &hs,
                                                      int32_t j, bool *is_new, int32_t *disp) {
  int32_t h = hs.home(j);
  int64_t s = h;
  *is_new = false;
  while (s < alloc) {
    int32_t old = atomicCAS(&keys[s], kEmpty, j);
    if (old == kEmpty) {
      *is_new = true;
      break;
    }
    if (old == j) break;
    ++s;
  }
  *disp = (int32_t)(s - h);
  return (int32_t)s;
}

// Slot holding key j (inserted earlier), or -1 if it is missing.
__device__ __forceinline__ int64_t global_find(const int32_t *keys, int64_t alloc, const RowHash &hs, int32_t j) {
  for (int64_t s = hs.home(j); s < alloc; ++s)
    if (gload(keys + s) == j) return s;
  return -1;
}

// Builds the row's key set in the table and returns its size.  The table
// has room for every product (c >= the row's multiplication count or its
// exact size), so no probe leaves it; a key that would is reported through
// *err (kErrInconsistent) rather than dropped silently.
__device__ int32_t wg_global_keys(const Operands &op, int64_t row, int32_t *keys, int64_t alloc,
                                  const RowHash &hs, WgScratch &ws, double *vals_or_null, int64_t *err) {
  for (int64_t s = threadIdx.x; s < alloc; s += kBlock) {
    keys[s] = kEmpty;
    if (vals_or_null) vals_or_null[s] = 0.0;
  }
  if (threadIdx.x == 0) {
    ws.cnt = 0;
    ws.dmax = 0;
  }
  wg_sync_global();
  wg_for_products(op, row, ws, [&](int64_t bpos, double) {
    int32_t j = op.b_col[bpos];
    bool nw;
    int32_t disp;
    int32_t s = global_probe_insert(keys, alloc, hs, j, &nw, &disp);
    if (s >= alloc) atomicOr((unsigned long long *)err, (unsigned long long)kErrInconsistent);
    if (nw) atomicAdd(&ws.cnt, 1);
    if (disp > 0) atomicMax(&ws.dmax, disp);
  });
  wg_sync_global();
  return ws.cnt;
}

// Values of the row into the table built by wg_global_keys.  Ordered: one
// wave takes the A entries in stored order, lanes over the B row (distinct
// columns, so distinct slots), and every entry's updates complete before
// the next entry's begin.  Fast: every product at once with atomic adds.
__device__ void wg_global_values(const Operands &op, int64_t row, const int32_t *keys, double *vals,
                                 int64_t alloc, const RowHash &hs, WgScratch &ws, bool fast) {
  if (fast) {
    wg_for_products(op, row, ws, [&](int64_t bpos, double av) {
      int32_t j = op.b_col[bpos];
      int64_t s = global_find(keys, alloc, hs, j);
      double p;
      {
#pragma clang fp contract(off)
        p = av * op.b_val[bpos];
      }
      if (s >= 0) atomicAdd(&vals[s], p);
    });
  } else if (threadIdx.x < kWave) {
    const int64_t as = op.a_rp[row], ae = op.a_rp[row + 1];
    for (int64_t e = as; e < ae; ++e) {
      int32_t k = op.a_col[e];
      double av = op.a_val[e];
      int64_t bs = op.b_rp[k], be = op.b_rp[k + 1];
      for (int64_t f = bs + threadIdx.x; f < be; f += kWave) {
        int32_t j = op.b_col[f];
        int64_t s = global_find(keys, alloc, hs, j);
        if (s >= 0) gstored(vals + s, mul_add_rn(gloadd(vals + s), av, op.b_val[f]));
      }
      __threadfence();
    }
  }
  wg_sync_global();
}

__device__ __forceinline__ void gstore(int32_t *p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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

// Sorted write-out of a device table by the whole workgroup.
__device__ void wg_global_extract(int32_t *keys, double *vals, int64_t alloc, int32_t dmax, WgScratch &ws,
                                  int32_t *out_col, double *out_val, int64_t lim) {
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

struct TileShared {
  int32_t off[kMaxTileRows];      // LDS pool offset of a row (hash table or merge staging)
  int32_t cnt[kMaxTileRows];
  int32_t dmax[kMaxTileRows];
  int32_t flag[kMaxTileRows];     // 1: the row did not fit its LDS slice
  int64_t out[kMaxTileRows];      // where the row starts in C
  int16_t list[3][kMaxTileRows];  // merge, hash, workgroup-level rows, each in row order
  int32_t nlist[3];
  int64_t tile, tile_excl, tile_total, used;
  int64_t wtot[kWavesPerBlock + 1];
  WgScratch ws;
};

size_t tile_static_lds(int mode) { return sizeof(TileShared); }

// Tile kernel.  A tile is a run of consecutive rows; its rows are tiered
// (merge / LDS hash / workgroup-level) and processed in phases:
//   A  merge rows, one thread each, into LDS staging (or counted only)
//   B  hashed rows, G lanes each, into their LDS tables
//   C  workgroup-level rows and hashed rows that ran out of LDS room,
//      one at a time by the whole workgroup in a device table
//   D  output offsets: from row_ptr (numeric pass) or a workgroup scan plus
//      a decoupled look-back over tiles (one pass)
//   E  write-out: staged merge rows copied by 16-lane groups (contiguous,
//      coalesced), hashed rows extracted in column order by their groups.
// HASH = false compiles phases B/C out for tiles that only hold merge and
// empty rows (fewer registers, more waves per CU).
template <int G, int M, int MODE, bool HASH>
__global__ void __launch_bounds__(kBlock) k_tile(TileParams p) {
  constexpr bool VALUES = (MODE != kSymbolic);
  constexpr int CG = 16;   // lanes per staged row in the copy-out
  extern __shared__ __align__(16) unsigned char pool_raw[];
  __shared__ TileShared sh;
  int32_t *pkeys = reinterpret_cast<int32_t *>(pool_raw);
  double *pvals = reinterpret_cast<double *>(pool_raw + (((size_t)p.pool_slots * 4 + 15) & ~(size_t)15));
  const Operands &op = p.op;
  const int64_t ntiles = p.counters[kCtrTiles];
  int32_t *gkeys = reinterpret_cast<int32_t *>(p.scratch + (size_t)blockIdx.x * (size_t)p.scratch_slots * 12);
  double *gvals = reinterpret_cast<double *>(p.scratch + (size_t)blockIdx.x * (size_t)p.scratch_slots * 12 +
                                             (size_t)p.scratch_slots * 4);
  const int gid = threadIdx.x / G;
  constexpr int NG = kBlock / G;

  while (true) {
    if (threadIdx.x == 0)
      sh.tile = (int64_t)__hip_atomic_fetch_add((unsigned long long *)&p.counters[kCtrTicket], 1ull, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int64_t t = sh.tile;
    if (t >= ntiles) break;
    const int64_t r0 = p.tile_row[t], r1 = p.tile_row[t + 1];
    const int nr = (int)(r1 - r0);

    // ---- classify rows: ordered tier lists and LDS offsets, one packed scan
    // (bits 0-9 merge rows, 10-19 hashed rows, 20-29 workgroup rows, 32-
    // pool slots)
    uint32_t tier2[2];
    int64_t use[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int r = 2 * threadIdx.x + k;
      tier2[k] = kTierEmpty;
      use[k] = 0;
      if (r < nr) {
        const int64_t row = r0 + r;
        const uint32_t inf = p.info[row];
        tier2[k] = info_tier(inf);
        sh.cnt[r] = 0;
        sh.dmax[r] = 0;
        sh.flag[r] = 0;
        if (tier2[k] == kTierHash) use[k] = info_dense(inf) ? info_slots(inf) : info_slots(inf) + p.pad;
        else if (tier2[k] == kTierMerge && VALUES) use[k] = p.cap[row];
        if (MODE == kNumeric) sh.out[r] = p.c_rp[row];
      }
    }
    auto pack = [&](int k) -> int64_t {
      int64_t v = use[k] << 32;
      if (tier2[k] != kTierEmpty) v += (int64_t)1 << (10 * (tier2[k] - 1));
      return v;
    };
    int64_t tot;
    const int64_t ex = block_exclusive_sum(pack(0) + pack(1), sh.wtot, &tot);
    int64_t run = ex;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int r = 2 * threadIdx.x + k;
      if (r < nr) {
        sh.off[r] = (int32_t)(run >> 32);
        if (tier2[k] != kTierEmpty) {
          const int sh10 = 10 * (tier2[k] - 1);
          sh.list[tier2[k] - 1][(run >> sh10) & 1023] = (int16_t)r;
        }
      }
      run += pack(k);
    }
    if (threadIdx.x == 0) {
      sh.nlist[0] = (int32_t)(tot & 1023);
      sh.nlist[1] = (int32_t)((tot >> 10) & 1023);
      sh.nlist[2] = (int32_t)((tot >> 20) & 1023);
      sh.used = tot >> 32;
    }
    __syncthreads();
    if (HASH && sh.nlist[1] > 0) {
      // empty markers for the hashed rows' tables (merge staging needs none)
      for (int i = gid; i < sh.nlist[1]; i += NG) {
        const int r = sh.list[1][i];
        const uint32_t inf = p.info[r0 + r];
        const int32_t alloc = info_dense(inf) ? (int32_t)info_slots(inf) : (int32_t)info_slots(inf) + p.pad;
        for (int32_t q = lane_id() & (G - 1); q < alloc; q += G) pkeys[sh.off[r] + q] = kEmpty;
      }
      __syncthreads();
    }

    // ---- phase A: register-merge rows, one thread each
    for (int i = threadIdx.x; i < sh.nlist[0]; i += kBlock) {
      const int r = sh.list[0][i];
      const int64_t row = r0 + r;
      if (VALUES) {
        const int64_t capr = p.cap[row];
        const int64_t n = merge_row<M, true>(op, row, pkeys + sh.off[r], pvals + sh.off[r], capr);
        sh.cnt[r] = (int32_t)n;
        if (n > capr) {
          sh.flag[r] = 1;   // staging too small (one pass): recomputed at write-out
          if (MODE == kOnePass) atomicAdd((unsigned long long *)&p.counters[kCtrOverflow], 1ull);
        }
        if (MODE == kNumeric && n != capr)
          atomicOr((unsigned long long *)&p.counters[kCtrError], (unsigned long long)kErrInconsistent);
      } else {
        sh.cnt[r] = (int32_t)merge_row<M, false>(op, row, nullptr, nullptr, 0);
      }
    }

    if constexpr (HASH) {
      // ---- phase B: LDS hash rows, G lanes each
      for (int i = gid; i < sh.nlist[1]; i += NG) {
        const int r = sh.list[1][i];
        const int64_t row = r0 + r;
        const uint32_t inf = p.info[row];
        const bool dense = info_dense(inf);
        const int32_t slots = (int32_t)info_slots(inf);
        const int32_t alloc = dense ? slots : slots + p.pad;
        const RowHash hs = make_hash(p.lo[row], p.hi[row], slots, dense);
        hash_row<G, VALUES>(op, row, pkeys + sh.off[r], pvals + sh.off[r], alloc, hs, &sh.cnt[r],
                            &sh.dmax[r], &sh.flag[r]);
      }
      __syncthreads();

      // hashed rows whose LDS probes ran out join the workgroup-level list
      if (threadIdx.x == 0) {
        for (int i = 0; i < sh.nlist[1]; ++i) {
          const int r = sh.list[1][i];
          if (sh.flag[r]) {
            sh.list[2][sh.nlist[2]++] = (int16_t)r;
            atomicAdd((unsigned long long *)&p.counters[kCtrOverflow], 1ull);
          }
        }
      }
      __syncthreads();

      // ---- phase C: workgroup-level rows (count; the numeric pass writes them)
      for (int i = 0; i < sh.nlist[2]; ++i) {
        const int r = sh.list[2][i];
        const int64_t row = r0 + r;
        const int64_t c = (MODE == kNumeric) ? (p.c_rp[row + 1] - p.c_rp[row]) : (int64_t)p.ub[row];
        const int64_t span = (int64_t)p.hi[row] - (int64_t)p.lo[row] + 1;
        bool dense;
        int64_t slots;
        const int64_t alloc = global_table_alloc(span, c, &dense, &slots);
        if (alloc > p.scratch_slots) {
          if (threadIdx.x == 0)
            atomicOr((unsigned long long *)&p.counters[kCtrError], (unsigned long long)kErrScratch);
          continue;
        }
        const RowHash hs = make_hash(p.lo[row], p.hi[row], slots, dense);
        const int32_t n = wg_global_keys(op, row, gkeys, alloc, hs, sh.ws, MODE == kNumeric ? gvals : nullptr,
                                         p.counters + kCtrError);
        if (threadIdx.x == 0) {
          sh.cnt[r] = n;
          sh.dmax[r] = sh.ws.dmax;
        }
        if (MODE == kNumeric) {
          wg_global_values(op, row, gkeys, gvals, alloc, hs, sh.ws, p.fast != 0);
          const int64_t o = sh.out[r];
          const int64_t lim = max((int64_t)0, min((int64_t)n, p.c_capacity - o));
          if (threadIdx.x == 0 && lim < n)
            atomicOr((unsigned long long *)&p.counters[kCtrError], (unsigned long long)kErrCapacity);
          wg_global_extract(gkeys, gvals, alloc, sh.ws.dmax, sh.ws, p.c_col + o, p.c_val + o, lim);
        }
        __syncthreads();
      }
    }
    __syncthreads();

    if (MODE == kSymbolic) {
      for (int r = threadIdx.x; r < nr; r += kBlock) p.cnt_out[r0 + r] = sh.cnt[r];
      __syncthreads();
      continue;
    }

    // ---- phase D: output offsets of the one-pass kernel
    if (MODE == kOnePass) {
      int64_t c0 = 0, c1 = 0;
      if (2 * threadIdx.x < nr) c0 = sh.cnt[2 * threadIdx.x];
      if (2 * threadIdx.x + 1 < nr) c1 = sh.cnt[2 * threadIdx.x + 1];
      int64_t agg;
      int64_t lex = block_exclusive_sum(c0 + c1, sh.wtot, &agg);
      if (threadIdx.x < kWave) {
        int64_t pre = lookback_exclusive(p.status, t, agg, p.counters + kCtrError, kErrLookback);
        if (threadIdx.x == 0) {
          sh.tile_excl = pre;
          sh.tile_total = pre + agg;
        }
      }
      __syncthreads();
      const int64_t base = sh.tile_excl;
      if (2 * threadIdx.x < nr) {
        sh.out[2 * threadIdx.x] = base + lex;
        p.c_rp[r0 + 2 * threadIdx.x] = base + lex;
      }
      if (2 * threadIdx.x + 1 < nr) {
        sh.out[2 * threadIdx.x + 1] = base + lex + c0;
        p.c_rp[r0 + 2 * threadIdx.x + 1] = base + lex + c0;
      }
      if (t == ntiles - 1 && threadIdx.x == 0) {
        p.c_rp[op.rows] = sh.tile_total;
        p.counters[kCtrNnz] = sh.tile_total;
        if (sh.tile_total > p.c_capacity)
          atomicOr((unsigned long long *)&p.counters[kCtrError], (unsigned long long)kErrCapacity);
      }
      __syncthreads();
    }

    // ---- phase E: staged merge rows, copied contiguously by 16-lane groups
    for (int i = threadIdx.x / CG; i < sh.nlist[0]; i += kBlock / CG) {
      const int r = sh.list[0][i];
      if (sh.flag[r]) continue;
      const int64_t o = sh.out[r];
      const int64_t n = sh.cnt[r];
      const int64_t lim = max((int64_t)0, min(n, p.c_capacity - o));
      if (MODE == kNumeric && lim < n && (threadIdx.x % CG) == 0)
        atomicOr((unsigned long long *)&p.counters[kCtrError], (unsigned long long)kErrCapacity);
      const int32_t so = sh.off[r];
      for (int64_t q = threadIdx.x % CG; q < lim; q += CG) {
        p.c_col[o + q] = pkeys[so + q];
        p.c_val[o + q] = pvals[so + q];
      }
    }
    if (MODE == kOnePass) {
      // merge rows whose staging was too small: merge again, straight into C
      for (int i = threadIdx.x; i < sh.nlist[0]; i += kBlock) {
        const int r = sh.list[0][i];
        if (!sh.flag[r]) continue;
        const int64_t o = sh.out[r];
        const int64_t lim = max((int64_t)0, min((int64_t)sh.cnt[r], p.c_capacity - o));
        if (lim > 0) merge_row<M, true>(op, r0 + r, p.c_col + o, p.c_val + o, lim);
      }
    }

    if constexpr (HASH) {
      // ---- phase E: hashed rows
      for (int i = gid; i < sh.nlist[1]; i += NG) {
        const int r = sh.list[1][i];
        if (sh.flag[r]) continue;
        const int64_t row = r0 + r;
        const uint32_t inf = p.info[row];
        const bool dense = info_dense(inf);
        const int32_t slots = (int32_t)info_slots(inf);
        const int32_t alloc = dense ? slots : slots + p.pad;
        const int64_t o = sh.out[r];
        const int64_t lim = max((int64_t)0, min((int64_t)sh.cnt[r], p.c_capacity - o));
        if (MODE == kNumeric && lim < sh.cnt[r] && lane_id() % G == 0)
          atomicOr((unsigned long long *)&p.counters[kCtrError], (unsigned long long)kErrCapacity);
        hash_extract<G, true>(pkeys + sh.off[r], pvals + sh.off[r], alloc, p.c_col + o, p.c_val + o, lim);
      }

      // ---- workgroup-level rows of the one-pass kernel: values and write-out
      if (MODE == kOnePass) {
        __syncthreads();
        for (int i = 0; i < sh.nlist[2]; ++i) {
          const int r = sh.list[2][i];
          const int64_t row = r0 + r;
          const int64_t c = (int64_t)p.ub[row];
          const int64_t span = (int64_t)p.hi[row] - (int64_t)p.lo[row] + 1;
          bool dense;
          int64_t slots;
          const int64_t alloc = global_table_alloc(span, c, &dense, &slots);
          if (alloc > p.scratch_slots) continue;
          const RowHash hs = make_hash(p.lo[row], p.hi[row], slots, dense);
          wg_global_keys(op, row, gkeys, alloc, hs, sh.ws, gvals, p.counters + kCtrError);
          wg_global_values(op, row, gkeys, gvals, alloc, hs, sh.ws, p.fast != 0);
          const int64_t o = sh.out[r];
          const int64_t lim = max((int64_t)0, min((int64_t)sh.cnt[r], p.c_capacity - o));
          wg_global_extract(gkeys, gvals, alloc, sh.ws.dmax, sh.ws, p.c_col + o, p.c_val + o, lim);
        }
      }
    }
    __syncthreads();
  }
}

// ===================================================== register-merge rows
// Matrices whose every row is a register-merge row need no tiles and no
// workgroup barriers: one thread per row, 64 consecutive rows per wave.
//   symbolic: merge without values, write the count;
//   numeric:  merge with values into the wave's LDS staging at the row's
//             offset inside the wave's output, then copy the wave's
//             contiguous output to C with all 64 lanes (coalesced stores;
//             one store per lane per row would scatter over 64 cache lines);
//   one pass: merge without values, scan the counts across the wave and
//             publish the wave's total (the wave is the look-back tile);
//             merge with values into the staging while predecessors
//             publish; then resolve the wave's offset and copy out.
// One-pass tickets are taken per workgroup; its waves are tiles 4t .. 4t+3.
constexpr int kWaveStage = 1024;   // staged entries per wave (12 KB)

__device__ __forceinline__ void status_publish(uint64_t *status, int64_t tile, int64_t agg) {
  if (lane_id() == 0) status_store(status + tile, (tile == 0 ? kFlagPre : kFlagAgg) | (uint64_t)agg);
}

// Exclusive prefix of a tile whose aggregate is already published: walk
// back 64 predecessors at a time to the nearest inclusive prefix, then
// publish this tile's inclusive prefix.  All 64 lanes of one wave.
__device__ inline int64_t lookback_resolve(uint64_t *status, int64_t tile, int64_t aggregate, int64_t *err,
                                           int64_t err_bit) {
  const int l = lane_id();
  if (tile == 0) return 0;
  int64_t excl = 0, j = tile - 1, polls = 0;
  while (true) {
    const int64_t idx = j - l;
    const uint64_t s = idx >= 0 ? status_load(status + idx) : (kFlagPre | 0ull);
    const uint64_t flag = s & ~kValMask;
    const uint64_t have_pre = ballot(flag == kFlagPre);
    const uint64_t invalid = ballot(flag == 0);
    const uint64_t upto = have_pre ? ((have_pre & (~have_pre + 1)) << 1) - 1ull : ~0ull;
    if (invalid & upto) {
      if (++polls > kSpinLimit) {
        if (l == 0 && err) atomicOr((unsigned long long *)err, (unsigned long long)err_bit);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
      continue;
    }
    excl += wave_sum((upto >> l) & 1ull ? (int64_t)(s & kValMask) : 0);
    if (have_pre) break;
    j -= kWave;
  }
  if (l == 0) status_store(status + tile, kFlagPre | (uint64_t)(excl + aggregate));
  return excl;
}

template <int M, int MODE>
__global__ void __launch_bounds__(kBlock) k_wave_merge(Operands op, int64_t *counters, uint64_t *status,
                                                       int32_t *cnt_out, int64_t *c_rp, int32_t *c_col,
                                                       double *c_val, int64_t c_capacity) {
  __shared__ int32_t sc[kWavesPerBlock][kWaveStage];
  __shared__ double sv[kWavesPerBlock][kWaveStage];
  __shared__ int64_t s_ticket;
  const int l = lane_id();
  const int w = threadIdx.x / kWave;
  int64_t wt;
  if (MODE == kOnePass) {
    if (threadIdx.x == 0)
      s_ticket = (int64_t)__hip_atomic_fetch_add((unsigned long long *)&counters[kCtrTicket], 1ull,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    wt = s_ticket * kWavesPerBlock + w;
  } else {
    wt = (int64_t)blockIdx.x * kWavesPerBlock + w;
  }
  const int64_t row0 = wt * kWave;
  if (row0 >= op.rows) return;   // whole wave: its tile is past the end
  const int64_t row = row0 + l;
  const bool valid = row < op.rows;
  if (MODE == kSymbolic) {
    if (valid) cnt_out[row] = (int32_t)merge_row<M, false>(op, row, nullptr, nullptr, 0);
    return;
  }
  int64_t base, o, n, tot;
  if (MODE == kNumeric) {
    base = c_rp[row0];
    const int64_t end = c_rp[min(row0 + kWave, op.rows)];
    tot = end - base;
    o = valid ? c_rp[row] - base : 0;
    n = valid ? c_rp[row + 1] - c_rp[row] : 0;
  } else {
    n = valid ? merge_row<M, false>(op, row, nullptr, nullptr, 0) : 0;
    const int64_t inc = wave_inclusive_sum(n);
    tot = __shfl(inc, kWave - 1, kWave);
    o = inc - n;
    status_publish(status, wt, tot);
  }
  const bool staged = tot <= kWaveStage;
  if (staged && valid) {
    const int64_t got = merge_row<M, true>(op, row, &sc[w][o], &sv[w][o], n);
    if (MODE == kNumeric && got != n)
      atomicOr((unsigned long long *)&counters[kCtrError], (unsigned long long)kErrInconsistent);
  }
  if (MODE == kOnePass) {
    base = lookback_resolve(status, wt, tot, counters + kCtrError, kErrLookback);
    if (valid) {
      c_rp[row] = base + o;
      if (row == op.rows - 1) {
        c_rp[op.rows] = base + tot;
        counters[kCtrNnz] = base + tot;
      }
    }
  }
  const int64_t lim = max((int64_t)0, min(tot, c_capacity - base));
  if (lim < tot && l == 0) atomicOr((unsigned long long *)&counters[kCtrError], (unsigned long long)kErrCapacity);
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  if (staged) {
    for (int64_t q = l; q < lim; q += kWave) {
      c_col[base + q] = sc[w][q];
      c_val[base + q] = sv[w][q];
    }
  } else if (valid) {
    // the wave's output does not fit the staging: rows write their own entries
    const int64_t rl = max((int64_t)0, min(n, lim - o));
    const int64_t got = merge_row<M, true>(op, row, c_col + base + o, c_val + base + o, rl);
    if (MODE == kNumeric && got != n)
      atomicOr((unsigned long long *)&counters[kCtrError], (unsigned long long)kErrInconsistent);
  }
}

hipError_t launch_wave_merge(const Operands &op, int mode, int merge_lists, int64_t *counters, uint64_t *status,
                             int32_t *cnt_out, int64_t *c_rp, int32_t *c_col, double *c_val, int64_t c_capacity,
                             hipStream_t s) {
  if (op.rows <= 0) return hipSuccess;
  const int64_t blocks = (op.rows + kBlock - 1) / kBlock;
#define SPG_WM(MM, MD)                                                                                        \
  hipLaunchKernelGGL((k_wave_merge<MM, MD>), dim3((unsigned)blocks), dim3(kBlock), 0, s, op, counters, status, \
                     cnt_out, c_rp, c_col, c_val, c_capacity)
  if (merge_lists == 4) {
    if (mode == kSymbolic) SPG_WM(4, kSymbolic);
    else if (mode == kNumeric) SPG_WM(4, kNumeric);
    else SPG_WM(4, kOnePass);
  } else if (merge_lists == 8) {
    if (mode == kSymbolic) SPG_WM(8, kSymbolic);
    else if (mode == kNumeric) SPG_WM(8, kNumeric);
    else SPG_WM(8, kOnePass);
  } else {
    return hipErrorInvalidValue;
  }
#undef SPG_WM
  return hipGetLastError();
}

template <int G, int M, bool HASH>
static hipError_t launch_tiles_ghm(const TileParams &tp, int mode, int grid, size_t lds, hipStream_t s) {
  switch (mode) {
    case kSymbolic:
      hipLaunchKernelGGL((k_tile<G, M, kSymbolic, HASH>), dim3(grid), dim3(kBlock), lds, s, tp);
      break;
    case kNumeric:
      hipLaunchKernelGGL((k_tile<G, M, kNumeric, HASH>), dim3(grid), dim3(kBlock), lds, s, tp);
      break;
    default:
      hipLaunchKernelGGL((k_tile<G, M, kOnePass, HASH>), dim3(grid), dim3(kBlock), lds, s, tp);
      break;
  }
  return hipGetLastError();
}

template <int M>
static hipError_t launch_tiles_m(const TileParams &tp, int mode, int group, bool hash, int grid, size_t lds,
                                 hipStream_t s) {
  if (!hash) return launch_tiles_ghm<8, M, false>(tp, mode, grid, lds, s);
  switch (group) {
    case 4: return launch_tiles_ghm<4, M, true>(tp, mode, grid, lds, s);
    case 8: return launch_tiles_ghm<8, M, true>(tp, mode, grid, lds, s);
    case 16: return launch_tiles_ghm<16, M, true>(tp, mode, grid, lds, s);
    case 32: return launch_tiles_ghm<32, M, true>(tp, mode, grid, lds, s);
    case 64: return launch_tiles_ghm<64, M, true>(tp, mode, grid, lds, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_tiles(const TileParams &tp, int mode, int group, int merge_lists, bool hash, int grid,
                        size_t lds_bytes, hipStream_t s) {
  switch (merge_lists) {
    case 4: return launch_tiles_m<4>(tp, mode, group, hash, grid, lds_bytes, s);
    case 8: return launch_tiles_m<8>(tp, mode, group, hash, grid, lds_bytes, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace spg
