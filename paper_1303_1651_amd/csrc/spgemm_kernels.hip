// HIP kernels of the SpGEMM pipeline for gfx950 (CDNA4, wave64).
//
// C = A * B on CSR FP64 operands, row by row as in the paper's row-major
// (Gustavson) algorithm, Section IV-A: row r of C accumulates a(r,c) * b(c,x)
// over the stored entries of row r of A (in stored order) and of row c of B.
// Output rows are sorted by column (Section IV-B append contract).
//
// Pipeline: features -> sizing/tiering -> scan of tile costs -> tile bounds
// -> tile kernel (symbolic, numeric, or one pass with decoupled look-back).
#include "device_common.h"
#include "spgemm_kernels.h"

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
__global__ void __launch_bounds__(kBlock) k_features(Operands op, Features f, int64_t *counters) {
  __shared__ int64_t s_sum[kWavesPerBlock];
  int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  int64_t ub = 0;
  if (i < op.rows) {
    int64_t s = op.a_rp[i], e = op.a_rp[i + 1];
    int32_t mx = 0, lo = 0x7fffffff, hi = -1;
    for (int64_t q = s; q < e; ++q) {
      int32_t k = op.a_col[q];
      int64_t bs = op.b_rp[k], be = op.b_rp[k + 1];
      int32_t len = (int32_t)(be - bs);
      ub += len;
      mx = max(mx, len);
      if (len > 0) {
        lo = min(lo, op.b_col[bs]);
        hi = max(hi, op.b_col[be - 1]);
      }
    }
    f.nnz_a[i] = (int32_t)(e - s);
    f.ub[i] = (int32_t)min(ub, (int64_t)op.b_cols);
    f.maxb[i] = mx;
    f.lo[i] = lo;
    f.hi[i] = hi;
  }
  int64_t w = wave_sum(ub);
  if (lane_id() == 0) s_sum[threadIdx.x / kWave] = w;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int j = 0; j < kWavesPerBlock; ++j) t += s_sum[j];
    if (t) atomicAdd((unsigned long long *)&counters[kCtrMults], (unsigned long long)t);
  }
}

hipError_t launch_features(const Operands &op, const Features &f, int64_t *counters, hipStream_t s) {
  if (op.rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_features, dim3((unsigned)((op.rows + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     s, op, f, counters);
  return hipGetLastError();
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
  __shared__ int64_t s_red[6][kWavesPerBlock];
  int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  // Tile budget HT (cost units): half the LDS pool when there is one, so a
  // tile's hashed rows always fit the pool; every row costs at least
  // ceil(HT / tile_rows), so a tile holds at most tile_rows rows.
  const int64_t H = sp.pool_slots / 2;
  const int64_t HT = tile_budget(sp.pool_slots, sp.tile_rows);
  const int64_t mincost = H > 0 ? (H + sp.tile_rows - 1) / sp.tile_rows : 1;
  int64_t n_tier[4] = {0, 0, 0, 0};
  int64_t capsum = 0, scratch = 0;
  if (i < op.rows) {
    int32_t m = pa.f.nnz_a[i];
    int64_t ub = pa.f.ub[i];
    int64_t mx = pa.f.maxb[i];
    int64_t c;
    if (sp.mode == kNumeric) {
      c = sp.cnt[i];
    } else if (sp.mode == kOnePass && sp.sizer == 2) {
      float p = sp.pred[i];
      double want = ceil((double)p * (1.0 + (double)sp.margin)) + (double)sp.slack;
      c = (int64_t)min((double)ub, max((double)mx, want));
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
    } else if (m <= sp.merge_lists && c <= sp.merge_max) {
      tier = kTierMerge;
      info = pack_info(kTierMerge, false, 0);
      cost = mincost;
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
    n_tier[tier] = 1;
    capsum = c;
  }
  int w = threadIdx.x / kWave;
  int64_t v[6] = {n_tier[1], n_tier[2], n_tier[3], n_tier[0], capsum, scratch};
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    int64_t t = wave_sum(v[j]);
    if (lane_id() == 0) s_red[j][w] = t;
  }
  {
    int64_t t = v[5];
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) t = max(t, __shfl_xor(t, d, kWave));
    if (lane_id() == 0) s_red[5][w] = t;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    int j = threadIdx.x;
    int64_t t = 0;
    for (int q = 0; q < kWavesPerBlock; ++q) t = (j == 5) ? max(t, s_red[j][q]) : t + s_red[j][q];
    const int dst[6] = {kCtrMerge, kCtrHash, kCtrGlobal, kCtrEmpty, kCtrCapSum, kCtrScratch};
    if (j == 5) {
      if (t) atomicMax((unsigned long long *)&pa.counters[dst[j]], (unsigned long long)t);
    } else if (t) {
      atomicAdd((unsigned long long *)&pa.counters[dst[j]], (unsigned long long)t);
    }
  }
}

hipError_t launch_size_rows(const Operands &op, const PlanArrays &pa, const SizeParams &sp,
                            hipStream_t s) {
  if (op.rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_size_rows, dim3((unsigned)((op.rows + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     s, op, pa, sp);
  return hipGetLastError();
}

// ------------------------------------------------------------------- scan
// Single-pass exclusive scan with decoupled look-back: each workgroup takes
// a ticket, scans 2048 items, publishes its aggregate and looks back for
// its prefix.  out[n] receives the total.  Safe in place (in == out).
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

template <typename TIn>
__global__ void __launch_bounds__(kBlock) k_scan(const TIn *in, int64_t *out, int64_t n,
                                                  uint64_t *status, int64_t *ticket,
                                                  int64_t *total_dst, int64_t *err) {
  __shared__ int64_t s_tile, s_excl;
  __shared__ int64_t s_wtot[kWavesPerBlock + 1];
  if (threadIdx.x == 0) s_tile = atomicAdd((unsigned long long *)ticket, 1ull);
  __syncthreads();
  const int64_t t = s_tile;
  const int64_t base = t * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int64_t v[kScanItems];
  int64_t sum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int64_t idx = base + k;
    v[k] = idx < n ? (int64_t)in[idx] : 0;
    sum += v[k];
  }
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
    int64_t idx = base + k;
    if (idx < n) {
      out[idx] = run;
      run += v[k];
      if (idx == n - 1) {
        out[n] = run;
        if (total_dst) *total_dst = run;
      }
    }
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
    for (int i = 0; i < ne; ++i) {
      const int64_t bsi = __shfl(bs, i, G);
      const int32_t bli = __shfl(bl, i, G);
      const double avi = VALUES ? __shfl(av, i, G) : 0.0;
      for (int32_t f = gl; f < bli; f += G) {
        const int32_t j = op.b_col[bsi + f];
        const double b = VALUES ? op.b_val[bsi + f] : 0.0;
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
            if (VALUES) vals[s] = first_add_rn(avi, b);
            break;
          }
          if (old == j) {
            if (VALUES) vals[s] = mul_add_rn(vals[s], avi, b);
            break;
          }
          ++s;
        }
        dmax = max(dmax, s - h);
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
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

// Rank of the key in slot s among all keys of the table: occupied slots
// before s, corrected for keys that probing pushed past larger ones (they
// sit at most dmax slots after their home).
template <bool GLOBAL = false>
__device__ __forceinline__ int64_t rank_fix(const int32_t *keys, int64_t alloc, int64_t s,
                                            int32_t key, int32_t dmax, const RowHash &hs) {
  auto ld = [&](int64_t q) { return GLOBAL ? gload(keys + q) : keys[q]; };
  int64_t fix = 0;
  int64_t end = min(s + (int64_t)dmax, alloc - 1);
  for (int64_t q = s + 1; q <= end; ++q) {
    int32_t y = ld(q);
    fix += (y != kEmpty && y < key) ? 1 : 0;
  }
  for (int64_t q = hs.home(key); q < s; ++q) fix -= (ld(q) > key) ? 1 : 0;
  return fix;
}

// Write the sorted row held by an LDS table (G lanes).
template <int G, bool VALUES>
__device__ void hash_extract(const int32_t *keys, const double *vals, int32_t alloc, const RowHash &hs,
                             int32_t dmax, int32_t *out_col, double *out_val, int64_t lim) {
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
      int64_t rank = run + __popcll(bal & lt);
      if (dmax > 0) rank += rank_fix(keys, alloc, s, key, dmax, hs);
      if (rank >= 0 && rank < lim) {
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

// Sorted write-out of a device table by the whole workgroup.
__device__ void wg_global_extract(const int32_t *keys, const double *vals, int64_t alloc,
                                  const RowHash &hs, int32_t dmax, WgScratch &ws, int32_t *out_col,
                                  double *out_val, int64_t lim) {
  int64_t run = 0;
  for (int64_t c = 0; c < alloc; c += kBlock) {
    int64_t s = c + threadIdx.x;
    int32_t key = s < alloc ? gload(keys + s) : kEmpty;
    int64_t occ = key != kEmpty ? 1 : 0;
    int64_t tot;
    int64_t ex = block_exclusive_sum(occ, ws.wtot, &tot);
    if (occ) {
      int64_t rank = run + ex;
      if (dmax > 0) rank += rank_fix<true>(keys, alloc, s, key, dmax, hs);
      if (rank >= 0 && rank < lim) {
        out_col[rank] = key;
        if (out_val) out_val[rank] = gloadd(vals + s);
      }
    }
    run += tot;
  }
  __syncthreads();
}

template <int MODE>
struct TileShared {
  int32_t off[kMaxTileRows];      // LDS pool offset of a hashed row
  int32_t cnt[kMaxTileRows];
  int32_t dmax[kMaxTileRows];
  int32_t flag[kMaxTileRows];     // 1: hashed row ran out of LDS probe room
  int64_t out[kMaxTileRows];      // where the row starts in C
  int16_t list[3][kMaxTileRows];  // merge, hash, workgroup-level rows
  int32_t nlist[3];
  int64_t tile, tile_excl, tile_total;
  int64_t wtot[kWavesPerBlock + 1];
  WgScratch ws;
};

size_t tile_static_lds(int mode) { return sizeof(TileShared<0>); }

template <int G, int M, int MODE>
__global__ void __launch_bounds__(kBlock) k_tile(TileParams p) {
  constexpr bool VALUES = (MODE != kSymbolic);
  extern __shared__ __align__(16) unsigned char pool_raw[];
  __shared__ TileShared<MODE> sh;
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
    if (threadIdx.x == 0) {
      sh.tile = (int64_t)atomicAdd((unsigned long long *)&p.counters[kCtrTicket], 1ull);
      sh.nlist[0] = sh.nlist[1] = sh.nlist[2] = 0;
    }
    __syncthreads();
    const int64_t t = sh.tile;
    if (t >= ntiles) break;
    const int64_t r0 = p.tile_row[t], r1 = p.tile_row[t + 1];
    const int nr = (int)(r1 - r0);

    // ---- classify rows, LDS offsets of hashed rows
    int64_t use2 = 0, use_a = 0;
    for (int k = 0; k < 2; ++k) {
      int r = 2 * threadIdx.x + k;
      int64_t use = 0;
      if (r < nr) {
        uint32_t inf = p.info[r0 + r];
        uint32_t tier = info_tier(inf);
        sh.cnt[r] = 0;
        sh.dmax[r] = 0;
        sh.flag[r] = 0;
        if (tier != kTierEmpty) {
          int slot = atomicAdd(&sh.nlist[tier - 1], 1);
          sh.list[tier - 1][slot] = (int16_t)r;
        }
        if (tier == kTierHash) use = info_dense(inf) ? info_slots(inf) : info_slots(inf) + p.pad;
      }
      if (k == 0) use_a = use;
      use2 += use;
    }
    int64_t used;
    int64_t ex = block_exclusive_sum(use2, sh.wtot, &used);
    if (2 * threadIdx.x < nr) sh.off[2 * threadIdx.x] = (int32_t)ex;
    if (2 * threadIdx.x + 1 < nr) sh.off[2 * threadIdx.x + 1] = (int32_t)(ex + use_a);
    for (int64_t s = threadIdx.x; s < used; s += kBlock) pkeys[s] = kEmpty;
    if (MODE == kNumeric) {
      for (int r = threadIdx.x; r < nr; r += kBlock) sh.out[r] = p.c_rp[r0 + r];
    }
    __syncthreads();

    // ---- phase A: register-merge rows, one thread each
    for (int i = threadIdx.x; i < sh.nlist[0]; i += kBlock) {
      const int r = sh.list[0][i];
      const int64_t row = r0 + r;
      if (MODE == kNumeric) {
        const int64_t o = sh.out[r];
        const int64_t want = p.c_rp[row + 1] - o;
        const int64_t lim = max((int64_t)0, min(want, p.c_capacity - o));
        int64_t n = merge_row<M, true>(op, row, p.c_col + o, p.c_val + o, lim);
        sh.cnt[r] = (int32_t)n;
        if (n != want) atomicOr((unsigned long long *)&p.counters[kCtrError], (unsigned long long)kErrInconsistent);
        if (lim < want) atomicOr((unsigned long long *)&p.counters[kCtrError], (unsigned long long)kErrCapacity);
      } else {
        sh.cnt[r] = (int32_t)merge_row<M, false>(op, row, nullptr, nullptr, 0);
      }
    }

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

    // rows whose LDS probes ran out join the workgroup-level list
    for (int i = threadIdx.x; i < sh.nlist[1]; i += kBlock) {
      const int r = sh.list[1][i];
      if (sh.flag[r]) {
        int slot = atomicAdd(&sh.nlist[2], 1);
        sh.list[2][slot] = (int16_t)r;
        atomicAdd((unsigned long long *)&p.counters[kCtrOverflow], 1ull);
      }
    }
    __syncthreads();

    // ---- phase C: workgroup-level rows (count; numeric pass writes them)
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
        wg_global_extract(gkeys, gvals, alloc, hs, sh.ws.dmax, sh.ws, p.c_col + o, p.c_val + o, lim);
      }
      __syncthreads();
    }
    __syncthreads();

    if (MODE == kSymbolic) {
      for (int r = threadIdx.x; r < nr; r += kBlock) p.cnt_out[r0 + r] = sh.cnt[r];
      __syncthreads();
      continue;
    }

    // ---- phase D: output offsets
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

      // merge rows: second pass with values, straight into C
      for (int i = threadIdx.x; i < sh.nlist[0]; i += kBlock) {
        const int r = sh.list[0][i];
        const int64_t o = sh.out[r];
        const int64_t lim = max((int64_t)0, min((int64_t)sh.cnt[r], p.c_capacity - o));
        if (lim > 0) merge_row<M, true>(op, r0 + r, p.c_col + o, p.c_val + o, lim);
      }
    }

    // ---- phase E: hashed rows
    for (int i = gid; i < sh.nlist[1]; i += NG) {
      const int r = sh.list[1][i];
      if (sh.flag[r]) continue;
      const int64_t row = r0 + r;
      const uint32_t inf = p.info[row];
      const bool dense = info_dense(inf);
      const int32_t slots = (int32_t)info_slots(inf);
      const int32_t alloc = dense ? slots : slots + p.pad;
      const RowHash hs = make_hash(p.lo[row], p.hi[row], slots, dense);
      const int64_t o = sh.out[r];
      const int64_t lim = max((int64_t)0, min((int64_t)sh.cnt[r], p.c_capacity - o));
      if (MODE == kNumeric && lim < sh.cnt[r] && lane_id() % G == 0)
        atomicOr((unsigned long long *)&p.counters[kCtrError], (unsigned long long)kErrCapacity);
      hash_extract<G, true>(pkeys + sh.off[r], pvals + sh.off[r], alloc, hs, sh.dmax[r], p.c_col + o,
                            p.c_val + o, lim);
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
        wg_global_extract(gkeys, gvals, alloc, hs, sh.ws.dmax, sh.ws, p.c_col + o, p.c_val + o, lim);
      }
    }
    __syncthreads();
  }
}

template <int G, int M>
static hipError_t launch_tiles_gm(const TileParams &tp, int mode, int grid, size_t lds, hipStream_t s) {
  switch (mode) {
    case kSymbolic:
      hipLaunchKernelGGL((k_tile<G, M, kSymbolic>), dim3(grid), dim3(kBlock), lds, s, tp);
      break;
    case kNumeric:
      hipLaunchKernelGGL((k_tile<G, M, kNumeric>), dim3(grid), dim3(kBlock), lds, s, tp);
      break;
    default:
      hipLaunchKernelGGL((k_tile<G, M, kOnePass>), dim3(grid), dim3(kBlock), lds, s, tp);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_tiles(const TileParams &tp, int mode, int group, int merge_lists, int grid,
                        size_t lds_bytes, hipStream_t s) {
  if (merge_lists != 8) return hipErrorInvalidValue;
  switch (group) {
    case 4: return launch_tiles_gm<4, 8>(tp, mode, grid, lds_bytes, s);
    case 8: return launch_tiles_gm<8, 8>(tp, mode, grid, lds_bytes, s);
    case 16: return launch_tiles_gm<16, 8>(tp, mode, grid, lds_bytes, s);
    case 32: return launch_tiles_gm<32, 8>(tp, mode, grid, lds_bytes, s);
    case 64: return launch_tiles_gm<64, 8>(tp, mode, grid, lds_bytes, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace spg
