// Kernel parameter blocks and launch entry points of the SpGEMM pipeline.
// Host code (spgemm_host.hip) fills these; the kernels live in
// spgemm_kernels.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"

namespace spg {

// Per-row tier.  EMPTY rows produce nothing; MERGE rows are merged in
// registers by one lane; HASH rows accumulate in the LDS table of a wave,
// the whole wave on one row; GLOBAL rows (too large for a wave's table)
// accumulate in a per-workgroup table in device memory.
enum Tier : uint32_t { kTierEmpty = 0, kTierMerge = 1, kTierHash = 2, kTierGlobal = 3 };

// info word of a row: bits 0-1 tier, bit 2 dense window, bits 3-31 table slots.
// esc: a hashed-tier row of the numeric pass whose products are sorted as
// they are (expand, sort, combine) instead of entering a hash table.
__host__ __device__ inline uint32_t pack_info(uint32_t tier, bool dense, uint32_t slots, bool esc = false) {
  return tier | (dense ? 4u : 0u) | (esc ? 8u : 0u) | (slots << 4);
}
__host__ __device__ inline uint32_t info_tier(uint32_t w) { return w & 3u; }
__host__ __device__ inline bool info_dense(uint32_t w) { return (w >> 2) & 1u; }
__host__ __device__ inline bool info_esc(uint32_t w) { return (w >> 3) & 1u; }
__host__ __device__ inline uint32_t info_slots(uint32_t w) { return w >> 4; }

// Pass kinds of the tile kernel.
// kComputeOnly: the numeric accumulation without storing C (row-per-thread
// merge kernels only).
enum Mode : int { kSymbolic = 0, kNumeric = 1, kOnePass = 2, kComputeOnly = 3 };

// counters[] layout (int64, device)
enum Counter : int {
  kCtrTicket = 0,      // tile ticket of the running tile kernel
  kCtrTiles = 1,       // number of tiles
  kCtrMults = 2,       // sum of per-row multiplication counts (exact, int64)
  kCtrCapSum = 3,      // sum of per-row capacities (learned capacity hint)
  kCtrMerge = 4, kCtrHash = 5,
  kCtrGlobal = 6,      // workgroup-tier rows (length of the list in PlanArrays::big)
  kCtrEmpty = 7,
  kCtrOverflow = 8,    // one-pass rows whose capacity was too small (length of PlanArrays::ovf)
  kCtrScratch = 9,     // largest device table (slots) a workgroup-level row needs
  kCtrError = 10,      // bit flags, see kErr*
  kCtrNnz = 11,        // nnz(C) after a one-pass numeric
  kCtrScanTicket = 12,
  kCtrStaged = 13,     // rows a numeric or one-pass tile stages in LDS
  kCtrSpillRows = 14,  // one pass: rows placed in the spill arena
  kCtrMaxA = 15,       // longest row of A
  kCtrUnpacked = 16,   // summed bounds of rows whose feature triple does not pack
  kCtrTable = 17,      // largest wave table (slots) a hashed row uses
  kCtrScratchRows = 18,  // rows that may need a workgroup-tier device table
  kCtrPadTotal = 19,   // one pass: entries of the padded buffer (sum of capacities)
  kCtrSpill = 20,      // one pass: entries claimed in the spill arena
  kCtrWaveSpan = 21,   // largest output of 64 consecutive rows (merge staging)
  kCtrHuge = 22,       // workgroup-tier rows of kHugeWork products or more (listed first)
  kCtrBigTail = 23,    // the other workgroup-tier rows (listed from the end of the list)
  kCtrBigTicket = 24,  // next list entry a k_big workgroup takes
  kCtrEsc = 25,        // numeric or one-pass sizing: hashed rows taken by expand-sort-combine
  kCtrWaveCap = 26,    // largest sum of capacities over 64 consecutive rows (merge one pass)
  kNumCounters = 32
};
enum : int64_t {
  kErrCapacity = 1, kErrNotCanonical = 2, kErrInconsistent = 4, kErrScratch = 8, kErrLookback = 16,
  kErrDescriptor = 32   // a descriptor's nnz differs from its row_ptr[rows]
};

struct Operands {
  const int64_t *a_rp;
  const int32_t *a_col;
  const double *a_val;
  const int64_t *b_rp;
  const int32_t *b_col;
  const double *b_val;
  int64_t rows;       // rows of A (and C)
  int32_t b_cols;     // columns of B (and C)
  int64_t b_rows;     // rows of B
  int64_t a_nnz, b_nnz;  // the descriptors' entry counts (checked by the plan)
};

struct Features {
  int32_t *nnz_a;     // entries of the A row
  int32_t *ub;        // multiplication count, saturated at b_cols
  int32_t *maxb;      // longest selected B row
  int32_t *lo, *hi;   // smallest / largest column any selected B row touches
  int32_t *brow;  // per row of B, 16-byte aligned: {entries, first column,
                  // last column, 0} (empty: {0, INT32_MAX, -1, 0}), written
                  // before the span pass
};

struct SizeParams {
  int mode;             // Mode of the pass being sized
  int sizer;            // spgemm_sizer for kOnePass
  int table_max;        // largest wave table (slots); 0: no wave hash tier
  int value_table_max;  // kSymbolic: the numeric pass's largest table (scratch sizing)
  int stage;            // LDS staging entries of a wave tile
  int stage_row_max;    // kNumeric: hashed rows up to this size are staged
  int merge_lists;      // template M of the merge tier
  int merge_max;        // largest capacity the merge tier takes
  int merge_apart;      // kNumeric: merge rows run in a launch of their own (not staged by tiles)
  float dense_ratio;
  float margin;
  int slack;
  const float *pred;    // learned prediction (kOnePass + learned)
  const int32_t *cnt;   // exact counts (kNumeric)
};

struct PlanArrays {
  Features f;
  uint32_t *info;       // per row
  int32_t *cap;         // per row capacity (keys)
  int64_t *cost;        // per row tile cost, scanned in place to an exclusive prefix (rows + 1)
  int32_t *tile_row;    // first row of every tile (tiles + 1)
  uint64_t *status;     // look-back status, one per tile
  uint64_t *scan_status;
  int64_t *counters;
  int32_t *cnt;         // exact per-row counts (symbolic output)
  float *pred;          // learned prediction
  int64_t *partials;    // per-workgroup partial sums (up to 10 per workgroup)
  int32_t *big;         // workgroup-tier rows (any order)
  int32_t *ovf;         // one pass: rows that outgrew their capacity (any order)
  int64_t *pad_rp;      // one pass: exclusive scan of the capacities (rows + 1)
  int64_t *pad_src;     // one pass: where a row sits in the padded buffer
  int64_t *parts;       // workgroup tier: part words of the split rows
                        // (-1: computed straight into C)
};

constexpr int64_t kMinTable = 64;   // smallest hashed wave table (slots)
constexpr int64_t kHugeWork = 8192;  // workgroup-tier rows of this many products start first
constexpr int kSplitParts = 16;       // column ranges of a split huge row
constexpr int64_t kSplitWork = 32768;  // huge rows of this many products are split
constexpr int64_t kMaxSplitRows = 2048;  // huge rows split per launch, at most

struct WaveTileParams {
  Operands op;
  const uint32_t *info;
  const int32_t *cap;       // per row: exact count (kNumeric), capacity (kOnePass)
  const int32_t *maxb;
  const int32_t *lo;
  const int32_t *tile_row;  // tile bounds (ntiles + 1); null: tiles of 64 rows
  int64_t ntiles;
  int64_t *counters;
  int32_t *cnt_out;         // kSymbolic, kOnePass: per-row counts
  int32_t *ovf_list;        // kOnePass: rows with no room (exact path)
  int64_t *pad_src;         // kOnePass: per-row place in the padded buffer
  int64_t spill_base;       // kOnePass: first entry of the spill arena
  int64_t spill_cap;        //           and its entries
  const int64_t *c_rp;      // kNumeric: exact offsets; kOnePass: padded offsets
  int32_t *c_col;           // C (kNumeric) or the padded buffer (kOnePass)
  double *c_val;
  int64_t c_capacity;
  int table_slots;          // LDS table of a wave (slots)
  int stage_slots;          // LDS staging of a wave (entries)
  int stage_row_max;        // hashed rows of at most this capacity are staged
};

struct CompactParams {
  int64_t rows;
  const uint32_t *info;
  const int64_t *pad_src;
  const int32_t *pad_col;
  const double *pad_val;
  const int64_t *c_rp;
  int32_t *c_col;
  double *c_val;
  int64_t c_capacity;
};

struct BigParams {
  Operands op;
  const int32_t *list;      // rows to compute, counters[count_ctr] of them
  int count_ctr;
  int huge_ctr;             // >= 0: the list holds counters[huge_ctr] rows at its
  int64_t list_len;         //   front and the rest from its end (list_len entries)
  const int32_t *ub;
  const int32_t *maxb;
  int32_t *cnt;             // kSymbolic: output; kNumeric: exact counts
  const int32_t *lo, *hi;
  int64_t *counters;
  const int64_t *c_rp;
  int32_t *c_col;
  double *c_val;
  int64_t c_capacity;
  char *scratch;            // per-workgroup device tables
  int64_t scratch_slots;    // slots per workgroup
  int fast;                 // reordered accumulation allowed
  float dense_ratio;        // dense window when the column region <= ratio * count
  int split;                // the first kMaxSplitRows rows of the huge front of
                            // the list take kSplitParts tickets each; those of
                            // kSplitWork products or more are computed as
                            // kSplitParts column ranges
  int64_t *parts;           // per split row: kSplitParts words (done flag |
                            // part size) and a finished-parts counter; cleared
                            // by the launcher
  int32_t bitmap_words;     // > 0: every listed row's columns fit a window of
                            // 32 * bitmap_words columns, and the rows take the
                            // LDS bitmap kernel (k_bitmap) instead of k_big
  int32_t grid_bitmap;      // workgroups of that kernel
};

// Workgroup-tier rows by a bitmap of the row's column window in LDS: B's
// column count at most kBitmapMaxCols (128 KB of bits, plus the rank groups
// and the step set: within one compute unit's 160 KB).
constexpr int32_t kBitmapMaxCols = 1 << 20;
constexpr int kBitmapGroup = 8;   // words per rank group
size_t bitmap_lds_bytes(int32_t words, int mode);
hipError_t bitmap_kernels_prepare();
// Register-merge rows of a tiled counting or numeric pass (those whose tier
// in `tiers` is the merge), by the row-per-thread kernel with merge_lists
// (4 or 8) lists; numeric staging of `stage` entries per wave.
hipError_t launch_wave_merge_tiered(const Operands &op, int mode, int merge_lists, int stage, const uint32_t *tiers,
                                    int64_t *counters, int32_t *cnt_out, const int64_t *c_rp, int32_t *c_col,
                                    double *c_val, int64_t c_capacity, hipStream_t s);

// Per row i of A: entries of the row (m), multiplication count (ub: the
// paper's estimate of Section IV-B taken per row), the longest selected B
// row (mx) and, with SPAN, the smallest/largest column any selected B row
// touches (lo, hi; from the per-row records of B in brow).
// The stored entries are taken eight at a time, each group's loads issued
// at once (three dependent gather rounds).
template <bool SPAN>
__device__ __forceinline__ void row_features(const Operands &op, int64_t i, int64_t &m, int64_t &ub, int32_t &mx,
                                             int32_t &lo, int32_t &hi, const int32_t *brow = nullptr) {
  const int64_t s = op.a_rp[i], e = op.a_rp[i + 1];
  m = e - s;
  ub = 0;
  mx = 0;
  lo = 0x7fffffff;
  hi = -1;
  // eight entries at a time: their gathers are in flight together
  for (int64_t q0 = s; q0 < e; q0 += 8) {
    const int cnt = (int)min((int64_t)8, e - q0);
    int32_t k[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) k[q] = q < cnt ? op.a_col[q0 + q] : 0;
    if (SPAN) {
      // one aligned 16-byte record per selected B row: length and span
      int4 r[8];
#pragma unroll
      for (int q = 0; q < 8; ++q)
        r[q] = q < cnt ? reinterpret_cast<const int4 *>(brow)[k[q]] : make_int4(0, 0x7fffffff, -1, 0);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        ub += r[q].x;
        mx = max(mx, r[q].x);
        lo = min(lo, r[q].y);
        hi = max(hi, r[q].z);
      }
    } else {
      int64_t bs[8], be[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        bs[q] = q < cnt ? op.b_rp[k[q]] : 0;
        be[q] = q < cnt ? op.b_rp[k[q] + 1] : 0;
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int32_t len = (int32_t)(be[q] - bs[q]);
        ub += len;
        mx = max(mx, len);
      }
    }
  }
}

// The same features for the rows held by the lanes of a wave (row i where
// `live`; every lane of the wave calls it).  A row of at most kFeatLong
// entries is walked by its own lane; longer rows (power-law rows reach
// thousands of entries) are walked by the whole wave, one after another,
// each lane taking every 64th entry, so that no lane walks a long row while
// the other 63 wait.  Integer sums, minima and maxima: the result does not
// depend on who walks the row.
constexpr int64_t kFeatLong = 32;
template <bool SPAN>
__device__ __forceinline__ void wave_row_features(const Operands &op, int64_t i, bool live, int64_t &m, int64_t &ub,
                                                  int32_t &mx, int32_t &lo, int32_t &hi,
                                                  const int32_t *brow = nullptr) {
  m = 0;
  ub = 0;
  mx = 0;
  lo = 0x7fffffff;
  hi = -1;
  int64_t s = 0, e = 0;
  if (live) {
    s = op.a_rp[i];
    e = op.a_rp[i + 1];
  }
  const bool longrow = live && e - s > kFeatLong;
  if (live && !longrow) row_features<SPAN>(op, i, m, ub, mx, lo, hi, brow);
  uint64_t pend = ballot(longrow);
  const int lane = lane_id();
  while (pend) {
    const int r = __ffsll((unsigned long long)pend) - 1;
    pend &= pend - 1;
    const int64_t rs = __shfl(s, r, kWave), re = __shfl(e, r, kWave);
    int64_t u = 0;
    int32_t x = 0, l = 0x7fffffff, h = -1;
    // four entries per lane at a time: their gathers are in flight together
    for (int64_t q0 = rs + lane; q0 < re; q0 += 4 * kWave) {
      int32_t k[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) k[q] = q0 + q * kWave < re ? op.a_col[q0 + q * kWave] : -1;
      if (SPAN) {
        int4 rr[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
          rr[q] = k[q] >= 0 ? reinterpret_cast<const int4 *>(brow)[k[q]] : make_int4(0, 0x7fffffff, -1, 0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          u += rr[q].x;
          x = max(x, rr[q].x);
          l = min(l, rr[q].y);
          h = max(h, rr[q].z);
        }
      } else {
        int64_t bs[4], be[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          bs[q] = k[q] >= 0 ? op.b_rp[k[q]] : 0;
          be[q] = k[q] >= 0 ? op.b_rp[k[q] + 1] : 0;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int32_t len = (int32_t)(be[q] - bs[q]);
          u += len;
          x = max(x, len);
        }
      }
    }
    u = wave_sum(u);
    x = wave_max32(x);
    if (SPAN) {
      l = wave_min32(l);
      h = wave_max32(h);
    }
    if (lane == r) {
      m = re - rs;
      ub = u;
      mx = x;
      lo = l;
      hi = h;
    }
  }
}

// ---- launchers (spgemm_kernels.hip) ----
hipError_t launch_fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_u64(uint64_t *p, uint64_t v, int64_t n, hipStream_t s);
hipError_t launch_validate(const int64_t *rp, const int32_t *col, int64_t rows, int64_t cols,
                           int64_t nnz, int64_t *counters, hipStream_t s);
// Sums into counters: kCtrMults, kCtrMaxA, kCtrEmpty, kCtrWaveCap (the
// largest multiplication count summed over 64 consecutive rows).  mode 2
// also writes the per-row plan arrays in f.
hipError_t launch_features(const Operands &op, const Features &f, int64_t *counters, int64_t *partials, int mode,
                           hipStream_t s, const int64_t *gate = nullptr, int64_t gate_max = 0);
// Longest row of A into counters[kCtrMaxA]; raises kErrDescriptor when a
// descriptor's nnz differs from its row_ptr[rows].
hipError_t launch_row_max(const Operands &op, int64_t *counters, int64_t *partials, hipStream_t s);
// Zeroes counters[i] for every bit i of mask.
hipError_t launch_clear_counters(int64_t *counters, uint32_t mask, hipStream_t s);
hipError_t launch_size_rows(const Operands &op, const PlanArrays &pa, const SizeParams &sp,
                            hipStream_t s);
// exclusive scan of rows int32 (or int64 when in64) values into out[0..n], out[n] = total
// group_max (may be null): receives the largest sum of 64 consecutive items
// starting at a multiple of 64.
hipError_t launch_scan_i32(const int32_t *in, int64_t *out, int64_t n, uint64_t *status,
                           int64_t *ticket, int64_t *total_dst, int64_t *err, hipStream_t s,
                           int64_t *group_max = nullptr);
hipError_t launch_scan_i64_inplace(int64_t *inout, int64_t n, uint64_t *status, int64_t *ticket,
                                   int64_t *err, hipStream_t s);
hipError_t launch_tile_bounds(const int64_t *cost, int64_t rows, int64_t half_pool,
                              int32_t *tile_row, int64_t *counters, hipStream_t s);
size_t wave_tile_lds(int mode, int table_slots, int stage_slots);
// has_merge: some row of the pass takes the merge tier
hipError_t launch_brow_ends(const Operands &op, Features f, hipStream_t s);
hipError_t launch_wave_tiles(const WaveTileParams &wp, int mode, int merge_lists, bool has_merge, bool esc_only,
                             bool esc_big, hipStream_t s);
hipError_t launch_compact(const CompactParams &cp, hipStream_t s);
hipError_t launch_big_rows(const BigParams &bp, int mode, int grid, hipStream_t s);
hipError_t launch_sum_partials(const int64_t *partials, int64_t nblocks, int n, int stride, const int32_t *dst,
                               const int32_t *is_max, int64_t *counters, hipStream_t s);
// Row-per-thread merge kernels for matrices whose rows all take the merge
// tier (merge_lists 4, 6, 8, 10 or 16).  kSymbolic: counts into cnt_out,
// multiplication count and empty rows into counters (through partials).
// kNumeric: C from the exact row_ptr c_rp, `stage` entries of LDS staging
// per wave.  kComputeOnly: every row accumulated, nothing of C stored; the
// row's entry count into cnt_out and its largest |value| into c_val (one
// per row).
hipError_t launch_wave_merge(const Operands &op, int mode, int merge_lists, int stage, int64_t *counters,
                             int32_t *cnt_out, int64_t *partials, const int64_t *c_rp, int32_t *c_col,
                             double *c_val, int64_t c_capacity, hipStream_t s);

}  // namespace spg
