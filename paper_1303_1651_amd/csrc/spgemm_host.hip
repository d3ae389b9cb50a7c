// Host side of the C ABI declared in include/spgemm.h: descriptor checks,
// workspace layout, tuning defaults, and the order of kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/spgemm.h"
#include "spgemm_kernels.h"
#include "spgemm_internal.h"

using namespace spg;

// --------------------------------------------------------------- helpers
namespace spg {

int device_cus() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cached[dev] = n;
  }
  return cached[dev];
}

// Small pinned host buffer for reading device counters (one per thread).
int64_t *host_counters() {
  static thread_local int64_t *buf = nullptr;
  if (!buf) {
    void *p = nullptr;
    if (hipHostMalloc(&p, sizeof(int64_t) * kNumCounters * 2, hipHostMallocDefault) != hipSuccess) return nullptr;
    buf = static_cast<int64_t *>(p);
  }
  return buf;
}

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Workspace carve-up: every array 256-byte aligned.
struct Layout {
  size_t counters, model, partials, nnz_a, ub, maxb, lo, hi, pred, cnt, info, cap, cost, tile_row, status, scan_status, big, ovf, pad_rp, pad_src, brow, parts, total;
};

Layout layout_for(int64_t rows, int64_t brows) {
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + std::max<size_t>(bytes, 1), 256);
    return at;
  };
  const size_t R = (size_t)std::max<int64_t>(rows, 0);
  const size_t tiles_max = 2 * R + 2;
  const size_t scan_tiles = R / 2048 + 2;
  L.counters = take(sizeof(int64_t) * kNumCounters);
  L.model = take(sizeof(float) * kMlpDevFloats);
  L.partials = take(sizeof(int64_t) * 10 * (R / 256 + 2));
  L.nnz_a = take(4 * R);
  L.ub = take(4 * R);
  L.maxb = take(4 * R);
  L.lo = take(4 * R);
  L.hi = take(4 * R);
  L.pred = take(4 * R);
  L.cnt = take(4 * R);
  L.info = take(4 * R);
  L.cap = take(4 * R);
  L.cost = take(8 * (R + 1));
  L.tile_row = take(4 * (tiles_max + 1));
  L.status = take(8 * tiles_max);
  L.scan_status = take(8 * scan_tiles);
  L.big = take(4 * R);
  L.ovf = take(4 * R);
  L.pad_rp = take(8 * (R + 1));
  L.pad_src = take(8 * R);
  const size_t BR = (size_t)std::max<int64_t>(brows, 0);
  L.brow = take(16 * BR);
  L.parts = take(8 * (size_t)kMaxSplitRows * (kSplitParts + 1));
  L.total = o;
  return L;
}

spgemm_tuning default_tuning(const spgemm_csr *A, const spgemm_csr *B) {
  (void)A;
  (void)B;
  spgemm_tuning t{};
  t.table_slots = 1024;
  t.stage_slots = 1024;
  t.merge_max_nnz = 64;
  t.merge_lists = 8;
  t.dense_ratio = 2.0f;
  t.margin = 0.05f;
  t.slack = 2;
  t.blocks_per_cu = 4;
  t.spill_ratio = 0.25f;
  t.split_merge = 1;
  // the LDS bitmap path is opt-in: its first GPU run (a batched one pass
  // with the learned sizer) ended in a memory violation whose cause has not
  // been found; device tables stay the default
  t.bitmap_cols = 0;
  return t;
}

static void merge_tuning(spgemm_tuning *t, const spgemm_tuning *u) {
  if (!u) return;
  if (u->table_slots) t->table_slots = u->table_slots < 0 ? 0 : u->table_slots;
  if (u->stage_slots) t->stage_slots = u->stage_slots;
  if (u->merge_max_nnz) t->merge_max_nnz = u->merge_max_nnz < 0 ? 0 : u->merge_max_nnz;
  if (u->merge_lists) t->merge_lists = u->merge_lists;
  if (u->dense_ratio > 0) t->dense_ratio = u->dense_ratio;
  if (u->margin > 0) t->margin = u->margin;
  if (u->slack) t->slack = u->slack;
  if (u->blocks_per_cu) t->blocks_per_cu = u->blocks_per_cu;
  if (u->spill_ratio) t->spill_ratio = u->spill_ratio < 0 ? 0.0f : u->spill_ratio;
  if (u->bitmap_cols) t->bitmap_cols = u->bitmap_cols < 0 ? 0 : u->bitmap_cols;
  if (u->split_merge) t->split_merge = u->split_merge < 0 ? 0 : 1;
}

static bool tuning_ok(const spgemm_tuning &t) {
  const int ts = t.table_slots;
  const bool t_ok = ts == 0 || ts == 256 || ts == 512 || ts == 1024 || ts == 2048 || ts == 4096;
  return t_ok && t.stage_slots >= 256 && t.stage_slots <= 8192 &&
         12 * ((int64_t)t.table_slots + t.stage_slots) <= 147456 && (t.merge_lists == 4 || t.merge_lists == 8) &&
         t.merge_max_nnz >= 0 && t.dense_ratio >= 0 && t.margin >= 0 && t.slack >= 0 && t.blocks_per_cu >= 1 &&
         t.blocks_per_cu <= 16 && t.spill_ratio >= 0 && t.spill_ratio <= 4 && t.bitmap_cols >= 0 &&
         t.bitmap_cols <= kBitmapMaxCols;
}

spgemm_status check_csr(const spgemm_csr *M, bool need_val) {
  if (!M) return SPGEMM_E_NULL;
  if (M->rows < 0 || M->cols < 0 || M->nnz < 0) return SPGEMM_E_DIM;
  if (M->cols >= ((int64_t)1 << 31) || M->rows >= ((int64_t)1 << 31)) return SPGEMM_E_INDEX_OVERFLOW;
  if (!M->row_ptr) return SPGEMM_E_NULL;
  if (M->nnz > 0 && !M->col_idx) return SPGEMM_E_NULL;
  if (need_val && M->nnz > 0 && !M->val) return SPGEMM_E_NULL;
  return SPGEMM_OK;
}

}  // namespace spg

// ------------------------------------------------------------------ plan
struct spgemm_plan {
  spgemm_csr A, B;
  spgemm_options opts;
  spgemm_tuning tune;
  char *ws;
  size_t ws_bytes;
  Layout L;
  PlanArrays pa;
  int stage;           // 0 planned, 1 symbolic done (EXACT), 2 numeric done
  int first_mode;      // kSymbolic (EXACT) or kOnePass
  int cur_mode;        // mode the current tiles were sized for
  int64_t ntiles;
  int64_t nbig;            // workgroup-tier rows of the current sizing
  int64_t esc_rows;        // expand-sort rows (counting: sort-count rows) of the current sizing
  int64_t scratch_slots;   // per workgroup, current sizing
  int64_t scratch_slots_plan;
  int64_t scratch_rows;    // rows that may need a workgroup-tier table (plan sizing)
  int32_t bitmap_words;    // > 0: workgroup-tier rows use the LDS bitmap of B's columns
  int64_t esc_big;         // numeric: expand-sort rows of more than kEscMaxSmall products
  int64_t pad_total;       // one pass: entries of the padded buffer (sum of capacities)
  int64_t spill_cap;       // one pass, learned: entries of the spill arena after it
  int table_launch;        // LDS table slots of the wave-tile launch
  int stage_launch;        // LDS staging entries of the wave-tile launch
  int64_t staged_rows;     // rows the last sized pass stages
  int merge_only;      // every row takes the register-merge tier: row-per-thread kernels
  int merge_m;         // lists of the row-per-thread merge (4, 6, 8, 10 or 16)
  int merge_stage;     // staged entries per merge wave
  int merge_off;       // numeric or one pass sized without the register-merge tier
  int stage_off;       // numeric or one pass sized without staging hashed rows
  spgemm_info info;
  hipError_t last_err;
  const spgemm_model *model;
  hipEvent_t ev0, ev1;   // SPGEMM_OPT_TIMING
  int timing_pending;
  int device;            // device current when the plan was created
};

#define HIPCK(plan, expr)                                  \
  do {                                                     \
    hipError_t _e = (expr);                                \
    if (_e != hipSuccess) {                                \
      if (plan) (plan)->last_err = _e;                     \
      return SPGEMM_E_HIP;                                 \
    }                                                      \
  } while (0)

static Operands operands_of(const spgemm_plan *p, const double *a_val, const double *b_val) {
  Operands op;
  op.a_rp = p->A.row_ptr;
  op.a_col = p->A.col_idx;
  op.a_val = a_val ? a_val : p->A.val;
  op.b_rp = p->B.row_ptr;
  op.b_col = p->B.col_idx;
  op.b_val = b_val ? b_val : p->B.val;
  op.rows = p->A.rows;
  op.b_cols = (int32_t)p->B.cols;
  op.b_rows = p->B.rows;
  op.a_nnz = p->A.nnz;
  op.b_nnz = p->B.nnz;
  return op;
}

static int64_t *ctr(spgemm_plan *p) { return p->pa.counters; }

// A look-back wait gave up (see lookback_exclusive): report a runtime error.
static spgemm_status lookback_failed(spgemm_plan *p) {
  p->last_err = hipErrorLaunchTimeOut;
  return SPGEMM_E_HIP;
}

// Device-side consistency failures (a key that found no slot, a numeric
// count that differs from the symbolic one, a look-back that gave up).
static spgemm_status device_errors(spgemm_plan *p, const int64_t *h) {
  if (h[kCtrError] & kErrScratch) return SPGEMM_E_WORKSPACE;
  if (h[kCtrError] & kErrLookback) return lookback_failed(p);
  if (h[kCtrError] & kErrInconsistent) return SPGEMM_E_STATE;
  return SPGEMM_OK;
}

// Read the device counters into the pinned host buffer, or into `into`
// (kNumCounters entries) when given (synchronises).
static spgemm_status read_counters(spgemm_plan *p, hipStream_t s, int64_t **out, int64_t *into = nullptr) {
  int64_t *h = into ? into : host_counters();
  if (!h) return SPGEMM_E_HIP;
  HIPCK(p, hipMemcpyAsync(h, ctr(p), sizeof(int64_t) * kNumCounters, hipMemcpyDeviceToHost, s));
  HIPCK(p, hipStreamSynchronize(s));
  if (p->timing_pending) {
    float ms = 0.f;
    HIPCK(p, hipEventElapsedTime(&ms, p->ev0, p->ev1));
    p->info.tile_ms = ms;
    p->info.tile_ms_total += ms;
    p->timing_pending = 0;
  }
  *out = h;
  return SPGEMM_OK;
}

// The row-per-thread merge path takes matrices whose A rows have at most this
// many entries; its per-wave staging holds at most kMergeStageMax entries
// (waves with more output write their rows directly).
constexpr int kMergeOnlyLists = 16;
constexpr double kMergeOnlyRowEst = 128.0;
constexpr int64_t kMergeStageMax = 2048;

// LDS staging (entries) of a merge wave for the largest output (numeric) or
// capacity sum (one pass, at most kMergeOnePassStage for rows of up to 8
// lists: capacities overstate the output) of a wave's 64 rows: rounded up to 8 entries so that
// workgroups pack the LDS closely; waves whose output exceeds it write their
// rows directly.
constexpr int64_t kMergeOnePassStage = 1024;
static int merge_stage_for(int64_t wave_max) {
  const int64_t st = std::max<int64_t>((wave_max + 7) & ~(int64_t)7, 64);
  return (int)std::min<int64_t>(st, kMergeStageMax);
}

// Hashed rows of at most this many entries (a wave's width) are staged in
// LDS by the numeric pass (copied out with the tile's other rows); larger
// rows are written to C by their own wave directly, with full-wave stores.
constexpr int kStageRowMax = 64;
constexpr int64_t kMergeFewRows = 64;   // merge rows under 1/64 of the rows: numeric / one pass without them
constexpr int64_t kSpillMin = 4096;   // smallest spill arena (entries)

// Sizing of one pass (tiers, capacities, tile costs) plus tile bounds.
// Hashed rows of at most this capacity are staged in LDS.  A learned
// capacity carries the sizing margin: the limit scales with it, so that a
// row predicted at kStageRowMax entries is staged like an exact one.
static int stage_row_max(const spgemm_plan *p, int mode) {
  if (p->stage_off) return 0;
  if (mode == kOnePass && p->opts.sizer == SPGEMM_SIZER_LEARNED)
    return (int)std::ceil(kStageRowMax * (1.0 + (double)p->tune.margin)) + p->tune.slack;
  return kStageRowMax;
}

static spgemm_status size_pass(spgemm_plan *p, int mode, hipStream_t s) {
  const int tvals = p->tune.table_slots;                   // values table (numeric, one pass)
  const int tkeys = std::min(4 * tvals, 16384);            // keys-only table (symbolic): same bytes
  const int stage = p->tune.stage_slots;
  SizeParams sp{};
  sp.mode = mode;
  sp.sizer = p->opts.sizer;
  sp.table_max = mode == kSymbolic ? tkeys : tvals;
  sp.value_table_max = tvals;
  sp.stage = stage;
  sp.stage_row_max = stage_row_max(p, mode);
  sp.merge_lists = p->tune.merge_lists;
  sp.merge_max = p->merge_off ? 0 : std::min(p->tune.merge_max_nnz, stage / 2);
  sp.merge_apart = (mode == kNumeric && p->tune.split_merge > 0) ? 1 : 0;
  sp.dense_ratio = p->tune.dense_ratio;
  sp.margin = p->tune.margin;
  sp.slack = p->tune.slack;
  sp.pred = p->pa.pred;
  sp.cnt = p->pa.cnt;
  Operands op = operands_of(p, nullptr, nullptr);
  HIPCK(p, launch_size_rows(op, p->pa, sp, s));
  const int64_t R = p->A.rows;
  if (mode != kSymbolic) {
    HIPCK(p, launch_scan_i64_inplace(p->pa.cost, R, p->pa.scan_status, ctr(p) + kCtrScanTicket,
                                     ctr(p) + kCtrError, s));
    HIPCK(p, launch_tile_bounds(p->pa.cost, R, stage / 2, p->pa.tile_row, ctr(p), s));
  }
  int64_t *h;
  spgemm_status st = read_counters(p, s, &h);
  if (st != SPGEMM_OK) return st;
  if (h[kCtrError] & kErrLookback) return lookback_failed(p);
  p->ntiles = mode == kSymbolic ? (R + 63) / 64 : h[kCtrTiles];
  p->nbig = h[kCtrGlobal];
  // expand-sort rows: their count, and above bit 32 those of more than
  // kEscMaxSmall products (the numeric launch then sorts 16 keys per lane)
  p->esc_rows = h[kCtrEsc] & 0xffffffffll;   // counting: the sort-count rows
  p->esc_big = mode == kNumeric ? (h[kCtrEsc] >> 32) : 0;
  // the bitmap kernel needs no device tables
  p->scratch_slots = p->bitmap_words > 0 ? 0 : (h[kCtrScratch] + 1) & ~(int64_t)1;
  p->scratch_rows = h[kCtrScratchRows];
  p->table_launch = (int)h[kCtrTable];
  // staging: every row of a one-pass tile; merge rows only in the numeric pass
  p->stage_launch = (mode != kSymbolic && h[kCtrStaged] > 0) ? stage : 0;
  p->staged_rows = mode != kSymbolic ? h[kCtrStaged] : 0;
  p->cur_mode = mode;
  p->info.rows_merge = h[kCtrMerge];
  p->info.rows_hash = h[kCtrHash];
  p->info.rows_global = h[kCtrGlobal];
  p->info.rows_empty = h[kCtrEmpty];
  p->info.tiles = p->ntiles;
  if (mode != kNumeric) p->info.c_capacity_hint = h[kCtrCapSum];
  return SPGEMM_OK;
}

// Staging buys contiguous copy-outs for rows shorter than a wave, but the
// launch then reserves the whole stage in every wave's LDS (fewer resident
// waves).  Where only a few rows would be staged (a stencil's boundary
// rows, say), the pass is sized again without staging hashed rows: they are
// written straight to their place like the longer ones.
// Merge tier switched off for a re-sizing; staging too when the rows staged
// after it (at most those staged now plus the merge rows) will be few, so
// that one re-sizing does what unstage_if_few would otherwise size again.
static void merge_off_for_resize(spgemm_plan *p) {
  p->merge_off = 1;
  const int64_t staged_max = p->staged_rows + p->info.rows_merge;
  if (!p->stage_off && staged_max > 0 && staged_max * kMergeFewRows < p->A.rows) p->stage_off = 1;
}

static spgemm_status unstage_if_few(spgemm_plan *p, int mode, hipStream_t s) {
  if (p->stage_off || (p->info.rows_merge > 0 && !(mode == kNumeric && p->tune.split_merge > 0)) ||
      p->staged_rows == 0 || p->staged_rows * kMergeFewRows >= p->A.rows)
    return SPGEMM_OK;
  p->stage_off = 1;
  return size_pass(p, mode, s);
}

static void timing_begin(spgemm_plan *p, hipStream_t s, hipError_t *e) {
  if (p->ev0 && *e == hipSuccess) *e = hipEventRecord(p->ev0, s);
}
static void timing_end(spgemm_plan *p, hipStream_t s, hipError_t *e) {
  if (p->ev1 && *e == hipSuccess) {
    *e = hipEventRecord(p->ev1, s);
    if (*e == hipSuccess) p->timing_pending = 1;
  }
}

// Wave tiles of one pass (the caller has sized the pass).  kOnePass: c_rp,
// c_col, c_val are the padded offsets and buffer.
static spgemm_status run_wave(spgemm_plan *p, int mode, const double *a_val, const double *b_val,
                              const int64_t *c_rp, int32_t *c_col, double *c_val, int64_t c_capacity, hipStream_t s) {
  if (p->ntiles == 0) return SPGEMM_OK;
  WaveTileParams wp{};
  wp.op = operands_of(p, a_val, b_val);
  wp.info = p->pa.info;
  wp.cap = p->pa.cap;
  wp.maxb = p->pa.f.maxb;
  wp.lo = p->pa.f.lo;
  wp.tile_row = mode == kSymbolic ? nullptr : p->pa.tile_row;
  wp.ntiles = p->ntiles;
  wp.counters = ctr(p);
  wp.cnt_out = p->pa.cnt;
  wp.ovf_list = p->pa.ovf;
  wp.pad_src = p->pa.pad_src;
  wp.spill_base = p->pad_total;
  wp.spill_cap = mode == kOnePass ? p->spill_cap : 0;
  wp.c_rp = c_rp;
  wp.c_col = c_col;
  wp.c_val = c_val;
  wp.c_capacity = c_capacity;
  wp.table_slots = p->table_launch;
  wp.stage_slots = p->stage_launch;
  wp.stage_row_max = stage_row_max(p, mode);
  // a pass whose hashed rows are all expand-sort rows (and no merge rows)
  // runs the tile kernel without the table path (fewer registers)
  const bool esc_only = p->esc_rows > 0 && p->esc_rows == p->info.rows_hash;
  bool has_merge = p->info.rows_merge > 0;
  if (has_merge && mode != kOnePass && p->tune.split_merge > 0) {
    // two-pass passes: the merge rows by the row-per-thread kernel at its own
    // occupancy (first: a numeric wave that stages copies its whole range,
    // which the tile and workgroup kernels then write their rows over), the
    // hashed rows by tiles compiled without the merge lists
    HIPCK(p, launch_wave_merge_tiered(wp.op, mode, p->tune.merge_lists, p->tune.stage_slots, p->pa.info, ctr(p),
                                      p->pa.cnt, c_rp, c_col, c_val, c_capacity, s));
    if (p->info.rows_hash == 0) return SPGEMM_OK;
    has_merge = false;
  }
  HIPCK(p, launch_wave_tiles(wp, mode, p->tune.merge_lists, has_merge, esc_only && !has_merge,
                             mode == kNumeric && p->esc_big > 0, s));
  return SPGEMM_OK;
}

// Scratch of a plan: the padded buffer of the one pass (capacity sum x 12
// bytes) first, then one device table per workgroup of k_big.
// Entries of the padded buffer and the spill arena after it.
static int64_t pad_entries(const spgemm_plan *p) {
  return p->first_mode == kOnePass && !p->merge_only ? p->pad_total + p->spill_cap : 0;
}
static size_t pad_bytes(const spgemm_plan *p) {
  const size_t e = (size_t)pad_entries(p);
  return e ? align_up(align_up(e * 4, 256) + e * 8, 256) : 0;
}

// Rows computed one workgroup each with device tables in the caller's
// scratch: the workgroup-tier list (kCtrGlobal rows) or, one pass, the rows
// that outgrew their capacity (kCtrOverflow rows, count known on the device).
static spgemm_status run_big(spgemm_plan *p, int mode, bool overflow_list, void *scratch, size_t scratch_bytes,
                             const double *a_val, const double *b_val, const int64_t *c_rp, int32_t *c_col,
                             double *c_val, int64_t c_capacity, hipStream_t s) {
  const int64_t nrows = overflow_list ? (p->opts.sizer == SPGEMM_SIZER_LEARNED ? p->A.rows : 0) : p->nbig;
  if (nrows == 0) return SPGEMM_OK;
  const size_t off = pad_bytes(p);
  const size_t per = (size_t)p->scratch_slots * 12;
  if (per > 0 && (!scratch || scratch_bytes < off + per || !aligned256(scratch))) return SPGEMM_E_WORKSPACE;
  BigParams bp{};
  bp.op = operands_of(p, a_val, b_val);
  bp.list = overflow_list ? p->pa.ovf : p->pa.big;
  bp.count_ctr = overflow_list ? kCtrOverflow : kCtrGlobal;
  bp.huge_ctr = overflow_list ? -1 : kCtrHuge;
  bp.list_len = p->A.rows;
  bp.ub = p->pa.f.ub;
  bp.maxb = p->pa.f.maxb;
  bp.cnt = p->pa.cnt;
  bp.lo = p->pa.f.lo;
  bp.hi = p->pa.f.hi;
  bp.counters = ctr(p);
  bp.c_rp = c_rp;
  bp.c_col = c_col;
  bp.c_val = c_val;
  bp.c_capacity = c_capacity;
  bp.scratch = static_cast<char *>(scratch) + off;
  bp.scratch_slots = p->scratch_slots;
  bp.fast = (p->opts.flags & SPGEMM_OPT_FAST) ? 1 : 0;
  bp.dense_ratio = p->tune.dense_ratio;
  // the list's huge rows are split into column ranges (the rows listed for
  // the exact path after a one pass are not)
  bp.split = overflow_list ? 0 : 1;
  bp.parts = p->pa.parts;
  bp.bitmap_words = p->bitmap_words;
  if (p->bitmap_words > 0) {
    // as many workgroups as the compute units hold with this window (the
    // static LDS of a workgroup is under 8 KB)
    const size_t lds = bitmap_lds_bytes(p->bitmap_words, mode == kSymbolic ? kSymbolic : kNumeric) + 8192;
    const int64_t per_cu = std::max<int64_t>(1, std::min<int64_t>(8, (int64_t)(163840 / lds)));
    bp.grid_bitmap = (int32_t)std::min<int64_t>((int64_t)device_cus() * per_cu, nrows);
  }
  int64_t g = (int64_t)device_cus() * p->tune.blocks_per_cu;
  g = std::min(g, nrows * (bp.split ? kSplitParts : 1));
  if (per > 0) g = std::min<int64_t>(g, (int64_t)((scratch_bytes - off) / per));
  HIPCK(p, launch_big_rows(bp, mode == kSymbolic ? kSymbolic : kNumeric, (int)g, s));
  return SPGEMM_OK;
}

static spgemm_status clear_run_counters(spgemm_plan *p, hipStream_t s) {
  const uint32_t mask = (1u << kCtrError) | (1u << kCtrOverflow) | (1u << kCtrTicket) | (1u << kCtrSpill) |
                        (1u << kCtrSpillRows);
  HIPCK(p, launch_clear_counters(ctr(p), mask, s));
  return SPGEMM_OK;
}

namespace spg {

// Kernel launches of the numeric pass (two-pass numeric or one pass), in
// stream order and without any synchronisation, so that a caller may
// capture them in a HIP graph.  The caller has checked the arguments.
spgemm_status numeric_enqueue(spgemm_plan *p, void *scratch, size_t scratch_bytes, const double *av,
                              const double *bv, int64_t *c_row_ptr, int32_t *c_col, double *c_val,
                              int64_t c_capacity, hipStream_t s) {
  spgemm_status st = clear_run_counters(p, s);
  if (st != SPGEMM_OK) return st;
  const int mode = p->first_mode == kSymbolic ? kNumeric : kOnePass;
  if (p->merge_only) {
    const Operands op = operands_of(p, av, bv);
    if (mode == kOnePass) {
      // counts, their scan into row_ptr and the numeric merge back to back
      // on the device; the merge is staged by the capacities' largest wave
      // sum, and a wave whose exact output exceeds it writes its rows directly
      HIPCK(p, launch_wave_merge(op, kSymbolic, p->merge_m, 0, ctr(p), p->pa.cnt, p->pa.partials, nullptr, nullptr,
                                 nullptr, 0, s));
      HIPCK(p, launch_scan_i32(p->pa.cnt, c_row_ptr, p->A.rows, p->pa.scan_status, ctr(p) + kCtrScanTicket,
                               ctr(p) + kCtrNnz, ctr(p) + kCtrError, s));
    }
    HIPCK(p, launch_wave_merge(op, kNumeric, p->merge_m, p->merge_stage, ctr(p), nullptr, nullptr, c_row_ptr, c_col,
                               c_val, c_capacity, s));
    return SPGEMM_OK;
  }
  if (mode == kNumeric) {
    st = run_wave(p, kNumeric, av, bv, c_row_ptr, c_col, c_val, c_capacity, s);
    if (st == SPGEMM_OK)
      st = run_big(p, kNumeric, false, scratch, scratch_bytes, av, bv, c_row_ptr, c_col, c_val, c_capacity, s);
    return st;
  }
  // one pass: workgroup-tier rows are counted first; the wave tiles write
  // every other row into their tile's padded range (the tile's share of the
  // scan of the capacities) or the spill arena and count it; the listed rows
  // (no room anywhere, or a learned-size table that filled) are counted
  // again; the counts are scanned into row_ptr, the rows moved to their
  // places, and the workgroup-tier and listed rows are computed into C with
  // their exact sizes
  const int64_t pe = pad_entries(p);
  if (pe > 0 && (!scratch || scratch_bytes < pad_bytes(p) || !aligned256(scratch))) return SPGEMM_E_WORKSPACE;
  int32_t *pcol = static_cast<int32_t *>(scratch);
  double *pval = reinterpret_cast<double *>(static_cast<char *>(scratch) + align_up((size_t)pe * 4, 256));
  st = run_big(p, kSymbolic, false, scratch, scratch_bytes, av, bv, nullptr, nullptr, nullptr, 0, s);
  if (st == SPGEMM_OK) st = run_wave(p, kOnePass, av, bv, p->pa.pad_rp, pcol, pval, pe, s);
  // rows whose learned-size table filled have no count yet: the listed rows
  // are counted again (learned sizer only; the list is empty otherwise)
  if (st == SPGEMM_OK)
    st = run_big(p, kSymbolic, true, scratch, scratch_bytes, av, bv, nullptr, nullptr, nullptr, 0, s);
  if (st != SPGEMM_OK) return st;
  HIPCK(p, launch_scan_i32(p->pa.cnt, c_row_ptr, p->A.rows, p->pa.scan_status, ctr(p) + kCtrScanTicket,
                           ctr(p) + kCtrNnz, ctr(p) + kCtrError, s));
  CompactParams cp{};
  cp.rows = p->A.rows;
  cp.info = p->pa.info;
  cp.pad_src = p->pa.pad_src;
  cp.pad_col = pcol;
  cp.pad_val = pval;
  cp.c_rp = c_row_ptr;
  cp.c_col = c_col;
  cp.c_val = c_val;
  cp.c_capacity = c_capacity;
  HIPCK(p, launch_compact(cp, s));
  st = run_big(p, kNumeric, false, scratch, scratch_bytes, av, bv, c_row_ptr, c_col, c_val, c_capacity, s);
  if (st == SPGEMM_OK)
    st = run_big(p, kNumeric, true, scratch, scratch_bytes, av, bv, c_row_ptr, c_col, c_val, c_capacity, s);
  return st;
}

int64_t *plan_counters(spgemm_plan *p) { return p->pa.counters; }
int plan_is_one_pass(const spgemm_plan *p) { return p->first_mode != kSymbolic; }
size_t plan_workspace_bytes(int64_t rows, int64_t brows) { return layout_for(rows, brows).total; }

spgemm_status plan_check_counters(spgemm_plan *p, const int64_t *h) { return device_errors(p, h); }

}  // namespace spg

extern "C" {

const char *spgemm_status_string(spgemm_status s) {
  switch (s) {
    case SPGEMM_OK: return "ok";
    case SPGEMM_E_NULL: return "null pointer";
    case SPGEMM_E_DIM: return "dimension mismatch";
    case SPGEMM_E_NOT_CANONICAL: return "input is not canonical CSR";
    case SPGEMM_E_INDEX_OVERFLOW: return "index does not fit in int32";
    case SPGEMM_E_WORKSPACE: return "workspace or scratch too small";
    case SPGEMM_E_CAPACITY: return "output capacity too small";
    case SPGEMM_E_NO_MODEL: return "learned sizing needs a model";
    case SPGEMM_E_STATE: return "call out of order";
    case SPGEMM_E_HIP: return "HIP runtime error";
    case SPGEMM_E_INVALID: return "invalid option";
    case SPGEMM_E_IO: return "model file error";
    default: break;
  }
  return "unknown status";
}

spgemm_status spgemm_plan_workspace_size(const spgemm_csr *A, const spgemm_csr *B,
                                         const spgemm_options *opts, size_t *bytes) {
  if (!bytes) return SPGEMM_E_NULL;
  spgemm_status st = check_csr(A, false);
  if (st != SPGEMM_OK) return st;
  st = check_csr(B, false);
  if (st != SPGEMM_OK) return st;
  if (A->cols != B->rows) return SPGEMM_E_DIM;
  (void)opts;
  *bytes = layout_for(A->rows, B->rows).total;
  return SPGEMM_OK;
}

spgemm_status spgemm_plan_create(const spgemm_csr *A, const spgemm_csr *B, const spgemm_options *opts,
                                 void *workspace, size_t workspace_bytes, void *stream,
                                 spgemm_plan **out, spgemm_info *info) {
  if (!out || !opts) return SPGEMM_E_NULL;
  *out = nullptr;
  spgemm_status st = check_csr(A, false);
  if (st != SPGEMM_OK) return st;
  st = check_csr(B, false);
  if (st != SPGEMM_OK) return st;
  if (A->cols != B->rows) return SPGEMM_E_DIM;
  if (opts->sizer < 0 || opts->sizer > 2) return SPGEMM_E_INVALID;
  if (opts->sizer == SPGEMM_SIZER_LEARNED && !opts->model) return SPGEMM_E_NO_MODEL;
  Layout L = layout_for(A->rows, B->rows);
  if (!workspace) return SPGEMM_E_NULL;
  if (workspace_bytes < L.total || !aligned256(workspace)) return SPGEMM_E_WORKSPACE;
  spgemm_tuning tune = default_tuning(A, B);
  merge_tuning(&tune, opts->tuning);
  if (!tuning_ok(tune)) return SPGEMM_E_INVALID;

  spgemm_plan *p = (spgemm_plan *)calloc(1, sizeof(spgemm_plan));
  if (!p) return SPGEMM_E_INVALID;
  p->A = *A;
  p->B = *B;
  p->opts = *opts;
  p->opts.tuning = nullptr;
  p->tune = tune;
  p->bitmap_words = (tune.bitmap_cols > 0 && B->cols > 0 && B->cols <= tune.bitmap_cols)
                        ? (int32_t)((B->cols + 31) / 32)
                        : 0;
  if (p->bitmap_words > 0 && bitmap_kernels_prepare() != hipSuccess) {
    free(p);
    return SPGEMM_E_HIP;
  }
  p->model = opts->model;
  p->ws = static_cast<char *>(workspace);
  p->ws_bytes = workspace_bytes;
  p->L = L;
  p->info.c_nnz = -1;
  if (hipGetDevice(&p->device) != hipSuccess) {
    free(p);
    return SPGEMM_E_HIP;
  }
  if (opts->flags & SPGEMM_OPT_TIMING) {
    if (hipEventCreate(&p->ev0) != hipSuccess || hipEventCreate(&p->ev1) != hipSuccess) {
      if (p->ev0) (void)hipEventDestroy(p->ev0);
      free(p);
      return SPGEMM_E_HIP;
    }
  }
  char *w = p->ws;
  p->pa.counters = (int64_t *)(w + L.counters);
  p->pa.f.nnz_a = (int32_t *)(w + L.nnz_a);
  p->pa.f.ub = (int32_t *)(w + L.ub);
  p->pa.f.maxb = (int32_t *)(w + L.maxb);
  p->pa.f.lo = (int32_t *)(w + L.lo);
  p->pa.f.hi = (int32_t *)(w + L.hi);
  p->pa.pred = (float *)(w + L.pred);
  p->pa.cnt = (int32_t *)(w + L.cnt);
  p->pa.info = (uint32_t *)(w + L.info);
  p->pa.cap = (int32_t *)(w + L.cap);
  p->pa.cost = (int64_t *)(w + L.cost);
  p->pa.tile_row = (int32_t *)(w + L.tile_row);
  p->pa.status = (uint64_t *)(w + L.status);
  p->pa.scan_status = (uint64_t *)(w + L.scan_status);
  p->pa.partials = (int64_t *)(w + L.partials);
  p->pa.big = (int32_t *)(w + L.big);
  p->pa.ovf = (int32_t *)(w + L.ovf);
  p->pa.pad_rp = (int64_t *)(w + L.pad_rp);
  p->pa.pad_src = (int64_t *)(w + L.pad_src);
  p->pa.parts = (int64_t *)(w + L.parts);
  p->pa.f.brow = (int32_t *)(w + L.brow);
  hipStream_t s = (hipStream_t)stream;

  auto fail = [&](spgemm_status e) {
    if (e != SPGEMM_OK) {
      spgemm_plan_destroy(p);
      *out = nullptr;
    }
    return e;
  };
  if (launch_fill_i64(p->pa.counters, 0, kNumCounters, s) != hipSuccess) return fail(SPGEMM_E_HIP);
  if (opts->flags & SPGEMM_OPT_VALIDATE) {
    if (launch_validate(A->row_ptr, A->col_idx, A->rows, A->cols, A->nnz, p->pa.counters, s) != hipSuccess ||
        launch_validate(B->row_ptr, B->col_idx, B->rows, B->cols, B->nnz, p->pa.counters, s) != hipSuccess)
      return fail(SPGEMM_E_HIP);
    int64_t *h;
    if (read_counters(p, s, &h) != SPGEMM_OK) return fail(SPGEMM_E_HIP);
    if (h[kCtrError] & kErrNotCanonical) return fail(SPGEMM_E_NOT_CANONICAL);
  }
  Operands op = operands_of(p, nullptr, nullptr);
  p->first_mode = opts->sizer == SPGEMM_SIZER_EXACT ? kSymbolic : kOnePass;
  const bool learned = opts->sizer == SPGEMM_SIZER_LEARNED;
  float *dev = (float *)(w + L.model);
  if (learned) {
    st = spgemm_model_upload(p->model, dev, stream);
    if (st != SPGEMM_OK) return fail(st);
  }
  // Longest row of A (row pointers only) decides the path.  Every row
  // merges in registers when no row of A has more stored entries than the
  // merge tier's lists (and the tier is not switched off); then no per-row
  // plan arrays are needed.  The merge pays per output entry for every
  // list: it takes rows with few entries of A and short outputs (estimated
  // from the mean row lengths of A and B).
  const double est_row = (A->rows > 0 ? (double)A->nnz / (double)A->rows : 0.0) *
                         (B->rows > 0 ? (double)B->nnz / (double)B->rows : 0.0);
  const int64_t merge_max_a = p->tune.merge_max_nnz <= 0 ? -1
                              : est_row <= kMergeOnlyRowEst
                                  ? kMergeOnlyLists
                                  : std::min<int64_t>(p->tune.merge_lists, kMergeOnlyLists);
  if (launch_row_max(op, p->pa.counters, p->pa.partials, s) != hipSuccess) return fail(SPGEMM_E_HIP);
  // The one-pass sizers' sums for the merge path (the multiplication count,
  // or the learned capacities) in the same round trip: their kernel reads
  // the longest row first and does the work only when the merge path is
  // taken (the tiled path's plan computes its own).
  if (p->first_mode != kSymbolic) {
    const int64_t *gate = p->pa.counters + kCtrMaxA;
    const hipError_t he = learned ? launch_mlp_capacity(dev, op, p->pa.counters, p->pa.partials, p->tune.margin,
                                                        p->tune.slack, s, gate, merge_max_a)
                                  : launch_features(op, p->pa.f, p->pa.counters, p->pa.partials, 0, s, gate,
                                                    merge_max_a);
    if (he != hipSuccess) return fail(SPGEMM_E_HIP);
  }
  int64_t *h;
  st = read_counters(p, s, &h);
  if (st != SPGEMM_OK) return fail(st);
  if (h[kCtrError] & kErrDescriptor) return fail(SPGEMM_E_DIM);
  p->merge_only = A->rows > 0 && h[kCtrMaxA] <= merge_max_a;
  // the fewest lists that hold every row of A (registers grow with them)
  {
    const int64_t ma = h[kCtrMaxA];
    p->merge_m = ma <= 4 ? 4 : ma <= 6 ? 6 : ma <= 8 ? 8 : ma <= 10 ? 10 : 16;
  }
  if (p->merge_only) {
    p->info.tiles = (A->rows + 63) / 64;
    p->ntiles = p->info.tiles;
    p->cur_mode = p->first_mode;
    if (p->first_mode == kSymbolic) {
      // the symbolic pass finds the multiplication counts and empty rows as
      // it counts, and the staging of the numeric pass from the exact counts
      p->info.multiplications = -1;
      p->info.c_capacity_hint = -1;
      p->scratch_slots_plan = 0;
      p->info.scratch_bytes = 0;
      if (info) *info = p->info;
      *out = p;
      return SPGEMM_OK;
    }
    // one pass: the capacities' sum (the size of C to allocate; the
    // multiplication count, or the learned sizes) and their largest sum
    // over a wave's 64 rows (the staging of the numeric merge), from the
    // gated pass above
    p->info.rows_empty = h[kCtrEmpty];
    p->info.rows_merge = A->rows - h[kCtrEmpty];
    p->info.c_capacity_hint = learned ? h[kCtrCapSum] + h[kCtrUnpacked] : h[kCtrMults];
    p->merge_stage =
        merge_stage_for(std::min<int64_t>(h[kCtrWaveCap], p->merge_m >= 10 ? kMergeStageMax : kMergeOnePassStage));
  } else {
    // per-row features (and their sums), the learned prediction, tiers
    if (launch_brow_ends(op, p->pa.f, s) != hipSuccess ||
        launch_features(op, p->pa.f, p->pa.counters, p->pa.partials, 2, s) != hipSuccess)
      return fail(SPGEMM_E_HIP);
    if (learned) {
      if (launch_mlp_predict(dev, p->pa.f.nnz_a, p->pa.f.ub, p->pa.f.maxb, A->rows, p->pa.pred, s, p->tune.margin,
                             p->tune.slack, nullptr) != hipSuccess)
        return fail(SPGEMM_E_HIP);
    }
    st = size_pass(p, p->first_mode, s);
    // a one pass with only a handful of merge rows is sized again without
    // the merge tier: the tile kernel that also merges holds more registers
    // (fewer resident waves) for every tile
    if (st == SPGEMM_OK && p->first_mode == kOnePass && p->info.rows_merge > 0 &&
        p->info.rows_merge * kMergeFewRows < A->rows) {
      merge_off_for_resize(p);
      st = size_pass(p, p->first_mode, s);
    }
    if (st == SPGEMM_OK && p->first_mode == kOnePass) st = unstage_if_few(p, p->first_mode, s);
    if (st != SPGEMM_OK) return fail(st);
    if (p->first_mode == kOnePass) {
      if (launch_scan_i32(p->pa.cap, p->pa.pad_rp, A->rows, p->pa.scan_status, p->pa.counters + kCtrScanTicket,
                          p->pa.counters + kCtrPadTotal, p->pa.counters + kCtrError, s) != hipSuccess)
        return fail(SPGEMM_E_HIP);
      st = read_counters(p, s, &h);
      if (st != SPGEMM_OK) return fail(st);
    } else {
      // the counters as the sizing pass read them (nothing has run since)
      h = host_counters();
    }
    p->pad_total = p->first_mode == kOnePass ? h[kCtrPadTotal] : 0;
    // learned capacities may fall short: rows their tile has no room for go
    // to an arena of spill_ratio times the padded buffer (at least kSpillMin)
    p->spill_cap = learned && !p->merge_only && p->tune.spill_ratio > 0
                       ? std::max<int64_t>((int64_t)((double)p->tune.spill_ratio * (double)p->pad_total), kSpillMin)
                       : 0;
  }
  if (h[kCtrError] & kErrDescriptor) return fail(SPGEMM_E_DIM);
  p->info.multiplications = h[kCtrMults];
  p->scratch_slots_plan = p->scratch_slots;
  // room for one table per resident workgroup of the workgroup-tier kernel
  // (no more workgroups than rows that may need one)
  int64_t groups = std::min<int64_t>((int64_t)device_cus() * p->tune.blocks_per_cu, std::max<int64_t>(p->scratch_rows, 1));
  p->info.scratch_bytes = pad_bytes(p) + (size_t)(p->scratch_slots * 12) * (size_t)groups;
  if (info) *info = p->info;
  *out = p;
  return SPGEMM_OK;
}

spgemm_status spgemm_symbolic(spgemm_plan *p, void *scratch, size_t scratch_bytes, int64_t *c_row_ptr,
                              int64_t *c_nnz, void *stream) {
  if (!p || !c_row_ptr || !c_nnz) return SPGEMM_E_NULL;
  if (p->first_mode != kSymbolic || p->stage != 0) return SPGEMM_E_STATE;
  hipStream_t s = (hipStream_t)stream;
  spgemm_status st = clear_run_counters(p, s);
  if (st != SPGEMM_OK) return st;
  hipError_t e = hipSuccess;
  timing_begin(p, s, &e);
  HIPCK(p, e);
  if (p->merge_only) {
    HIPCK(p, launch_wave_merge(operands_of(p, nullptr, nullptr), kSymbolic, p->merge_m, 0, ctr(p), p->pa.cnt,
                               p->pa.partials, nullptr, nullptr, nullptr, 0, s));
  } else {
    st = run_wave(p, kSymbolic, nullptr, nullptr, nullptr, nullptr, nullptr, 0, s);
    if (st == SPGEMM_OK)
      st = run_big(p, kSymbolic, false, scratch, scratch_bytes, nullptr, nullptr, nullptr, nullptr, nullptr, 0, s);
    if (st != SPGEMM_OK) return st;
  }
  timing_end(p, s, &e);
  HIPCK(p, e);
  // merge rows: the scan also finds the largest output of a wave's 64 rows
  // (the staging of the numeric merge waves)
  HIPCK(p, launch_scan_i32(p->pa.cnt, c_row_ptr, p->A.rows, p->pa.scan_status, ctr(p) + kCtrScanTicket,
                           ctr(p) + kCtrNnz, ctr(p) + kCtrError, s, p->merge_only ? ctr(p) + kCtrWaveSpan : nullptr));
  int64_t *h;
  st = read_counters(p, s, &h);
  if (st != SPGEMM_OK) return st;
  st = device_errors(p, h);
  if (st != SPGEMM_OK) return st;
  int64_t nnz = p->A.rows > 0 ? h[kCtrNnz] : 0;
  p->info.c_nnz = nnz;
  *c_nnz = nnz;
  if (p->merge_only) {
    p->merge_stage = merge_stage_for(h[kCtrWaveSpan]);
    p->info.multiplications = p->A.rows > 0 ? h[kCtrMults] : 0;
    p->info.rows_empty = p->A.rows > 0 ? h[kCtrEmpty] : 0;
    p->info.rows_merge = p->A.rows - p->info.rows_empty;
  }
  // size the numeric pass from the exact counts; with only a handful of
  // merge rows (a stencil's corners, say) sized again without the merge
  // tier, as for the one pass
  if (!p->merge_only) {
    st = size_pass(p, kNumeric, s);
    if (st == SPGEMM_OK && !p->merge_off && p->info.rows_merge > 0 &&
        p->info.rows_merge * kMergeFewRows < p->A.rows) {
      merge_off_for_resize(p);
      st = size_pass(p, kNumeric, s);
    }
    if (st == SPGEMM_OK) st = unstage_if_few(p, kNumeric, s);
    if (st != SPGEMM_OK) return st;
  }
  p->info.c_capacity_hint = nnz;
  p->stage = 1;
  return SPGEMM_OK;
}

}  // extern "C"

// The numeric call; `hbuf` (kNumCounters entries) receives the counters
// when given, else the thread's pinned buffer does.
static spgemm_status numeric_call(spgemm_plan *p, void *scratch, size_t scratch_bytes, const double *a_val,
                                  const double *b_val, int64_t *c_row_ptr, int32_t *c_col, double *c_val,
                                  int64_t c_capacity, int64_t *c_nnz, void *stream, int64_t *hbuf) {
  if (!p || !c_row_ptr || !c_nnz) return SPGEMM_E_NULL;
  if (c_capacity > 0 && (!c_col || !c_val)) return SPGEMM_E_NULL;
  if (c_capacity < 0) return SPGEMM_E_INVALID;
  const double *av = a_val ? a_val : p->A.val;
  const double *bv = b_val ? b_val : p->B.val;
  if ((p->A.nnz > 0 && !av) || (p->B.nnz > 0 && !bv)) return SPGEMM_E_NULL;
  hipStream_t s = (hipStream_t)stream;
  const bool two_pass = p->first_mode == kSymbolic;
  if (two_pass) {
    if (p->stage < 1) return SPGEMM_E_STATE;
    if (p->info.c_nnz > c_capacity) {
      *c_nnz = p->info.c_nnz;
      return SPGEMM_E_CAPACITY;
    }
  } else if (p->A.rows == 0) {
    HIPCK(p, launch_fill_i64(c_row_ptr, 0, 1, s));
    HIPCK(p, hipStreamSynchronize(s));
    *c_nnz = 0;
    p->info.c_nnz = 0;
    p->stage = 2;
    return SPGEMM_OK;
  }
  hipError_t e = hipSuccess;
  timing_begin(p, s, &e);
  HIPCK(p, e);
  spgemm_status st = numeric_enqueue(p, scratch, scratch_bytes, av, bv, c_row_ptr, c_col, c_val, c_capacity, s);
  if (st != SPGEMM_OK) return st;
  timing_end(p, s, &e);
  HIPCK(p, e);
  int64_t *h;
  st = read_counters(p, s, &h, hbuf);
  if (st != SPGEMM_OK) return st;
  st = device_errors(p, h);
  if (st != SPGEMM_OK) return st;
  if (two_pass) {
    *c_nnz = p->info.c_nnz;
  } else {
    p->info.c_nnz = h[kCtrNnz];
    p->info.overflow_rows = h[kCtrOverflow];
    p->info.spilled_rows = h[kCtrSpillRows];
    *c_nnz = h[kCtrNnz];
    if (h[kCtrNnz] > c_capacity) return SPGEMM_E_CAPACITY;
  }
  if (h[kCtrError] & kErrCapacity) return SPGEMM_E_CAPACITY;
  p->stage = 2;
  return SPGEMM_OK;
}

// ------------------------------------------- numeric pass without allocation
// The device tables of spgemm_numeric_static live in this array, one copy
// per device, held until the process ends.  In host code its name stands
// for a host-side symbol, not a device address: kernels are given the
// address hipGetSymbolAddress returns for the current device.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
constexpr int kStaticDevices = 64;
static __device__ __align__(256) char scratch_arena[kStaticScratchBytes];

static std::mutex g_arena_mu;
static void *g_arena_ptr[kStaticDevices];

// Device address of the current device's arena, looked up once per device
// (with that device current); nullptr when the lookup fails.
static void *arena_of_current_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kStaticDevices) return nullptr;
  std::lock_guard<std::mutex> g(g_arena_mu);
  if (!g_arena_ptr[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch_arena)) != hipSuccess || !ptr) return nullptr;
    g_arena_ptr[dev] = ptr;
  }
  return g_arena_ptr[dev];
}

extern "C" {

size_t spgemm_numeric_static_limit(void) { return kStaticScratchBytes; }

spgemm_status spgemm_numeric_static(spgemm_plan *p, const double *a_val, const double *b_val, int64_t *c_row_ptr,
                                    int32_t *c_col, double *c_val, int64_t c_capacity, int64_t *c_nnz,
                                    void *stream) {
  if (!p || !c_row_ptr || !c_nnz) return SPGEMM_E_NULL;
  int dev = -1;
  HIPCK(p, hipGetDevice(&dev));
  if (dev != p->device) return SPGEMM_E_STATE;
  // the one pass's padded buffer and one workgroup-tier table must fit;
  // fewer workgroup-tier workgroups run when not every table fits
  if (pad_bytes(p) + (size_t)p->scratch_slots * 12 > kStaticScratchBytes) return SPGEMM_E_WORKSPACE;
  void *arena = arena_of_current_device();
  if (!arena) {
    p->last_err = hipErrorInvalidSymbol;
    return SPGEMM_E_HIP;
  }
  int64_t h[kNumCounters];
  return numeric_call(p, arena, kStaticScratchBytes, a_val, b_val, c_row_ptr, c_col, c_val, c_capacity, c_nnz,
                      stream, h);
}

spgemm_status spgemm_numeric(spgemm_plan *p, void *scratch, size_t scratch_bytes, const double *a_val,
                             const double *b_val, int64_t *c_row_ptr, int32_t *c_col, double *c_val,
                             int64_t c_capacity, int64_t *c_nnz, void *stream) {
  return numeric_call(p, scratch, scratch_bytes, a_val, b_val, c_row_ptr, c_col, c_val, c_capacity, c_nnz, stream,
                      nullptr);
}

spgemm_status spgemm_compute_only(spgemm_plan *p, const double *a_val, const double *b_val, int32_t *row_nnz,
                                  double *row_maxabs, void *stream) {
  if (!p || (p->A.rows > 0 && (!row_nnz || !row_maxabs))) return SPGEMM_E_NULL;
  const double *av = a_val ? a_val : p->A.val;
  const double *bv = b_val ? b_val : p->B.val;
  if ((p->A.nnz > 0 && !av) || (p->B.nnz > 0 && !bv)) return SPGEMM_E_NULL;
  if (!p->merge_only && p->A.rows > 0) return SPGEMM_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  timing_begin(p, s, &e);
  HIPCK(p, e);
  HIPCK(p, launch_wave_merge(operands_of(p, av, bv), kComputeOnly, p->merge_m, 0, ctr(p), row_nnz, nullptr, nullptr,
                             nullptr, row_maxabs, 0, s));
  timing_end(p, s, &e);
  HIPCK(p, e);
  int64_t *h;
  spgemm_status st = read_counters(p, s, &h);
  if (st != SPGEMM_OK) return st;
  return device_errors(p, h);
}

spgemm_status spgemm_plan_info(const spgemm_plan *p, spgemm_info *info) {
  if (!p || !info) return SPGEMM_E_NULL;
  *info = p->info;
  return SPGEMM_OK;
}

int spgemm_plan_last_hip_error(const spgemm_plan *p) { return p ? (int)p->last_err : 0; }

void spgemm_plan_destroy(spgemm_plan *p) {
  if (!p) return;
  if (p->ev0) (void)hipEventDestroy(p->ev0);
  if (p->ev1) (void)hipEventDestroy(p->ev1);
  free(p);
}

}  // extern "C"
