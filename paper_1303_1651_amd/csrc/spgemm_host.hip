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
  size_t counters, model, partials, keys, nnz_a, ub, maxb, lo, hi, pred, cnt, info, cap, cost, tile_row, status, scan_status, total;
};

Layout layout_for(int64_t rows) {
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
  L.partials = take(sizeof(int64_t) * 8 * (R / 256 + 2));
  L.keys = take(sizeof(uint64_t) * R);
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
  L.total = o;
  return L;
}

spgemm_tuning default_tuning(const spgemm_csr *A, const spgemm_csr *B) {
  spgemm_tuning t{};
  double avg_b = B->rows > 0 ? (double)B->nnz / (double)B->rows : 1.0;
  int g = 4;
  while (g < 64 && g < avg_b) g <<= 1;
  t.hash_group = g;
  t.pool_slots = 4096;
  t.max_tile_rows = 256;
  t.merge_max_nnz = 64;
  t.merge_lists = 8;
  t.dense_ratio = 2.0f;
  t.margin = 0.05f;
  t.slack = 2;
  t.blocks_per_cu = 4;
  return t;
}

static void merge_tuning(spgemm_tuning *t, const spgemm_tuning *u) {
  if (!u) return;
  if (u->hash_group) t->hash_group = u->hash_group;
  if (u->pool_slots) t->pool_slots = u->pool_slots < 0 ? 0 : u->pool_slots;
  if (u->max_tile_rows) t->max_tile_rows = u->max_tile_rows;
  if (u->merge_max_nnz) t->merge_max_nnz = u->merge_max_nnz < 0 ? 0 : u->merge_max_nnz;
  if (u->merge_lists) t->merge_lists = u->merge_lists;
  if (u->dense_ratio > 0) t->dense_ratio = u->dense_ratio;
  if (u->margin > 0) t->margin = u->margin;
  if (u->slack) t->slack = u->slack;
  if (u->blocks_per_cu) t->blocks_per_cu = u->blocks_per_cu;
}

static bool tuning_ok(const spgemm_tuning &t) {
  bool g_ok = t.hash_group == 4 || t.hash_group == 8 || t.hash_group == 16 || t.hash_group == 32 ||
              t.hash_group == 64;
  return g_ok && t.pool_slots >= 0 && t.pool_slots <= 12288 && t.max_tile_rows >= 1 &&
         t.max_tile_rows <= kMaxTileRows && (t.merge_lists == 4 || t.merge_lists == 8) && t.merge_max_nnz >= 0 &&
         t.dense_ratio >= 0 && t.margin >= 0 && t.slack >= 0 && t.blocks_per_cu >= 1 &&
         t.blocks_per_cu <= 16;
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
  int64_t scratch_slots;   // per workgroup, current sizing
  int64_t scratch_slots_plan;
  int grid;
  int has_pool;
  int has_hash;
  int merge_only;      // every row takes the register-merge tier: row-per-thread kernels
  spgemm_info info;
  hipError_t last_err;
  const spgemm_model *model;
  uint64_t *keys;        // packed feature triple per row
  hipEvent_t ev0, ev1;   // SPGEMM_OPT_TIMING
  int timing_pending;
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

// Read the device counters into the pinned host buffer (synchronises).
static spgemm_status read_counters(spgemm_plan *p, hipStream_t s, int64_t **out) {
  int64_t *h = host_counters();
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

// Sizing of one pass (tiers, capacities, tile costs) plus tile bounds.
static spgemm_status size_pass(spgemm_plan *p, int mode, hipStream_t s) {
  SizeParams sp{};
  sp.mode = mode;
  sp.sizer = p->opts.sizer;
  sp.pool_slots = p->tune.pool_slots;
  sp.pad = 16;
  sp.merge_lists = p->tune.merge_lists;
  sp.merge_max = p->tune.merge_max_nnz;
  sp.tile_rows = p->tune.max_tile_rows;
  sp.dense_ratio = p->tune.dense_ratio;
  sp.margin = p->tune.margin;
  sp.slack = p->tune.slack;
  sp.pred = p->pa.pred;
  sp.cnt = p->pa.cnt;
  Operands op = operands_of(p, nullptr, nullptr);
  HIPCK(p, launch_size_rows(op, p->pa, sp, s));
  const int64_t R = p->A.rows;
  HIPCK(p, launch_scan_i64_inplace(p->pa.cost, R, p->pa.scan_status, ctr(p) + kCtrScanTicket,
                                   ctr(p) + kCtrError, s));
  HIPCK(p, launch_tile_bounds(p->pa.cost, R, tile_budget(p->tune.pool_slots, p->tune.max_tile_rows),
                              p->pa.tile_row, ctr(p), s));
  int64_t *h;
  spgemm_status st = read_counters(p, s, &h);
  if (st != SPGEMM_OK) return st;
  if (h[kCtrError] & kErrLookback) return lookback_failed(p);
  p->ntiles = h[kCtrTiles];
  p->scratch_slots = (h[kCtrScratch] + 1) & ~(int64_t)1;
  p->has_pool = h[kCtrPoolRows] > 0;
  p->has_hash = h[kCtrHash] + h[kCtrGlobal] > 0;
  p->cur_mode = mode;
  p->info.rows_merge = h[kCtrMerge];
  p->info.rows_hash = h[kCtrHash];
  p->info.rows_global = h[kCtrGlobal];
  p->info.rows_empty = h[kCtrEmpty];
  p->info.tiles = p->ntiles;
  if (mode != kNumeric) p->info.c_capacity_hint = h[kCtrCapSum];
  return SPGEMM_OK;
}

static int tile_grid(const spgemm_plan *p, size_t scratch_bytes) {
  int64_t g = (int64_t)device_cus() * p->tune.blocks_per_cu;
  g = std::min<int64_t>(g, std::max<int64_t>(p->ntiles, 1));
  if (p->scratch_slots > 0) {
    int64_t by_scratch = (int64_t)(scratch_bytes / ((size_t)p->scratch_slots * 12));
    g = std::min(g, by_scratch);
  }
  return (int)g;
}

static size_t pool_bytes(const spgemm_plan *p) {
  if (!p->has_pool) return 0;
  return (((size_t)p->tune.pool_slots * 4 + 15) & ~(size_t)15) + (size_t)p->tune.pool_slots * 8;
}

static spgemm_status run_tiles(spgemm_plan *p, int mode, void *scratch, size_t scratch_bytes,
                               const double *a_val, const double *b_val, int64_t *c_rp, int32_t *c_col,
                               double *c_val, int64_t c_capacity, hipStream_t s) {
  if (p->ntiles == 0) return SPGEMM_OK;
  if (p->scratch_slots > 0 && (!scratch || scratch_bytes < (size_t)p->scratch_slots * 12))
    return SPGEMM_E_WORKSPACE;
  TileParams tp{};
  tp.op = operands_of(p, a_val, b_val);
  tp.info = p->pa.info;
  tp.cap = p->pa.cap;
  tp.ub = p->pa.f.ub;
  tp.lo = p->pa.f.lo;
  tp.hi = p->pa.f.hi;
  tp.cost = p->pa.cost;
  tp.tile_row = p->pa.tile_row;
  tp.counters = ctr(p);
  tp.status = p->pa.status;
  tp.cnt_out = p->pa.cnt;
  tp.c_rp = c_rp;
  tp.c_col = c_col;
  tp.c_val = c_val;
  tp.c_capacity = c_capacity;
  tp.scratch = static_cast<char *>(scratch);
  tp.scratch_slots = p->scratch_slots;
  tp.pool_slots = p->tune.pool_slots;
  tp.pad = 16;
  tp.fast = (p->opts.flags & SPGEMM_OPT_FAST) ? 1 : 0;
  HIPCK(p, launch_fill_i64(ctr(p) + kCtrTicket, 0, 1, s));
  HIPCK(p, launch_fill_i64(ctr(p) + kCtrError, 0, 1, s));
  HIPCK(p, launch_fill_i64(ctr(p) + kCtrOverflow, 0, 1, s));
  if (mode == kOnePass) HIPCK(p, launch_fill_u64(p->pa.status, 0, p->ntiles, s));
  int grid = tile_grid(p, scratch_bytes);
  if (p->ev0) HIPCK(p, hipEventRecord(p->ev0, s));
  HIPCK(p, launch_tiles(tp, mode, p->tune.hash_group, p->tune.merge_lists, p->has_hash != 0, grid,
                        pool_bytes(p), s));
  if (p->ev1) {
    HIPCK(p, hipEventRecord(p->ev1, s));
    p->timing_pending = 1;
  }
  return SPGEMM_OK;
}

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
  *bytes = layout_for(A->rows).total;
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
  Layout L = layout_for(A->rows);
  if (!workspace) return SPGEMM_E_NULL;
  if (workspace_bytes < L.total) return SPGEMM_E_WORKSPACE;
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
  p->model = opts->model;
  p->ws = static_cast<char *>(workspace);
  p->ws_bytes = workspace_bytes;
  p->L = L;
  p->info.c_nnz = -1;
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
  p->keys = (uint64_t *)(w + L.keys);
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
  // Row sums (multiplications, longest A row, empty rows) and, for the
  // learned sizer, the packed feature triple of every row and the learned
  // capacity; one synchronisation.
  if (launch_features(op, p->pa.f, p->keys, p->pa.counters, p->pa.partials, learned ? 1 : 0, s) != hipSuccess)
    return fail(SPGEMM_E_HIP);
  if (learned) {
    if (launch_mlp_capacity(dev, p->keys, A->rows, s, p->tune.margin, p->tune.slack, p->pa.partials) != hipSuccess)
      return fail(SPGEMM_E_HIP);
    const int32_t dst[1] = {kCtrCapSum};
    if (launch_sum_partials(p->pa.partials, std::max<int64_t>(1, mlp_predict_blocks(A->rows)), 1, 1, dst, nullptr,
                            p->pa.counters, s) != hipSuccess)
      return fail(SPGEMM_E_HIP);
  }
  int64_t *h;
  st = read_counters(p, s, &h);
  if (st != SPGEMM_OK) return fail(st);
  // Every row merges in registers when no row of A has more stored entries
  // than the merge tier's lists (and the tier is not switched off); then no
  // per-row plan arrays are needed.
  p->merge_only = A->rows > 0 && h[kCtrMaxA] <= p->tune.merge_lists && p->tune.merge_max_nnz > 0;
  if (p->merge_only) {
    p->info.rows_empty = h[kCtrEmpty];
    p->info.rows_merge = A->rows - h[kCtrEmpty];
    p->info.tiles = (A->rows + 63) / 64;
    p->info.c_capacity_hint = learned ? h[kCtrCapSum] + h[kCtrUnpacked] : h[kCtrMults];
    p->ntiles = p->info.tiles;
    p->cur_mode = p->first_mode;
  } else {
    if (launch_features(op, p->pa.f, p->keys, p->pa.counters, p->pa.partials, 2, s) != hipSuccess)
      return fail(SPGEMM_E_HIP);
    if (learned) {
      if (launch_mlp_predict(dev, p->pa.f.nnz_a, p->pa.f.ub, p->pa.f.maxb, A->rows, p->pa.pred, s, p->tune.margin,
                             p->tune.slack, nullptr) != hipSuccess)
        return fail(SPGEMM_E_HIP);
    }
    st = size_pass(p, p->first_mode, s);
    if (st != SPGEMM_OK) return fail(st);
    st = read_counters(p, s, &h);
    if (st != SPGEMM_OK) return fail(st);
  }
  p->info.multiplications = h[kCtrMults];
  p->scratch_slots_plan = p->scratch_slots;
  // room for one table per resident workgroup
  int64_t groups = (int64_t)device_cus() * p->tune.blocks_per_cu;
  p->info.scratch_bytes = (size_t)(p->scratch_slots * 12) * (size_t)groups;
  if (info) *info = p->info;
  *out = p;
  return SPGEMM_OK;
}

spgemm_status spgemm_symbolic(spgemm_plan *p, void *scratch, size_t scratch_bytes, int64_t *c_row_ptr,
                              int64_t *c_nnz, void *stream) {
  if (!p || !c_row_ptr || !c_nnz) return SPGEMM_E_NULL;
  if (p->first_mode != kSymbolic || p->stage != 0) return SPGEMM_E_STATE;
  hipStream_t s = (hipStream_t)stream;
  spgemm_status st = SPGEMM_OK;
  if (p->merge_only) {
    HIPCK(p, launch_fill_i64(ctr(p) + kCtrError, 0, 1, s));
    HIPCK(p, launch_wave_merge(operands_of(p, nullptr, nullptr), kSymbolic, p->tune.merge_lists, ctr(p),
                               p->pa.status, p->pa.cnt, nullptr, nullptr, nullptr, 0, s));
  } else {
    st = run_tiles(p, kSymbolic, scratch, scratch_bytes, nullptr, nullptr, nullptr, nullptr, nullptr, 0, s);
    if (st != SPGEMM_OK) return st;
  }
  HIPCK(p, launch_scan_i32(p->pa.cnt, c_row_ptr, p->A.rows, p->pa.scan_status, ctr(p) + kCtrScanTicket,
                           ctr(p) + kCtrNnz, ctr(p) + kCtrError, s));
  int64_t *h;
  st = read_counters(p, s, &h);
  if (st != SPGEMM_OK) return st;
  st = device_errors(p, h);
  if (st != SPGEMM_OK) return st;
  int64_t nnz = p->A.rows > 0 ? h[kCtrNnz] : 0;
  p->info.c_nnz = nnz;
  p->info.c_capacity_hint = nnz;
  *c_nnz = nnz;
  // size the numeric pass from the exact counts
  if (!p->merge_only) {
    st = size_pass(p, kNumeric, s);
    if (st != SPGEMM_OK) return st;
  }
  p->info.c_capacity_hint = nnz;
  p->stage = 1;
  return SPGEMM_OK;
}

spgemm_status spgemm_numeric(spgemm_plan *p, void *scratch, size_t scratch_bytes, const double *a_val,
                             const double *b_val, int64_t *c_row_ptr, int32_t *c_col, double *c_val,
                             int64_t c_capacity, int64_t *c_nnz, void *stream) {
  if (!p || !c_row_ptr || !c_nnz) return SPGEMM_E_NULL;
  if (c_capacity > 0 && (!c_col || !c_val)) return SPGEMM_E_NULL;
  if (c_capacity < 0) return SPGEMM_E_INVALID;
  const double *av = a_val ? a_val : p->A.val;
  const double *bv = b_val ? b_val : p->B.val;
  if ((p->A.nnz > 0 && !av) || (p->B.nnz > 0 && !bv)) return SPGEMM_E_NULL;
  hipStream_t s = (hipStream_t)stream;
  if (p->first_mode == kSymbolic) {
    if (p->stage < 1) return SPGEMM_E_STATE;
    if (p->info.c_nnz > c_capacity) {
      *c_nnz = p->info.c_nnz;
      return SPGEMM_E_CAPACITY;
    }
    spgemm_status st = SPGEMM_OK;
    if (p->merge_only) {
      HIPCK(p, launch_fill_i64(ctr(p) + kCtrError, 0, 1, s));
      if (p->ev0) HIPCK(p, hipEventRecord(p->ev0, s));
      HIPCK(p, launch_wave_merge(operands_of(p, av, bv), kNumeric, p->tune.merge_lists, ctr(p), p->pa.status,
                                 nullptr, c_row_ptr, c_col, c_val, c_capacity, s));
      if (p->ev1) {
        HIPCK(p, hipEventRecord(p->ev1, s));
        p->timing_pending = 1;
      }
    } else {
      st = run_tiles(p, kNumeric, scratch, scratch_bytes, av, bv, c_row_ptr, c_col, c_val, c_capacity, s);
      if (st != SPGEMM_OK) return st;
    }
    int64_t *h;
    st = read_counters(p, s, &h);
    if (st != SPGEMM_OK) return st;
    st = device_errors(p, h);
    if (st != SPGEMM_OK) return st;
    *c_nnz = p->info.c_nnz;
    if (h[kCtrError] & kErrCapacity) return SPGEMM_E_CAPACITY;
    p->stage = 2;
    return SPGEMM_OK;
  }
  // one-pass sizers
  if (p->A.rows == 0) {
    HIPCK(p, launch_fill_i64(c_row_ptr, 0, 1, s));
    HIPCK(p, hipStreamSynchronize(s));
    *c_nnz = 0;
    p->info.c_nnz = 0;
    return SPGEMM_OK;
  }
  spgemm_status st = SPGEMM_OK;
  if (p->merge_only) {
    HIPCK(p, launch_fill_i64(ctr(p) + kCtrTicket, 0, 1, s));
    HIPCK(p, launch_fill_i64(ctr(p) + kCtrError, 0, 1, s));
    HIPCK(p, launch_fill_u64(p->pa.status, 0, p->ntiles, s));
    if (p->ev0) HIPCK(p, hipEventRecord(p->ev0, s));
    HIPCK(p, launch_wave_merge(operands_of(p, av, bv), kOnePass, p->tune.merge_lists, ctr(p), p->pa.status,
                               nullptr, c_row_ptr, c_col, c_val, c_capacity, s));
    if (p->ev1) {
      HIPCK(p, hipEventRecord(p->ev1, s));
      p->timing_pending = 1;
    }
  } else {
    st = run_tiles(p, kOnePass, scratch, scratch_bytes, av, bv, c_row_ptr, c_col, c_val, c_capacity, s);
    if (st != SPGEMM_OK) return st;
  }
  int64_t *h;
  st = read_counters(p, s, &h);
  if (st != SPGEMM_OK) return st;
  st = device_errors(p, h);
  if (st != SPGEMM_OK) return st;
  int64_t nnz = h[kCtrNnz];
  p->info.c_nnz = nnz;
  p->info.overflow_rows = h[kCtrOverflow];
  *c_nnz = nnz;
  if (h[kCtrError] & kErrCapacity) return SPGEMM_E_CAPACITY;
  p->stage = 2;
  return SPGEMM_OK;
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
