// Batched products C_i = A_i * B_i (the C ABI of include/spgemm.h).
//
// The instances are laid side by side in one row space: the rows of all A_i
// follow each other, A_i's column indices are shifted by the number of B
// rows before instance i, and the B_i are stacked.  Row r of that product
// then combines only rows of its own B_i, so C is the concatenation of the
// C_i with every column index still in its instance's own range.  One plan
// (features, sizing, tiles) and one persistent numeric launch cover every
// row of every instance; after the first run the launches are captured in a
// HIP graph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../../include/spgemm.h"
#include "spgemm_kernels.h"
#include "spgemm_internal.h"

using namespace spg;

namespace {

constexpr int kCopyBlock = 256;
constexpr int64_t kChunk = 2048;   // elements per copy workgroup

struct InstDev {
  const int64_t *a_rp;
  const int32_t *a_col;
  const double *a_val;
  const int64_t *b_rp;
  const int32_t *b_col;
  const double *b_val;
  int64_t a_rows, b_rows, a_nnz, b_nnz;
  int64_t rbase, kbase, abase, bbase;
};

// A run of at most kChunk elements of one instance.
struct Chunk {
  int64_t inst;
  int64_t off;
};

enum CopyKind : int {
  kARows = 0,     // A row pointers (+ entry base)
  kBRows = 1,     // B row pointers (+ entry base)
  kAEnt = 2,      // A columns (+ B row base) and values
  kBEnt = 3,      // B columns and values
  kAVal = 4,      // A values only
  kBVal = 5,      // B values only
  kSplit = 6,     // per-instance row pointers of C from the concatenated ones
};

struct CopyArgs {
  const InstDev *inst;
  const Chunk *chunks;
  int kind;
  int64_t *a_rp;
  int32_t *a_col;
  double *a_val;
  int64_t *b_rp;
  int32_t *b_col;
  double *b_val;
  const int64_t *c_rp;     // concatenated row pointers of C (kSplit)
  int64_t *row_pool;       // kSplit output
};

__global__ void __launch_bounds__(kCopyBlock) k_batch_copy(CopyArgs a) {
  const Chunk ch = a.chunks[blockIdx.x];
  const InstDev d = a.inst[ch.inst];
  int64_t n;
  switch (a.kind) {
    case kARows: n = d.a_rows; break;
    case kBRows: n = d.b_rows; break;
    case kAEnt:
    case kAVal: n = d.a_nnz; break;
    case kBEnt:
    case kBVal: n = d.b_nnz; break;
    default: n = d.a_rows + 1; break;
  }
  const int64_t end = min(n, ch.off + kChunk);
  for (int64_t q = ch.off + threadIdx.x; q < end; q += kCopyBlock) {
    switch (a.kind) {
      case kARows: a.a_rp[d.rbase + q] = d.a_rp[q] + d.abase; break;
      case kBRows: a.b_rp[d.kbase + q] = d.b_rp[q] + d.bbase; break;
      case kAEnt:
        a.a_col[d.abase + q] = d.a_col[q] + (int32_t)d.kbase;
        a.a_val[d.abase + q] = d.a_val[q];
        break;
      case kBEnt:
        a.b_col[d.bbase + q] = d.b_col[q];
        a.b_val[d.bbase + q] = d.b_val[q];
        break;
      case kAVal: a.a_val[d.abase + q] = d.a_val[q]; break;
      case kBVal: a.b_val[d.bbase + q] = d.b_val[q]; break;
      default: a.row_pool[d.rbase + ch.inst + q] = a.c_rp[d.rbase + q] - a.c_rp[d.rbase]; break;
    }
  }
}

// Entry base and size of every instance in the concatenated C.
__global__ void k_batch_bounds(const InstDev *inst, int64_t count, const int64_t *c_rp, int64_t *out) {
  const int64_t i = blockIdx.x * (int64_t)kCopyBlock + threadIdx.x;
  if (i < count) {
    const int64_t b = c_rp[inst[i].rbase];
    out[i] = b;
    out[count + 1 + i] = c_rp[inst[i].rbase + inst[i].a_rows] - b;
  }
  if (i == count) out[count] = c_rp[inst[count - 1].rbase + inst[count - 1].a_rows];
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

struct spgemm_batch {
  int64_t count;
  std::vector<spgemm_csr> A, B;
  spgemm_options opts;
  spgemm_tuning tune;
  int has_tune;
  int64_t R, K, nnzA, nnzB, bcols;
  std::vector<InstDev> inst;
  std::vector<Chunk> chunks[7];
  // workspace offsets
  size_t o_inst, o_chunk[7], o_arp, o_acol, o_aval, o_brp, o_bcol, o_bval, o_crp, o_bounds, o_plan, total;
  size_t plan_bytes;
  char *ws;
  spgemm_plan *plan;
  spgemm_csr Acat, Bcat;
  int64_t *pinned;             // bounds (2 * count + 1) then counters
  hipGraph_t graph;
  hipGraphExec_t exec;
  void *g_scratch, *g_row, *g_col, *g_val;
  int64_t g_cap;
  int symbolic_done;
  hipStream_t cap_stream;      // capture stream (default priority)
  hipError_t last_err;
};

namespace {

template <typename T>
T *at(spgemm_batch *b, size_t off) {
  return reinterpret_cast<T *>(b->ws + off);
}

void add_chunks(std::vector<Chunk> &v, int64_t inst, int64_t n) {
  for (int64_t o = 0; o < n; o += kChunk) v.push_back({inst, o});
}

hipError_t launch_copy(spgemm_batch *b, int kind, hipStream_t s) {
  const std::vector<Chunk> &c = b->chunks[kind];
  if (c.empty()) return hipSuccess;
  CopyArgs a{};
  a.inst = at<InstDev>(b, b->o_inst);
  a.chunks = at<Chunk>(b, b->o_chunk[kind]);
  a.kind = kind;
  a.a_rp = at<int64_t>(b, b->o_arp);
  a.a_col = at<int32_t>(b, b->o_acol);
  a.a_val = at<double>(b, b->o_aval);
  a.b_rp = at<int64_t>(b, b->o_brp);
  a.b_col = at<int32_t>(b, b->o_bcol);
  a.b_val = at<double>(b, b->o_bval);
  a.c_rp = at<int64_t>(b, b->o_crp);
  a.row_pool = static_cast<int64_t *>(b->g_row);
  hipLaunchKernelGGL(k_batch_copy, dim3((unsigned)c.size()), dim3(kCopyBlock), 0, s, a);
  return hipGetLastError();
}

#define BCK(b, expr)                  \
  do {                                \
    hipError_t _e = (expr);           \
    if (_e != hipSuccess) {           \
      (b)->last_err = _e;             \
      return SPGEMM_E_HIP;            \
    }                                 \
  } while (0)

// Values of A and B into the concatenated operands, the numeric pass, the
// per-instance row pointers and bounds, and their copy to pinned memory:
// everything a run does on the device, in stream order.
spgemm_status enqueue_run(spgemm_batch *b, void *scratch, size_t scratch_bytes, int32_t *c_col, double *c_val,
                          int64_t c_capacity, hipStream_t s) {
  BCK(b, launch_copy(b, kAVal, s));
  BCK(b, launch_copy(b, kBVal, s));
  spgemm_status st = numeric_enqueue(b->plan, scratch, scratch_bytes, at<double>(b, b->o_aval),
                                     at<double>(b, b->o_bval), at<int64_t>(b, b->o_crp), c_col, c_val, c_capacity, s);
  if (st != SPGEMM_OK) return st;
  BCK(b, launch_copy(b, kSplit, s));
  hipLaunchKernelGGL(k_batch_bounds, dim3((unsigned)((b->count + kCopyBlock) / kCopyBlock)), dim3(kCopyBlock), 0, s,
                     at<InstDev>(b, b->o_inst), b->count, at<int64_t>(b, b->o_crp), at<int64_t>(b, b->o_bounds));
  BCK(b, hipGetLastError());
  BCK(b, hipMemcpyAsync(b->pinned, at<int64_t>(b, b->o_bounds), sizeof(int64_t) * (2 * b->count + 1),
                        hipMemcpyDeviceToHost, s));
  BCK(b, hipMemcpyAsync(b->pinned + 2 * b->count + 1, plan_counters(b->plan), sizeof(int64_t) * kNumCounters,
                        hipMemcpyDeviceToHost, s));
  return SPGEMM_OK;
}

spgemm_status finish_run(spgemm_batch *b, int64_t c_capacity, int64_t *c_nnz_base, int64_t *c_nnz,
                         int64_t *c_required) {
  const int64_t *h = b->pinned + 2 * b->count + 1;
  spgemm_status st = plan_check_counters(b->plan, h);
  if (st != SPGEMM_OK) return st;
  const int64_t total = b->pinned[b->count];
  if (c_required) *c_required = total;
  if (total > c_capacity || (h[kCtrError] & kErrCapacity)) return SPGEMM_E_CAPACITY;
  for (int64_t i = 0; i <= b->count; ++i) c_nnz_base[i] = b->pinned[i];
  for (int64_t i = 0; i < b->count; ++i) c_nnz[i] = b->pinned[b->count + 1 + i];
  return SPGEMM_OK;
}

void drop_graph(spgemm_batch *b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

}  // namespace

extern "C" {

spgemm_status spgemm_batched_plan(int64_t count, const spgemm_csr *A, const spgemm_csr *B,
                                  const spgemm_options *opts, int64_t *c_row_base, size_t *workspace_bytes,
                                  spgemm_batch **out) {
  if (!out || !opts || !workspace_bytes || !c_row_base) return SPGEMM_E_NULL;
  *out = nullptr;
  if (count < 0) return SPGEMM_E_INVALID;
  if (count > 0 && (!A || !B)) return SPGEMM_E_NULL;
  if (opts->sizer < 0 || opts->sizer > 2) return SPGEMM_E_INVALID;
  if (opts->sizer == SPGEMM_SIZER_LEARNED && !opts->model) return SPGEMM_E_NO_MODEL;
  spgemm_batch *b = new (std::nothrow) spgemm_batch();
  if (!b) return SPGEMM_E_INVALID;
  b->count = count;
  b->opts = *opts;
  if (opts->tuning) {
    b->tune = *opts->tuning;
    b->has_tune = 1;
  }
  b->opts.tuning = nullptr;
  int64_t R = 0, K = 0, na = 0, nb = 0, bc = 0;
  c_row_base[0] = 0;
  for (int64_t i = 0; i < count; ++i) {
    const spgemm_csr &a = A[i], &bb = B[i];
    if (a.rows < 0 || a.cols < 0 || a.nnz < 0 || bb.rows < 0 || bb.cols < 0 || bb.nnz < 0 || a.cols != bb.rows) {
      delete b;
      return SPGEMM_E_DIM;
    }
    if (!a.row_ptr || !bb.row_ptr || (a.nnz > 0 && (!a.col_idx || !a.val)) || (bb.nnz > 0 && (!bb.col_idx || !bb.val))) {
      delete b;
      return SPGEMM_E_NULL;
    }
    InstDev d{a.row_ptr, a.col_idx, a.val, bb.row_ptr, bb.col_idx, bb.val, a.rows, bb.rows, a.nnz, bb.nnz,
              R, K, na, nb};
    b->inst.push_back(d);
    add_chunks(b->chunks[kARows], i, a.rows);
    add_chunks(b->chunks[kBRows], i, bb.rows);
    add_chunks(b->chunks[kAEnt], i, a.nnz);
    add_chunks(b->chunks[kBEnt], i, bb.nnz);
    add_chunks(b->chunks[kSplit], i, a.rows + 1);
    R += a.rows;
    K += bb.rows;
    na += a.nnz;
    nb += bb.nnz;
    bc = std::max<int64_t>(bc, bb.cols);
    c_row_base[i + 1] = c_row_base[i] + a.rows + 1;
  }
  b->chunks[kAVal] = b->chunks[kAEnt];
  b->chunks[kBVal] = b->chunks[kBEnt];
  if (R >= ((int64_t)1 << 31) || K >= ((int64_t)1 << 31) || bc >= ((int64_t)1 << 31)) {
    delete b;
    return SPGEMM_E_INDEX_OVERFLOW;
  }
  b->A.assign(A, A + count);
  b->B.assign(B, B + count);
  b->R = R;
  b->K = K;
  b->nnzA = na;
  b->nnzB = nb;
  b->bcols = bc;
  // concatenated operands (descriptors only; the data lives in the workspace)
  b->Acat = spgemm_csr{R, K, na, nullptr, nullptr, nullptr};
  b->Bcat = spgemm_csr{K, bc, nb, nullptr, nullptr, nullptr};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t a = o;
    o = align256(o + std::max<size_t>(bytes, 1));
    return a;
  };
  b->o_inst = take(sizeof(InstDev) * (size_t)std::max<int64_t>(count, 1));
  for (int k = 0; k < 7; ++k) b->o_chunk[k] = take(sizeof(Chunk) * b->chunks[k].size());
  b->o_arp = take(8 * (size_t)(R + 1));
  b->o_acol = take(4 * (size_t)na);
  b->o_aval = take(8 * (size_t)na);
  b->o_brp = take(8 * (size_t)(K + 1));
  b->o_bcol = take(4 * (size_t)nb);
  b->o_bval = take(8 * (size_t)nb);
  b->o_crp = take(8 * (size_t)(R + 1));
  b->o_bounds = take(8 * (size_t)(2 * count + 1));
  b->plan_bytes = plan_workspace_bytes(R, K);
  b->o_plan = take(b->plan_bytes);
  b->total = o;
  *workspace_bytes = b->total;
  *out = b;
  return SPGEMM_OK;
}

spgemm_status spgemm_batched_reserve(spgemm_batch *b, void *workspace, size_t workspace_bytes, int64_t *c_capacity,
                                     size_t *scratch_bytes, void *stream) {
  if (!b || !workspace || !c_capacity || !scratch_bytes) return SPGEMM_E_NULL;
  if (workspace_bytes < b->total || !aligned256(workspace)) return SPGEMM_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  if (!b->pinned) {
    // host buffer the runs read the instances' sizes and the counters into
    void *pin = nullptr;
    if (hipHostMalloc(&pin, sizeof(int64_t) * (2 * b->count + 1 + kNumCounters), hipHostMallocDefault) != hipSuccess)
      return SPGEMM_E_HIP;
    b->pinned = static_cast<int64_t *>(pin);
  }
  drop_graph(b);
  if (b->plan) {
    spgemm_plan_destroy(b->plan);
    b->plan = nullptr;
  }
  b->ws = static_cast<char *>(workspace);
  b->symbolic_done = 0;
  if (b->count > 0) {
    BCK(b, hipMemcpyAsync(b->ws + b->o_inst, b->inst.data(), sizeof(InstDev) * b->count, hipMemcpyHostToDevice, s));
    for (int k = 0; k < 7; ++k)
      if (!b->chunks[k].empty())
        BCK(b, hipMemcpyAsync(b->ws + b->o_chunk[k], b->chunks[k].data(), sizeof(Chunk) * b->chunks[k].size(),
                              hipMemcpyHostToDevice, s));
  }
  BCK(b, launch_fill_i64(at<int64_t>(b, b->o_arp) + b->R, b->nnzA, 1, s));
  BCK(b, launch_fill_i64(at<int64_t>(b, b->o_brp) + b->K, b->nnzB, 1, s));
  BCK(b, launch_copy(b, kARows, s));
  BCK(b, launch_copy(b, kBRows, s));
  BCK(b, launch_copy(b, kAEnt, s));
  BCK(b, launch_copy(b, kBEnt, s));
  b->Acat.row_ptr = at<int64_t>(b, b->o_arp);
  b->Acat.col_idx = at<int32_t>(b, b->o_acol);
  b->Acat.val = at<double>(b, b->o_aval);
  b->Bcat.row_ptr = at<int64_t>(b, b->o_brp);
  b->Bcat.col_idx = at<int32_t>(b, b->o_bcol);
  b->Bcat.val = at<double>(b, b->o_bval);
  spgemm_options o = b->opts;
  o.tuning = b->has_tune ? &b->tune : nullptr;
  spgemm_info info{};
  spgemm_status st = spgemm_plan_create(&b->Acat, &b->Bcat, &o, b->ws + b->o_plan, b->plan_bytes, stream, &b->plan,
                                        &info);
  if (st != SPGEMM_OK) return st;
  if (info.c_capacity_hint < 0) {
    // an exact plan whose rows all merge in registers learns its sizes from
    // its symbolic pass (which needs no scratch): the pools get the exact size
    int64_t nnz = 0;
    st = spgemm_symbolic(b->plan, nullptr, 0, at<int64_t>(b, b->o_crp), &nnz, stream);
    if (st != SPGEMM_OK) return st;
    b->symbolic_done = 1;
    info.c_capacity_hint = nnz;
  }
  *c_capacity = info.c_capacity_hint;
  *scratch_bytes = info.scratch_bytes;
  return SPGEMM_OK;
}

spgemm_status spgemm_batched(spgemm_batch *b, void *scratch, size_t scratch_bytes, int64_t *c_row_pool,
                             int32_t *c_col_pool, double *c_val_pool, int64_t c_capacity, int64_t *c_nnz_base,
                             int64_t *c_nnz, int64_t *c_required, void *stream) {
  if (!b || !c_nnz_base || !c_nnz) return SPGEMM_E_NULL;
  if (!b->plan) return SPGEMM_E_STATE;
  if (b->count > 0 && !c_row_pool) return SPGEMM_E_NULL;
  if (c_capacity < 0) return SPGEMM_E_INVALID;
  if (c_capacity > 0 && (!c_col_pool || !c_val_pool)) return SPGEMM_E_NULL;
  if (b->count == 0) {
    c_nnz_base[0] = 0;
    if (c_required) *c_required = 0;
    return SPGEMM_OK;
  }
  hipStream_t s = (hipStream_t)stream;
  const bool same = b->exec && b->g_scratch == scratch && b->g_row == (void *)c_row_pool &&
                    b->g_col == (void *)c_col_pool && b->g_val == (void *)c_val_pool && b->g_cap == c_capacity;
  if (same) {
    BCK(b, hipGraphLaunch(b->exec, s));
    BCK(b, hipStreamSynchronize(s));
    spgemm_status st = finish_run(b, c_capacity, c_nnz_base, c_nnz, c_required);
    if (st == SPGEMM_OK || st == SPGEMM_E_CAPACITY) return st;
    drop_graph(b);   // fall back to a checked run below
  }
  drop_graph(b);
  b->g_row = c_row_pool;
  // first run (or new pointers): the checked host path, which also settles
  // the launch shapes the graph will keep
  BCK(b, launch_copy(b, kAVal, s));
  BCK(b, launch_copy(b, kBVal, s));
  int64_t nnz = 0;
  spgemm_status st = SPGEMM_OK;
  if (!plan_is_one_pass(b->plan) && !b->symbolic_done) {
    st = spgemm_symbolic(b->plan, scratch, scratch_bytes, at<int64_t>(b, b->o_crp), &nnz, stream);
    if (st != SPGEMM_OK) return st;
    b->symbolic_done = 1;
  }
  st = spgemm_numeric(b->plan, scratch, scratch_bytes, at<double>(b, b->o_aval), at<double>(b, b->o_bval),
                      at<int64_t>(b, b->o_crp), c_col_pool, c_val_pool, c_capacity, &nnz, stream);
  if (st == SPGEMM_E_CAPACITY) {
    if (c_required) *c_required = nnz;
    return st;
  }
  if (st != SPGEMM_OK) return st;
  BCK(b, launch_copy(b, kSplit, s));
  hipLaunchKernelGGL(k_batch_bounds, dim3((unsigned)((b->count + kCopyBlock) / kCopyBlock)), dim3(kCopyBlock), 0, s,
                     at<InstDev>(b, b->o_inst), b->count, at<int64_t>(b, b->o_crp), at<int64_t>(b, b->o_bounds));
  BCK(b, hipGetLastError());
  BCK(b, hipMemcpyAsync(b->pinned, at<int64_t>(b, b->o_bounds), sizeof(int64_t) * (2 * b->count + 1),
                        hipMemcpyDeviceToHost, s));
  BCK(b, hipMemcpyAsync(b->pinned + 2 * b->count + 1, plan_counters(b->plan), sizeof(int64_t) * kNumCounters,
                        hipMemcpyDeviceToHost, s));
  BCK(b, hipStreamSynchronize(s));
  st = finish_run(b, c_capacity, c_nnz_base, c_nnz, c_required);
  if (st != SPGEMM_OK) return st;
  // capture the same launches for later calls with these pointers (on the
  // batch's own stream: the caller's may be the null stream, which cannot
  // be captured; the graph is launched on the caller's stream)
  if (!b->cap_stream) BCK(b, hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
  BCK(b, hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
  spgemm_status cst = enqueue_run(b, scratch, scratch_bytes, c_col_pool, c_val_pool, c_capacity, b->cap_stream);
  hipGraph_t g = nullptr;
  hipError_t ee = hipStreamEndCapture(b->cap_stream, &g);
  if (cst != SPGEMM_OK || ee != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return SPGEMM_OK;   // this run's result stands; later calls take the checked path again
  }
  hipGraphExec_t ex = nullptr;
  if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g);
    return SPGEMM_OK;
  }
  b->graph = g;
  b->exec = ex;
  b->g_scratch = scratch;
  b->g_col = c_col_pool;
  b->g_val = c_val_pool;
  b->g_cap = c_capacity;
  return SPGEMM_OK;
}

int spgemm_batched_uses_graph(const spgemm_batch *b) { return b && b->exec ? 1 : 0; }

void spgemm_batched_destroy(spgemm_batch *b) {
  if (!b) return;
  drop_graph(b);
  if (b->plan) spgemm_plan_destroy(b->plan);
  if (b->pinned) (void)hipHostFree(b->pinned);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  delete b;
}

}  // extern "C"
