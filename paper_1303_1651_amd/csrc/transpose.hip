// Transpose of a CSR matrix: the conversion of a right-hand operand given by
// columns (CSC) to rows (CSR).  Section IV-A multiplies CSR by CSR row by row
// and takes a CSC right-hand side by converting it to CSR first; the arrays
// of a CSC matrix are those of the CSR of its transpose, so the conversion is
// this transpose.
//
// Steps: count the entries of every column, each entry keeping the count it
// found as its place in its column (an atomic add, so the order inside a
// column is not yet fixed); scan the counts into the row pointers of the
// transpose; move every entry of M to its place, into scratch; then each row
// of the transpose is written in increasing column order, every entry at the
// number of smaller columns in its row (the columns of a row are distinct
// for a canonical M): counted by shuffles for short rows, by a sort in LDS
// for rows of up to kTrSortMax entries, and for longer ones from sorted
// chunks (the entry's place in its chunk plus a binary search in each
// other chunk).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.h"
#include "spgemm_internal.h"
#include "spgemm_kernels.h"

namespace spg {
namespace {

constexpr int64_t kTrErrRange = 1;     // a column index outside [0, cols)
constexpr int64_t kTrErrRowPtr = 2;    // row_ptr[rows] differs from nnz
constexpr int64_t kTrLong = 256;       // rows longer than this are ordered by a workgroup
constexpr int kTrSortMax = 4096;       // ... by a bitonic sort in LDS up to this length

__global__ void __launch_bounds__(kBlock) k_tr_zero(int32_t *p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) p[i] = 0;
}

__global__ void __launch_bounds__(kBlock) k_tr_check(const int64_t *rp, int64_t rows, int64_t nnz, int64_t *err) {
  if (blockIdx.x == 0 && threadIdx.x == 0 && rp[rows] != nnz)
    atomicOr((unsigned long long *)err, (unsigned long long)kTrErrRowPtr);
}

// Entries per column of M (rows of the transpose); each entry keeps its
// place in its column.
__global__ void __launch_bounds__(kBlock) k_tr_count(const int32_t *col, int64_t nnz, int64_t cols, int32_t *cnt,
                                                     int32_t *place, int64_t *err) {
  for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * kBlock) {
    const int32_t c = col[e];
    if (c < 0 || (int64_t)c >= cols) {
      atomicOr((unsigned long long *)err, (unsigned long long)kTrErrRange);
      place[e] = -1;
      continue;
    }
    place[e] = atomicAdd(&cnt[c], 1);
  }
}

// A group of 2^lg lanes per row (2^lg at least the mean row length, at most
// a wave), 64 >> lg rows per wave at a time.
// Entry (r, c) of M goes to its place in row c of the transpose (in
// scratch).
__global__ void __launch_bounds__(kBlock) k_tr_scatter(const int64_t *rp, const int32_t *col, const double *val,
                                                       int64_t rows, const int64_t *t_rp, const int32_t *place,
                                                       int32_t *tmp_col, double *tmp_val, int lg) {
  const int G = 1 << lg;
  const int gl = (int)(threadIdx.x & (G - 1));
  const int64_t ng = (int64_t)gridDim.x * (kBlock >> lg);
  for (int64_t r = (blockIdx.x * (int64_t)kBlock + threadIdx.x) >> lg; r < rows; r += ng) {
    const int64_t e1 = rp[r + 1];
    for (int64_t e = rp[r] + gl; e < e1; e += G) {
      const int32_t q = place[e];
      if (q < 0) continue;   // a column out of range, reported by the count
      const int64_t at = t_rp[col[e]] + q;
      tmp_col[at] = (int32_t)r;
      if (tmp_val) tmp_val[at] = val[e];
    }
  }
}

// Each row of the transpose (a group of 2^lg lanes): every entry goes to the
// number of smaller columns in the row, counted 2^lg columns at a time
// (every lane of the group holds one of them, shared by shuffles inside
// the group; the group's lanes share the row, so they run the same loops).
// Rows longer than kTrLong are listed (longs, counted in *nlong) for
// k_tr_order_long.
__global__ void __launch_bounds__(kBlock) k_tr_order(const int64_t *t_rp, int64_t t_rows, const int32_t *tmp_col,
                                                     const double *tmp_val, int32_t *t_col, double *t_val, int lg,
                                                     int64_t *longs, int64_t *nlong) {
  const int G = 1 << lg;
  const int lane = (int)(threadIdx.x & (kWave - 1));
  const int gl = lane & (G - 1), gbase = lane & ~(G - 1);
  const int64_t ng = (int64_t)gridDim.x * (kBlock >> lg);
  for (int64_t q = (blockIdx.x * (int64_t)kBlock + threadIdx.x) >> lg; q < t_rows; q += ng) {
    const int64_t s = t_rp[q], len = t_rp[q + 1] - s;
    if (len > kTrLong) {
      if (gl == 0) longs[atomicAdd((unsigned long long *)nlong, 1ull)] = q;
      continue;
    }
    for (int64_t i0 = 0; i0 < len; i0 += G) {
      const int64_t i = i0 + gl;
      const int32_t key = i < len ? tmp_col[s + i] : 0x7fffffff;
      int64_t rank = 0;
      for (int64_t j0 = 0; j0 < len; j0 += G) {
        const int32_t other = j0 + gl < len ? tmp_col[s + j0 + gl] : 0x7fffffff;
        const int dn = (int)min((int64_t)G, len - j0);   // the group's lanes holding columns
        for (int d = 0; d < dn; ++d) rank += __shfl(other, gbase + d, kWave) < key ? 1 : 0;
      }
      if (i < len) {
        t_col[s + rank] = key;
        if (t_val) t_val[s + rank] = tmp_val[s + i];
      }
    }
  }
}

// The listed rows of the transpose (longer than kTrLong), one workgroup each: up to
// kTrSortMax entries sorted as (column, source index) pairs by a bitonic
// network in LDS (columns distinct, so the order is unique) and written out;
// a longer row is cut into chunks of kTrSortMax entries, each chunk sorted
// the same way and put back in place in the scratch (columns and values),
// for k_tr_rank_long.
__global__ void __launch_bounds__(kBlock) k_tr_order_long(const int64_t *t_rp, const int64_t *longs,
                                                          const int64_t *nlong, int32_t *tmp_col, double *tmp_val,
                                                          int32_t *t_col, double *t_val) {
  __shared__ int32_t sk[kTrSortMax];
  __shared__ int32_t si[kTrSortMax];
  const int t = threadIdx.x;
  const int64_t nl = *nlong;
  for (int64_t li = blockIdx.x; li < nl; li += gridDim.x) {
    const int64_t q = longs[li];
    const int64_t s0 = t_rp[q], len0 = t_rp[q + 1] - s0;
    for (int64_t c0 = 0; c0 < len0; c0 += kTrSortMax) {
      // the whole row (len0 <= kTrSortMax), or one chunk of a longer row
      const int64_t s = s0 + c0, len = min((int64_t)kTrSortMax, len0 - c0);
      int n = 1;
      while (n < len) n <<= 1;
      for (int i = t; i < n; i += kBlock) {
        sk[i] = i < len ? tmp_col[s + i] : 0x7fffffff;
        si[i] = i;
      }
      __syncthreads();
      for (int k = 2; k <= n; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
          for (int i = t; i < n; i += kBlock) {
            const int p = i ^ j;
            if (p > i) {
              const bool up = (i & k) == 0;
              const int32_t a = sk[i], b = sk[p];
              if ((a > b) == up) {
                sk[i] = b;
                sk[p] = a;
                const int32_t x = si[i];
                si[i] = si[p];
                si[p] = x;
              }
            }
          }
          __syncthreads();
        }
      }
      if (len0 <= kTrSortMax) {
        for (int i = t; i < len; i += kBlock) {
          t_col[s + i] = sk[i];
          if (t_val) t_val[s + i] = tmp_val[s + si[i]];
        }
      } else {
        // the chunk sorted in place: every value read before any is written
        constexpr int kPer = kTrSortMax / kBlock;
        double v[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
          const int i = t + u * kBlock;
          v[u] = (tmp_val && i < len) ? tmp_val[s + si[i]] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
          const int i = t + u * kBlock;
          if (i < len) {
            tmp_col[s + i] = sk[i];
            if (tmp_val) tmp_val[s + i] = v[u];
          }
        }
      }
      __syncthreads();
    }
  }
}

// Rows of the transpose longer than kTrSortMax, their chunks sorted: every
// entry's place in the row is its place in its chunk plus, for every other
// chunk, the number of its columns below the entry's (a binary search; the
// columns of a row are distinct).  All workgroups share each row's entries.
__global__ void __launch_bounds__(kBlock) k_tr_rank_long(const int64_t *t_rp, const int64_t *longs,
                                                         const int64_t *nlong, const int32_t *tmp_col,
                                                         const double *tmp_val, int32_t *t_col, double *t_val) {
  const int64_t nl = *nlong;
  const int64_t tid = (int64_t)blockIdx.x * kBlock + threadIdx.x, nt = (int64_t)gridDim.x * kBlock;
  for (int64_t li = 0; li < nl; ++li) {
    const int64_t q = longs[li];
    const int64_t s = t_rp[q], len = t_rp[q + 1] - s;
    if (len <= kTrSortMax) continue;
    const int64_t nch = (len + kTrSortMax - 1) / kTrSortMax;
    for (int64_t i = tid; i < len; i += nt) {
      const int32_t key = tmp_col[s + i];
      const int64_t mine = i / kTrSortMax;
      int64_t rank = i - mine * kTrSortMax;
      for (int64_t d = 0; d < nch; ++d) {
        if (d == mine) continue;
        int64_t lo = d * kTrSortMax, hi = min(len, lo + kTrSortMax);
        while (lo < hi) {
          const int64_t mid = (lo + hi) >> 1;
          if (tmp_col[s + mid] < key) lo = mid + 1;
          else hi = mid;
        }
        rank += lo - d * kTrSortMax;
      }
      t_col[s + rank] = key;
      if (t_val) t_val[s + rank] = tmp_val[s + i];
    }
  }
}

struct TrLayout {
  size_t cnt, place, tmp_col, tmp_val, status, ctr, longs, total;
};

TrLayout tr_layout(int64_t cols, int64_t nnz) {
  TrLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = (o + std::max<size_t>(bytes, 1) + 255) & ~(size_t)255;
    return at;
  };
  const size_t C = (size_t)std::max<int64_t>(cols, 0), N = (size_t)std::max<int64_t>(nnz, 0);
  L.cnt = take(4 * C);
  L.place = take(4 * N);
  L.tmp_col = take(4 * N);
  L.tmp_val = take(8 * N);
  L.status = take(8 * (C / 2048 + 2));   // scan tiles (at most one per 2048 entries)
  L.ctr = take(8 * 4);                    // error word, scan ticket, scan total, long rows
  L.longs = take(8 * (N / (kTrLong + 1) + 1));   // rows longer than kTrLong, at most
  L.total = o;
  return L;
}

// log2 of the lanes per row: the power of two at least the mean length,
// at most a wave.
int lanes_log2_for(int64_t entries, int64_t rows) {
  const int64_t mean = rows > 0 ? (entries + rows - 1) / rows : 1;
  int lg = 0;
  while ((1 << lg) < mean && lg < 6) ++lg;
  return lg;
}

int grid_for(int64_t work, int per_block) {
  const int64_t b = (work + per_block - 1) / per_block;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, 1 << 16));
}

}  // namespace
}  // namespace spg

using namespace spg;

extern "C" {

size_t spgemm_transpose_scratch(const spgemm_csr *M) {
  if (!M) return 0;
  return tr_layout(M->cols, M->nnz).total;
}

spgemm_status spgemm_transpose(const spgemm_csr *M, int64_t *t_row_ptr, int32_t *t_col, double *t_val,
                               void *scratch, size_t scratch_bytes, void *stream) {
  if (!M || !t_row_ptr || !scratch) return SPGEMM_E_NULL;
  if (M->rows < 0 || M->cols < 0 || M->nnz < 0) return SPGEMM_E_DIM;
  if (!M->row_ptr || (M->nnz > 0 && (!M->col_idx || !t_col)) || (M->nnz > 0 && t_val && !M->val))
    return SPGEMM_E_NULL;
  if (M->rows >= ((int64_t)1 << 31) || M->cols >= ((int64_t)1 << 31)) return SPGEMM_E_INDEX_OVERFLOW;
  const TrLayout L = tr_layout(M->cols, M->nnz);
  if (scratch_bytes < L.total || !aligned256(scratch)) return SPGEMM_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  char *w = static_cast<char *>(scratch);
  int32_t *cnt = reinterpret_cast<int32_t *>(w + L.cnt);
  int32_t *place = reinterpret_cast<int32_t *>(w + L.place);
  int32_t *tmp_col = reinterpret_cast<int32_t *>(w + L.tmp_col);
  double *tmp_val = t_val ? reinterpret_cast<double *>(w + L.tmp_val) : nullptr;
  uint64_t *status = reinterpret_cast<uint64_t *>(w + L.status);
  int64_t *ctr = reinterpret_cast<int64_t *>(w + L.ctr);   // [0] error, [1] ticket, [2] total, [3] long rows
  int64_t *longs = reinterpret_cast<int64_t *>(w + L.longs);
  const int64_t rows = M->rows, cols = M->cols, nnz = M->nnz;
  if (launch_fill_i64(ctr, 0, 4, s) != hipSuccess) return SPGEMM_E_HIP;
  // the row pointers must cover nnz before any row is walked
  hipLaunchKernelGGL(k_tr_check, dim3(1), dim3(kBlock), 0, s, M->row_ptr, rows, nnz, ctr);
  if (hipGetLastError() != hipSuccess) return SPGEMM_E_HIP;
  int64_t herr = 0;
  if (hipMemcpyAsync(&herr, ctr, sizeof(herr), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return SPGEMM_E_HIP;
  if (herr & kTrErrRowPtr) return SPGEMM_E_DIM;
  hipLaunchKernelGGL(k_tr_zero, dim3(grid_for(cols, kBlock)), dim3(kBlock), 0, s, cnt, cols);
  if (nnz > 0)
    hipLaunchKernelGGL(k_tr_count, dim3(grid_for(nnz, kBlock)), dim3(kBlock), 0, s, M->col_idx, nnz, cols, cnt,
                       place, ctr);
  if (hipGetLastError() != hipSuccess) return SPGEMM_E_HIP;
  if (launch_scan_i32(cnt, t_row_ptr, cols, status, ctr + 1, ctr + 2, ctr, s) != hipSuccess) return SPGEMM_E_HIP;
  if (nnz > 0) {
    // the ordering's work grows with the square of a row over its lanes: at
    // least 16 lanes per row there, so that a long row in a matrix of short
    // ones stays cheap
    const int lg_m = lanes_log2_for(nnz, rows), lg_t = std::max(lanes_log2_for(nnz, cols), 4);
    hipLaunchKernelGGL(k_tr_scatter, dim3(grid_for(rows, kBlock >> lg_m)), dim3(kBlock), 0, s, M->row_ptr,
                       M->col_idx, t_val ? M->val : nullptr, rows, (const int64_t *)t_row_ptr, (const int32_t *)place,
                       tmp_col, tmp_val, lg_m);
    hipLaunchKernelGGL(k_tr_order, dim3(grid_for(cols, kBlock >> lg_t)), dim3(kBlock), 0, s,
                       (const int64_t *)t_row_ptr, cols, tmp_col, tmp_val, t_col, t_val, lg_t, longs, ctr + 3);
    hipLaunchKernelGGL(k_tr_order_long, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(nnz / (kTrLong + 1) + 1, 1024))),
                       dim3(kBlock), 0, s, (const int64_t *)t_row_ptr, (const int64_t *)longs, (const int64_t *)(ctr + 3),
                       tmp_col, tmp_val, t_col, t_val);
    // rows longer than one LDS sort: only when M has that many entries
    if (nnz > kTrSortMax)
      hipLaunchKernelGGL(k_tr_rank_long, dim3((unsigned)grid_for(nnz, kBlock)), dim3(kBlock), 0, s,
                         (const int64_t *)t_row_ptr, (const int64_t *)longs, (const int64_t *)(ctr + 3), tmp_col,
                         tmp_val, t_col, t_val);
  }
  if (hipGetLastError() != hipSuccess) return SPGEMM_E_HIP;
  if (hipMemcpyAsync(&herr, ctr, sizeof(herr), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return SPGEMM_E_HIP;
  if (herr & kTrErrRange) return SPGEMM_E_NOT_CANONICAL;
  if (herr) return SPGEMM_E_STATE;
  return SPGEMM_OK;
}

}  // extern "C"
