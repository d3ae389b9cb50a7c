// Learned row-size network: inference and training kernels (FP32).
//
// Not part of the paper.  The paper sizes C from the multiplication count,
// an estimate that never underestimates (Section IV-B), and decides per row
// between two storing strategies with a quick rule (Section IV-B, the
// "Combined" kernel), noting that the decision criterion could be improved
// (Section VI).  Here a 3-32-32-1 perceptron predicts where nnz(C_row) falls
// between the longest selected B row and the multiplication count; the
// prediction sizes each row's accumulator and the output.
//
// Parameter layout (1217 floats): W1[32][3], b1[32], W2[32][32], b2[32],
// w3[32], b3.  Device parameter block: theta, then mu[3], sd[3].
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../../include/spgemm.h"
#include "device_common.h"
#include "spgemm_internal.h"
#include "spgemm_kernels.h"

namespace spg {

constexpr int H = kMlpHidden;
constexpr int OW1 = 0, OB1 = OW1 + H * 3, OW2 = OB1 + H, OB2 = OW2 + H * H, OW3 = OB2 + H, OB3 = OW3 + H;
static_assert(OB3 + 1 == kMlpParams, "parameter layout");

__device__ __forceinline__ void mlp_inputs(const float *mu, const float *sd, int32_t f1, int32_t f2, int32_t f3,
                                           float x[3]) {
  x[0] = (log2f(1.0f + (float)f1) - mu[0]) / sd[0];
  x[1] = (log2f(1.0f + (float)f2) - mu[1]) / sd[1];
  x[2] = (log2f(1.0f + (float)f3) - mu[2]) / sd[2];
}

__device__ __forceinline__ float logistic(float z) { return 1.0f / (1.0f + expf(-z)); }

// Forward pass of one sample.  P: parameters (uniform across the wave, so
// the compiler reads them through the scalar cache).
__device__ __forceinline__ float mlp_forward(const float *__restrict__ P, const float x[3]) {
  float h1[H];
#pragma unroll
  for (int j = 0; j < H; ++j) {
    float a = P[OB1 + j];
    a = fmaf(P[OW1 + 3 * j + 0], x[0], a);
    a = fmaf(P[OW1 + 3 * j + 1], x[1], a);
    a = fmaf(P[OW1 + 3 * j + 2], x[2], a);
    h1[j] = fmaxf(a, 0.0f);
  }
  float z = P[OB3];
#pragma unroll
  for (int j = 0; j < H; ++j) {
    float a = P[OB2 + j];
#pragma unroll
    for (int i = 0; i < H; ++i) a = fmaf(P[OW2 + H * j + i], h1[i], a);
    z = fmaf(P[OW3 + j], fmaxf(a, 0.0f), z);
  }
  return z;
}

__device__ __forceinline__ float predict_one(const float *__restrict__ dev, int32_t f1, int32_t f2, int32_t f3) {
  float x[3];
  mlp_inputs(dev + kMlpParams, dev + kMlpParams + 3, f1, f2, f3, x);
  float rho = logistic(mlp_forward(dev, x));
  return (float)f3 + rho * (float)(f2 - f3);
}

// The same prediction computed by a half-wave of 32 lanes: lane j owns
// hidden unit j of both layers.  W (LDS) holds the device parameter block;
// hbuf (LDS, 32 floats per half-wave) passes the first layer across lanes.
// Every lane of the half-wave returns the prediction.
__device__ __forceinline__ float predict_coop(const float *W, float *hbuf, int32_t f1, int32_t f2, int32_t f3) {
  const int j = lane_id() & 31;
  float x[3];
  mlp_inputs(W + kMlpParams, W + kMlpParams + 3, f1, f2, f3, x);
  float a1 = W[OB1 + j];
  a1 = fmaf(W[OW1 + 3 * j + 0], x[0], a1);
  a1 = fmaf(W[OW1 + 3 * j + 1], x[1], a1);
  a1 = fmaf(W[OW1 + 3 * j + 2], x[2], a1);
  hbuf[j] = fmaxf(a1, 0.0f);
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  float a2 = W[OB2 + j];
#pragma unroll 8
  for (int i = 0; i < H; ++i) a2 = fmaf(W[OW2 + H * j + i], hbuf[i], a2);
  float z = W[OW3 + j] * fmaxf(a2, 0.0f);
#pragma unroll
  for (int d = 16; d > 0; d >>= 1) z += __shfl_xor(z, d, 32);
  z += W[OB3];
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  const float rho = logistic(z);
  return (float)f3 + rho * (float)(f2 - f3);
}

// ---------------------------------------------------------------- predict
// Rows with the same feature triple get the same prediction, and sparse
// matrices repeat triples heavily (a stencil has a handful).  Each
// workgroup collects the distinct triples of its 2048 rows in an LDS hash,
// evaluates the network once per distinct triple (one per lane), and hands
// the results back to the rows.
// Rows per thread: four for the per-row arrays; one where the features
// are gathered from the operands (their gathers are not overlapped across
// a thread's rows, so more workgroups hide them better).
template <bool FEAT>
struct PredShape {
  static constexpr int kRowsPerThread = FEAT ? 2 : 4;
  static constexpr int kRows = kBlock * kRowsPerThread;
  static constexpr int kTab = 2 * kRows;
};
constexpr uint64_t kNoKey = 1ull << 63;

__device__ __forceinline__ uint64_t triple_key(int32_t f1, int32_t f2, int32_t f3) {
  if ((uint32_t)f1 >= (1u << 21) || (uint32_t)f2 >= (1u << 22) || (uint32_t)f3 >= (1u << 20)) return kNoKey;
  return (uint64_t)f1 | ((uint64_t)f2 << 21) | ((uint64_t)f3 << 43);
}

__device__ __forceinline__ uint32_t triple_hash(uint64_t k, int tab) {
  k ^= k >> 29;
  k *= 0xbf58476d1ce4e5b9ull;
  k ^= k >> 32;
  return (uint32_t)k & (uint32_t)(tab - 1);
}

// KEYS: the rows' packed feature triples come from `keys` (written by the
// feature kernel; all ones when a field did not fit) and only
// per-workgroup partial sums of the learned capacity are written.
// Otherwise the features come from the per-row arrays and the prediction
// of every row is stored.
// FEAT: the rows' feature triples are computed here from the operands (no
// per-row arrays), only capacity sums are kept, and partials get kCapParts
// words per workgroup: the summed capacities, their largest sum over 64
// consecutive rows (a merge wave's rows), the multiplication count, the
// longest row of A, the empty rows, and the summed bounds of the rows whose
// triple does not pack (sized by their bound by the caller).  Otherwise the
// features come from the per-row arrays and every row's prediction is stored.
constexpr int kCapParts = 6;

// gate (FEAT, may be null): the longest row of A, already summed; when it
// exceeds gate_max the product takes the tiled path, which predicts its
// rows' sizes there, and every workgroup only passes the longest row on.
template <bool FEAT>
__global__ void __launch_bounds__(kBlock) k_mlp_predict(const float *__restrict__ dev, Operands op,
                                                        const int32_t *f1a, const int32_t *f2a, const int32_t *f3a,
                                                        int64_t n, float *pred, float margin, int slack,
                                                        int64_t *partials, int64_t *err, const int64_t *gate,
                                                        int64_t gate_max) {
  if (FEAT && gate && *gate > gate_max) {
    if (partials && threadIdx.x < kCapParts)
      partials[kCapParts * blockIdx.x + threadIdx.x] = threadIdx.x == 3 ? *gate : 0;
    return;
  }
  constexpr int kPredRowsPerThread = PredShape<FEAT>::kRowsPerThread;
  constexpr int kPredRows = PredShape<FEAT>::kRows;
  constexpr int kPredTab = PredShape<FEAT>::kTab;
  __shared__ unsigned long long keys[kPredTab];
  __shared__ int32_t slot_idx[kPredTab];
  __shared__ uint64_t ukey[kPredRows];
  __shared__ float upred[kPredRows];
  __shared__ int64_t wtot[kWavesPerBlock + 1];
  __shared__ float W[kMlpDevFloats];
  __shared__ float hbuf[kBlock / 32][32];
  for (int s = threadIdx.x; s < kPredTab; s += kBlock) keys[s] = kNoKey;
  for (int s = threadIdx.x; s < kMlpDevFloats; s += kBlock) W[s] = dev[s];
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kPredRows;
  uint64_t mine[kPredRowsPerThread];
  int64_t mults = 0, max_a = 0, empty = 0, unpacked = 0;
  if (FEAT && blockIdx.x == 0 && threadIdx.x == 0 &&
      (op.a_rp[op.rows] != op.a_nnz || op.b_rp[op.b_rows] != op.b_nnz))
    atomicOr((unsigned long long *)err, (unsigned long long)kErrDescriptor);
#pragma unroll
  for (int j = 0; j < kPredRowsPerThread; ++j) {
    const int64_t r = base + j * kBlock + threadIdx.x;
    mine[j] = kNoKey;
    if (FEAT) {
      // every lane takes part: long rows are walked by the whole wave
      int64_t m, ub;
      int32_t mx, lo, hi;
      wave_row_features<false>(op, r, r < n, m, ub, mx, lo, hi);
      if (r < n) {
        const int64_t u = min(ub, (int64_t)op.b_cols);
        mine[j] = triple_key((int32_t)min(m, (int64_t)0x7fffffff), (int32_t)u, mx);
        if (mine[j] == kNoKey) unpacked += u;
        mults += ub;
        max_a = max(max_a, m);
        empty += ub == 0 ? 1 : 0;
      }
    } else if (r < n) {
      mine[j] = triple_key(f1a[r], f2a[r], f3a[r]);
    }
  }
#pragma unroll
  for (int j = 0; j < kPredRowsPerThread; ++j) {
    // one insertion per distinct triple per wave: the lowest lane holding a
    // triple inserts it for every lane that holds the same one (rows of a
    // stencil share a handful of triples; contended atomics on one LDS slot
    // would serialise them)
    uint64_t pending = __ballot(mine[j] != kNoKey);
    while (pending) {
      const int leader = __ffsll((unsigned long long)pending) - 1;
      const uint64_t lk = __shfl(mine[j], leader, kWave);
      const uint64_t same = __ballot(mine[j] == lk);
      if (lane_id() == leader) {
        uint32_t s = triple_hash(lk, kPredTab);
        while (true) {
          unsigned long long cur = keys[s];
          if (cur == lk) break;
          if (cur == kNoKey) {
            unsigned long long old = atomicCAS(&keys[s], (unsigned long long)kNoKey, (unsigned long long)lk);
            if (old == kNoKey || old == lk) break;
          }
          s = (s + 1) & (kPredTab - 1);
        }
      }
      pending &= ~same;
    }
  }
  __syncthreads();
  // compact the distinct triples
  constexpr int kPer = kPredTab / kBlock;
  int64_t cnt = 0;
#pragma unroll
  for (int q = 0; q < kPer; ++q) cnt += keys[threadIdx.x * kPer + q] != kNoKey ? 1 : 0;
  int64_t total;
  int64_t at = block_exclusive_sum(cnt, wtot, &total);
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    int s = threadIdx.x * kPer + q;
    if (keys[s] != kNoKey) {
      slot_idx[s] = (int32_t)at;
      ukey[at] = keys[s];
      ++at;
    }
  }
  __syncthreads();
  // distinct triples, one per half-wave at a time (uniform trip count per
  // half-wave, so every lane of it takes part in every shuffle)
  const int half = threadIdx.x / 32;
  for (int u0 = 0; u0 < total; u0 += kBlock / 32) {
    const int u = u0 + half;
    if (u < total) {
      const uint64_t k = ukey[u];
      const int32_t a = (int32_t)(k & ((1u << 21) - 1));
      const int32_t b = (int32_t)((k >> 21) & ((1u << 22) - 1));
      const int32_t c = (int32_t)(k >> 43);
      float pr = predict_coop(W, hbuf[half], a, b, c);
      // finite weights can still overflow to a NaN: such a row is sized by
      // its bound, which never underestimates
      if (!(pr >= (float)c && pr <= (float)b)) pr = (float)b;
      if ((threadIdx.x & 31) == 0) upred[u] = pr;
    }
  }
  __syncthreads();
  int64_t capsum = 0, wave_cap = 0;
#pragma unroll
  for (int j = 0; j < kPredRowsPerThread; ++j) {
    const int64_t r = base + j * kBlock + threadIdx.x;
    int64_t rc = 0;   // this row's capacity
    if (r < n) {
      const uint64_t k = mine[j];
      float p;
      int32_t b, c;
      if (k == kNoKey) {
        // features too large to pack: the row is sized by its bound (its
        // multiplication count) instead of a prediction
        if (FEAT) {
          p = -1.0f;
          b = c = 0;
        } else {
          b = f2a[r];
          c = f3a[r];
          p = (float)b;
        }
      } else {
        uint32_t s = triple_hash(k, kPredTab);
        while (keys[s] != k) s = (s + 1) & (kPredTab - 1);
        p = upred[slot_idx[s]];
        b = (int32_t)((k >> 21) & ((1u << 22) - 1));
        c = (int32_t)(k >> 43);
      }
      if (!FEAT) pred[r] = p;
      if (p >= 0.0f) rc = learned_capacity(p, b, c, margin, slack);
    }
    capsum += rc;
    // rows base + j * kBlock + 64w .. + 63 are one merge wave's rows
    if (FEAT) wave_cap = max(wave_cap, wave_sum(rc));
  }
  if (!partials) return;
  if (FEAT) {
    __shared__ int64_t s_part[kCapParts][kWavesPerBlock];
    int64_t v[kCapParts] = {wave_sum(capsum), wave_cap, wave_sum(mults), wave_max64(max_a), wave_sum(empty),
                            wave_sum(unpacked)};
    if (lane_id() == 0)
      for (int q = 0; q < kCapParts; ++q) s_part[q][threadIdx.x / kWave] = v[q];
    __syncthreads();
    if (threadIdx.x < kCapParts) {
      const int q = threadIdx.x;
      const bool is_max = q == 1 || q == 3;
      int64_t t = 0;
      for (int w = 0; w < kWavesPerBlock; ++w) t = is_max ? max(t, s_part[q][w]) : t + s_part[q][w];
      partials[kCapParts * blockIdx.x + q] = t;
    }
  } else {
    int64_t tot;
    block_exclusive_sum(capsum, wtot, &tot);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
  }
}

int64_t mlp_predict_blocks(int64_t n) { return (n + PredShape<false>::kRows - 1) / PredShape<false>::kRows; }

hipError_t launch_mlp_predict(const float *dev, const int32_t *f1, const int32_t *f2, const int32_t *f3,
                              int64_t n, float *pred, hipStream_t s, float margin, int slack,
                              int64_t *partials) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = mlp_predict_blocks(n);
  hipLaunchKernelGGL(k_mlp_predict<false>, dim3((unsigned)blocks), dim3(kBlock), 0, s, dev, Operands{}, f1, f2, f3, n,
                     pred, margin, slack, partials, (int64_t *)nullptr, (const int64_t *)nullptr, (int64_t)0);
  return hipGetLastError();
}

hipError_t launch_mlp_capacity(const float *dev, const Operands &op, int64_t *counters, int64_t *partials,
                               float margin, int slack, hipStream_t s, const int64_t *gate, int64_t gate_max) {
  const int32_t dst[kCapParts] = {kCtrCapSum, kCtrWaveCap, kCtrMults, kCtrMaxA, kCtrEmpty, kCtrUnpacked};
  const int32_t mx[kCapParts] = {0, 1, 0, 1, 0, 0};
  if (op.rows <= 0) {
    for (int q = 0; q < kCapParts; ++q) {
      hipError_t e = launch_fill_i64(counters + dst[q], 0, 1, s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  const int64_t blocks = (op.rows + PredShape<true>::kRows - 1) / PredShape<true>::kRows;
  hipLaunchKernelGGL(k_mlp_predict<true>, dim3((unsigned)blocks), dim3(kBlock), 0, s, dev, op,
                     (const int32_t *)nullptr, (const int32_t *)nullptr, (const int32_t *)nullptr, op.rows,
                     (float *)nullptr, margin, slack, partials, counters + kCtrError, gate, gate_max);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_sum_partials(partials, blocks, kCapParts, kCapParts, dst, mx, counters, s);
}

// --------------------------------------------------------------- gradient
// One workgroup, 256 samples: forward, backward through the logistic and
// both ReLU layers, and the per-workgroup sums of the parameter gradients
// (outer products reduced over the samples in LDS).  Writes kMlpParams + 2
// floats per workgroup: the unnormalised gradient sums, the weighted squared
// error sum and the weight sum.  A second kernel adds the workgroups in
// order and divides by the total weight, so results do not depend on timing.
constexpr int kPartial = kMlpParams + 2;

__global__ void __launch_bounds__(kBlock) k_mlp_grad_partial(const float *__restrict__ dev,
                                                             const int32_t *f1, const int32_t *f2,
                                                             const int32_t *f3, const int32_t *lab,
                                                             int64_t n0, int64_t n1, float *partial) {
  __shared__ float hs[kBlock][H + 1];
  __shared__ float ds[kBlock][H + 1];
  __shared__ float red[2][kWavesPerBlock];
  const float *__restrict__ P = dev;
  const int64_t s_idx = n0 + (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool valid = s_idx < n1;
  float x[3] = {0.f, 0.f, 0.f};
  float t = 0.f, w = 0.f;
  if (valid) {
    int32_t a = f1[s_idx], b = f2[s_idx], c = f3[s_idx];
    mlp_inputs(dev + kMlpParams, dev + kMlpParams + 3, a, b, c, x);
    if (b > c) {
      w = 1.f;
      t = (float)(lab[s_idx] - c) / (float)(b - c);
    }
  }
  float a1[H], h1[H], h2[H];
  uint32_t m2 = 0;
#pragma unroll
  for (int j = 0; j < H; ++j) {
    float a = P[OB1 + j];
    a = fmaf(P[OW1 + 3 * j + 0], x[0], a);
    a = fmaf(P[OW1 + 3 * j + 1], x[1], a);
    a = fmaf(P[OW1 + 3 * j + 2], x[2], a);
    a1[j] = a;
    h1[j] = fmaxf(a, 0.f);
  }
  float z = P[OB3];
#pragma unroll
  for (int j = 0; j < H; ++j) {
    float a = P[OB2 + j];
#pragma unroll
    for (int i = 0; i < H; ++i) a = fmaf(P[OW2 + H * j + i], h1[i], a);
    if (a > 0.f) m2 |= 1u << j;
    h2[j] = fmaxf(a, 0.f);
    z = fmaf(P[OW3 + j], h2[j], z);
  }
  const float rho = logistic(z);
  const float err = rho - t;
  const float d3 = valid ? 2.f * w * err * rho * (1.f - rho) : 0.f;
  float d2[H];
#pragma unroll
  for (int j = 0; j < H; ++j) d2[j] = ((m2 >> j) & 1u) ? d3 * P[OW3 + j] : 0.f;
  float d1[H];
#pragma unroll
  for (int i = 0; i < H; ++i) {
    float acc = 0.f;
#pragma unroll
    for (int j = 0; j < H; ++j) acc = fmaf(P[OW2 + H * j + i], d2[j], acc);
    d1[i] = a1[i] > 0.f ? acc : 0.f;
  }
  float *out = partial + (size_t)blockIdx.x * kPartial;

  // W2, b2: sum_s d2[s][j] * h1[s][i]
#pragma unroll
  for (int j = 0; j < H; ++j) {
    hs[threadIdx.x][j] = h1[j];
    ds[threadIdx.x][j] = d2[j];
  }
  __syncthreads();
  {
    const int j = threadIdx.x >> 3, i0 = (threadIdx.x & 7) * 4;
    float g0 = 0.f, g1 = 0.f, g2 = 0.f, g3 = 0.f, gb = 0.f;
    for (int s = 0; s < kBlock; ++s) {
      float d = ds[s][j];
      g0 = fmaf(d, hs[s][i0 + 0], g0);
      g1 = fmaf(d, hs[s][i0 + 1], g1);
      g2 = fmaf(d, hs[s][i0 + 2], g2);
      g3 = fmaf(d, hs[s][i0 + 3], g3);
      gb += d;
    }
    out[OW2 + H * j + i0 + 0] = g0;
    out[OW2 + H * j + i0 + 1] = g1;
    out[OW2 + H * j + i0 + 2] = g2;
    out[OW2 + H * j + i0 + 3] = g3;
    if (i0 == 0) out[OB2 + j] = gb;
  }
  __syncthreads();
  // w3, b3 (d3 * h2) and W1, b1 (d1 * x)
#pragma unroll
  for (int j = 0; j < H; ++j) {
    hs[threadIdx.x][j] = h2[j];
    ds[threadIdx.x][j] = d1[j];
  }
  hs[threadIdx.x][H] = d3;
  __syncthreads();
  if (threadIdx.x < H) {
    const int j = threadIdx.x;
    float g = 0.f;
    for (int s = 0; s < kBlock; ++s) g = fmaf(hs[s][H], hs[s][j], g);
    out[OW3 + j] = g;
  } else if (threadIdx.x == H) {
    float g = 0.f;
    for (int s = 0; s < kBlock; ++s) g += hs[s][H];
    out[OB3] = g;
  }
  __syncthreads();
  // x into hs columns 0..2 (d1 stays in ds)
  hs[threadIdx.x][0] = x[0];
  hs[threadIdx.x][1] = x[1];
  hs[threadIdx.x][2] = x[2];
  __syncthreads();
  if (threadIdx.x < H * 4) {
    const int j = threadIdx.x >> 2, m = threadIdx.x & 3;
    float g = 0.f;
    if (m < 3) {
      for (int s = 0; s < kBlock; ++s) g = fmaf(ds[s][j], hs[s][m], g);
      out[OW1 + 3 * j + m] = g;
    } else {
      for (int s = 0; s < kBlock; ++s) g += ds[s][j];
      out[OB1 + j] = g;
    }
  }
  // loss numerator and weight sum
  float le = valid ? w * err * err : 0.f, lw = valid ? w : 0.f;
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) {
    le += __shfl_xor(le, d, kWave);
    lw += __shfl_xor(lw, d, kWave);
  }
  if (lane_id() == 0) {
    red[0][threadIdx.x / kWave] = le;
    red[1][threadIdx.x / kWave] = lw;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float a = 0.f, b = 0.f;
    for (int q = 0; q < kWavesPerBlock; ++q) {
      a += red[0][q];
      b += red[1][q];
    }
    out[kMlpParams] = a;
    out[kMlpParams + 1] = b;
  }
}

// grad[k] = sum_b partial[b][k] / W, loss = sum_b err_b / W (in block order)
__global__ void k_mlp_reduce(const float *partial, int nblocks, float *grad, float *loss) {
  int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= kPartial) return;
  float wsum = 0.f;
  for (int b = 0; b < nblocks; ++b) wsum += partial[(size_t)b * kPartial + kMlpParams + 1];
  float g = 0.f;
  for (int b = 0; b < nblocks; ++b) g += partial[(size_t)b * kPartial + k];
  float inv = wsum > 0.f ? 1.f / wsum : 0.f;
  if (k < kMlpParams) grad[k] = g * inv;
  else if (k == kMlpParams && loss) *loss = g * inv;
}

// Adam (Kingma and Ba, Algorithm 1), one parameter per thread.
__global__ void k_mlp_adam(float *theta, float *m, float *v, const float *grad, float lr, float b1, float b2,
                           float eps, float c1, float c2) {
  int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= kMlpParams) return;
  float g = grad[k];
  float mk = b1 * m[k] + (1.f - b1) * g;
  float vk = b2 * v[k] + (1.f - b2) * g * g;
  m[k] = mk;
  v[k] = vk;
  float mh = mk / c1, vh = vk / c2;
  theta[k] -= lr * mh / (sqrtf(vh) + eps);
}

// ---------------------------------------------------------- feature stats
// Per-workgroup sums (double) of log2(1 + f) and its square for the three
// features, then an in-order reduction.
__global__ void k_stats_partial(const int32_t *f1, const int32_t *f2, const int32_t *f3, int64_t n,
                                double *partial) {
  __shared__ double red[6][kWavesPerBlock];
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x; r < n; r += (int64_t)gridDim.x * kBlock) {
    double a = log2(1.0 + (double)f1[r]), b = log2(1.0 + (double)f2[r]), c = log2(1.0 + (double)f3[r]);
    acc[0] += a;
    acc[1] += a * a;
    acc[2] += b;
    acc[3] += b * b;
    acc[4] += c;
    acc[5] += c * c;
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    double t = acc[q];
    for (int d = kWave / 2; d > 0; d >>= 1) t += __shfl_xor(t, d, kWave);
    if (lane_id() == 0) red[q][threadIdx.x / kWave] = t;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    double t = 0;
    for (int w = 0; w < kWavesPerBlock; ++w) t += red[threadIdx.x][w];
    partial[(size_t)blockIdx.x * 6 + threadIdx.x] = t;
  }
}

__global__ void k_stats_final(const double *partial, int nblocks, int64_t n, float *musd) {
  if (threadIdx.x >= 3) return;
  double s = 0, ss = 0;
  for (int b = 0; b < nblocks; ++b) {
    s += partial[(size_t)b * 6 + 2 * threadIdx.x];
    ss += partial[(size_t)b * 6 + 2 * threadIdx.x + 1];
  }
  double mu = n > 0 ? s / (double)n : 0.0;
  double var = n > 0 ? ss / (double)n - mu * mu : 0.0;
  double sd = var > 1e-12 ? sqrt(var) : 1.0;
  musd[threadIdx.x] = (float)mu;
  musd[3 + threadIdx.x] = (float)sd;
}

__global__ void k_zero_f32(float *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) p[i] = 0.f;
}

__global__ void k_features_only(const int64_t *a_rp, const int32_t *a_col, const int64_t *b_rp, int64_t rows,
                                int64_t b_cols, int32_t *f1, int32_t *f2, int32_t *f3) {
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= rows) return;
  int64_t s = a_rp[i], e = a_rp[i + 1];
  int64_t ub = 0;
  int32_t mx = 0;
  for (int64_t q = s; q < e; ++q) {
    int32_t k = a_col[q];
    int32_t len = (int32_t)(b_rp[k + 1] - b_rp[k]);
    ub += len;
    mx = max(mx, len);
  }
  f1[i] = (int32_t)(e - s);
  f2[i] = (int32_t)min(ub, b_cols);
  f3[i] = mx;
}

}  // namespace spg

using namespace spg;

static size_t grad_partial_bytes(int64_t n) {
  int64_t blocks = (n + kBlock - 1) / kBlock;
  return (size_t)std::max<int64_t>(blocks, 1) * kPartial * sizeof(float);
}

extern "C" {

spgemm_status spgemm_model_create(const float *theta, const float *mu, const float *sd, spgemm_model **out) {
  if (!theta || !mu || !sd || !out) return SPGEMM_E_NULL;
  // a model whose parameters are not finite (or whose scales are not
  // positive) would predict NaN: refused, whether it comes from the caller,
  // a file or a training run that diverged
  for (int i = 0; i < kMlpParams; ++i)
    if (!std::isfinite(theta[i])) return SPGEMM_E_INVALID;
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(mu[i]) || !std::isfinite(sd[i]) || !(sd[i] > 0.0f)) return SPGEMM_E_INVALID;
  spgemm_model *m = (spgemm_model *)malloc(sizeof(spgemm_model));
  if (!m) return SPGEMM_E_INVALID;
  memcpy(m->theta, theta, sizeof(m->theta));
  memcpy(m->mu, mu, sizeof(m->mu));
  memcpy(m->sd, sd, sizeof(m->sd));
  *out = m;
  return SPGEMM_OK;
}

spgemm_status spgemm_model_get(const spgemm_model *m, float *theta, float *mu, float *sd) {
  if (!m) return SPGEMM_E_NULL;
  if (theta) memcpy(theta, m->theta, sizeof(m->theta));
  if (mu) memcpy(mu, m->mu, sizeof(m->mu));
  if (sd) memcpy(sd, m->sd, sizeof(m->sd));
  return SPGEMM_OK;
}

void spgemm_model_destroy(spgemm_model *m) { free(m); }

// File format: 8-byte magic "SPGMLP01", int32 parameter count, then
// theta, mu, sd as little-endian float32.
spgemm_status spgemm_model_save(const spgemm_model *m, const char *path) {
  if (!m || !path) return SPGEMM_E_NULL;
  FILE *f = fopen(path, "wb");
  if (!f) return SPGEMM_E_IO;
  int32_t np = kMlpParams;
  bool ok = fwrite("SPGMLP01", 1, 8, f) == 8 && fwrite(&np, 4, 1, f) == 1 &&
            fwrite(m->theta, 4, kMlpParams, f) == (size_t)kMlpParams && fwrite(m->mu, 4, 3, f) == 3 &&
            fwrite(m->sd, 4, 3, f) == 3;
  ok = (fclose(f) == 0) && ok;
  return ok ? SPGEMM_OK : SPGEMM_E_IO;
}

spgemm_status spgemm_model_load(const char *path, spgemm_model **out) {
  if (!path || !out) return SPGEMM_E_NULL;
  FILE *f = fopen(path, "rb");
  if (!f) return SPGEMM_E_IO;
  char magic[8];
  int32_t np = 0;
  spgemm_model tmp;
  bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, "SPGMLP01", 8) == 0 && fread(&np, 4, 1, f) == 1 &&
            np == kMlpParams && fread(tmp.theta, 4, kMlpParams, f) == (size_t)kMlpParams &&
            fread(tmp.mu, 4, 3, f) == 3 && fread(tmp.sd, 4, 3, f) == 3;
  fclose(f);
  if (!ok) return SPGEMM_E_IO;
  return spgemm_model_create(tmp.theta, tmp.mu, tmp.sd, out);
}

size_t spgemm_model_device_bytes(void) { return sizeof(float) * kMlpDevFloats; }

spgemm_status spgemm_model_upload(const spgemm_model *m, void *dev_params, void *stream) {
  if (!m || !dev_params) return SPGEMM_E_NULL;
  float host[kMlpDevFloats];
  memcpy(host, m->theta, sizeof(m->theta));
  memcpy(host + kMlpParams, m->mu, sizeof(m->mu));
  memcpy(host + kMlpParams + 3, m->sd, sizeof(m->sd));
  if (hipMemcpyAsync(dev_params, host, sizeof(host), hipMemcpyHostToDevice, (hipStream_t)stream) != hipSuccess)
    return SPGEMM_E_HIP;
  // the host staging array leaves scope: make sure the copy has consumed it
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return SPGEMM_E_HIP;
  return SPGEMM_OK;
}

spgemm_status spgemm_row_features(const spgemm_csr *A, const spgemm_csr *B, int32_t *f_nnz_a, int32_t *f_ub,
                                  int32_t *f_maxb, void *stream) {
  if (!A || !B || !f_nnz_a || !f_ub || !f_maxb) return SPGEMM_E_NULL;
  if (A->cols != B->rows) return SPGEMM_E_DIM;
  if (A->rows <= 0) return SPGEMM_OK;
  hipLaunchKernelGGL(k_features_only, dim3((unsigned)((A->rows + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     (hipStream_t)stream, A->row_ptr, A->col_idx, B->row_ptr, A->rows, B->cols, f_nnz_a, f_ub,
                     f_maxb);
  return hipGetLastError() == hipSuccess ? SPGEMM_OK : SPGEMM_E_HIP;
}

size_t spgemm_model_stats_scratch(int64_t n) {
  (void)n;
  return 1024 * 6 * sizeof(double) + 256;
}

spgemm_status spgemm_model_feature_stats(const int32_t *f1, const int32_t *f2, const int32_t *f3, int64_t n,
                                         float *mu, float *sd, void *scratch, void *stream) {
  if (!f1 || !f2 || !f3 || !mu || !sd || !scratch) return SPGEMM_E_NULL;
  hipStream_t s = (hipStream_t)stream;
  int blocks = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n + kBlock - 1) / kBlock));
  double *partial = (double *)scratch;
  float *musd = (float *)((char *)scratch + 1024 * 6 * sizeof(double));
  hipLaunchKernelGGL(k_stats_partial, dim3(blocks), dim3(kBlock), 0, s, f1, f2, f3, n, partial);
  hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(64), 0, s, (const double *)partial, blocks, n, musd);
  float host[6];
  if (hipMemcpyAsync(host, musd, sizeof(host), hipMemcpyDeviceToHost, s) != hipSuccess) return SPGEMM_E_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return SPGEMM_E_HIP;
  memcpy(mu, host, 3 * sizeof(float));
  memcpy(sd, host + 3, 3 * sizeof(float));
  return SPGEMM_OK;
}

size_t spgemm_model_grad_scratch(int64_t n) {
  return 256 + sizeof(float) * kMlpDevFloats + grad_partial_bytes(n) + 256;
}

spgemm_status spgemm_model_loss_grad(const spgemm_model *m, const int32_t *f1, const int32_t *f2,
                                     const int32_t *f3, const int32_t *nnz_c, int64_t n, float *grad,
                                     void *scratch, float *loss, void *stream) {
  if (!m || !f1 || !f2 || !f3 || !nnz_c || !grad || !scratch || !loss) return SPGEMM_E_NULL;
  if (n <= 0) return SPGEMM_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  float *dev = (float *)scratch;
  float *dloss = (float *)((char *)scratch + sizeof(float) * kMlpDevFloats);
  float *partial = (float *)((char *)scratch + 256 + sizeof(float) * kMlpDevFloats);
  spgemm_status st = spgemm_model_upload(m, dev, stream);
  if (st != SPGEMM_OK) return st;
  int blocks = (int)((n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_mlp_grad_partial, dim3(blocks), dim3(kBlock), 0, s, (const float *)dev, f1, f2, f3, nnz_c,
                     (int64_t)0, n, partial);
  hipLaunchKernelGGL(k_mlp_reduce, dim3((kPartial + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
                     (const float *)partial, blocks, grad, dloss);
  if (hipGetLastError() != hipSuccess) return SPGEMM_E_HIP;
  if (hipMemcpyAsync(loss, dloss, sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess) return SPGEMM_E_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return SPGEMM_E_HIP;
  return SPGEMM_OK;
}

size_t spgemm_model_train_scratch(int64_t n, int32_t batch_size) {
  (void)n;
  size_t per = grad_partial_bytes(batch_size > 0 ? batch_size : 1);
  return sizeof(float) * kMlpDevFloats + 3 * sizeof(float) * 1280 + per + 256;
}

spgemm_status spgemm_model_train(const float *theta0, const float *mu, const float *sd, const int32_t *f1,
                                 const int32_t *f2, const int32_t *f3, const int32_t *nnz_c, int64_t n,
                                 const spgemm_train_params *hp, void *scratch, size_t scratch_bytes,
                                 float *loss_curve, spgemm_model **out, void *stream) {
  if (!theta0 || !mu || !sd || !f1 || !f2 || !f3 || !nnz_c || !hp || !scratch || !out) return SPGEMM_E_NULL;
  if (n <= 0 || hp->epochs <= 0 || hp->batch_size <= 0 || hp->lr <= 0) return SPGEMM_E_INVALID;
  if (scratch_bytes < spgemm_model_train_scratch(n, hp->batch_size)) return SPGEMM_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  char *base = (char *)scratch;
  float *dev = (float *)base;                                   // theta | mu | sd
  float *mom = (float *)(base + sizeof(float) * kMlpDevFloats);  // m
  float *vel = mom + 1280;                                      // v
  float *grad = vel + 1280;
  float *partial = grad + 1280;
  const int64_t nb = (n + hp->batch_size - 1) / hp->batch_size;
  const int64_t steps = nb * hp->epochs;
  // per-step losses go after the partials
  spgemm_model init;
  memcpy(init.theta, theta0, sizeof(init.theta));
  memcpy(init.mu, mu, sizeof(init.mu));
  memcpy(init.sd, sd, sizeof(init.sd));
  spgemm_status st = spgemm_model_upload(&init, dev, stream);
  if (st != SPGEMM_OK) return st;
  hipLaunchKernelGGL(k_zero_f32, dim3(10), dim3(kBlock), 0, s, mom, (int64_t)1280 * 2);
  std::vector<float> losses((size_t)hp->epochs, 0.f);
  float *dloss_step = nullptr;
  // loss of each step: a device float we read back once per epoch
  float *dl = grad + kMlpParams;   // spare floats after the gradient
  double b1t = 1.0, b2t = 1.0;
  for (int ep = 0; ep < hp->epochs; ++ep) {
    double ep_loss = 0.0;
    for (int64_t b = 0; b < nb; ++b) {
      int64_t n0 = b * hp->batch_size, n1 = std::min<int64_t>(n, n0 + hp->batch_size);
      int blocks = (int)((n1 - n0 + kBlock - 1) / kBlock);
      hipLaunchKernelGGL(k_mlp_grad_partial, dim3(blocks), dim3(kBlock), 0, s, (const float *)dev, f1, f2, f3,
                         nnz_c, n0, n1, partial);
      hipLaunchKernelGGL(k_mlp_reduce, dim3((kPartial + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
                         (const float *)partial, blocks, grad, dl);
      b1t *= hp->beta1;
      b2t *= hp->beta2;
      hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpParams + kBlock - 1) / kBlock), dim3(kBlock), 0, s, dev, mom, vel,
                         (const float *)grad, hp->lr, hp->beta1, hp->beta2, hp->eps, (float)(1.0 - b1t),
                         (float)(1.0 - b2t));
      if (hipGetLastError() != hipSuccess) return SPGEMM_E_HIP;
      if (loss_curve && b == nb - 1) {
        float h = 0.f;
        if (hipMemcpyAsync(&h, dl, sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess) return SPGEMM_E_HIP;
        if (hipStreamSynchronize(s) != hipSuccess) return SPGEMM_E_HIP;
        ep_loss = h;
      }
    }
    losses[(size_t)ep] = (float)ep_loss;
  }
  (void)dloss_step;
  (void)steps;
  float host[kMlpDevFloats];
  if (hipMemcpyAsync(host, dev, sizeof(host), hipMemcpyDeviceToHost, s) != hipSuccess) return SPGEMM_E_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return SPGEMM_E_HIP;
  if (loss_curve) memcpy(loss_curve, losses.data(), sizeof(float) * (size_t)hp->epochs);
  return spgemm_model_create(host, host + kMlpParams, host + kMlpParams + 3, out);
}

spgemm_status spgemm_model_predict(const spgemm_model *m, const int32_t *f1, const int32_t *f2, const int32_t *f3,
                                   int64_t n, float *pred, void *dev_params, void *stream) {
  if (!m || !f1 || !f2 || !f3 || !pred || !dev_params) return SPGEMM_E_NULL;
  spgemm_status st = spgemm_model_upload(m, dev_params, stream);
  if (st != SPGEMM_OK) return st;
  if (launch_mlp_predict((const float *)dev_params, f1, f2, f3, n, pred, (hipStream_t)stream) != hipSuccess)
    return SPGEMM_E_HIP;
  return SPGEMM_OK;
}

}  // extern "C"
