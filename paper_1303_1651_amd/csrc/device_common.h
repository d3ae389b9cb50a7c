// Device-side helpers shared by the HIP kernels of the library (gfx950,
// wave64).  Nothing here is visible through the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spg {

constexpr int kWave = 64;
constexpr int kBlock = 256;                  // threads per workgroup everywhere
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int32_t kEmpty = -1;               // empty accumulator slot (columns are >= 0)
constexpr int32_t kColMax = 0x7fffffff;      // "no more entries" in the merge tier

// One FP64 multiply rounded, then one FP64 add rounded: the update of the
// dense temporary row in the paper's row-major kernel (Section IV-A).  No
// contraction into a fused multiply-add.
__device__ __forceinline__ double mul_add_rn(double acc, double a, double b) {
#pragma clang fp contract(off)
  double p = a * b;
  return acc + p;
}

// +0.0 + a*b: the first update of a slot.  Starting from +0.0 turns a
// product of -0.0 into +0.0, exactly as adding into a zero-filled vector.
__device__ __forceinline__ double first_add_rn(double a, double b) {
#pragma clang fp contract(off)
  double p = a * b;
  double z = 0.0;
  return z + p;
}

__device__ __forceinline__ int lane_id() {
  return __builtin_amdgcn_mbcnt_hi(-1, __builtin_amdgcn_mbcnt_lo(-1, 0));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Mask of the G lanes of the caller's group (groups are aligned runs of G
// lanes inside the wave).
template <int G>
__device__ __forceinline__ uint64_t group_mask() {
  if constexpr (G == 64) return ~0ull;
  else {
    int first = lane_id() & ~(G - 1);
    return ((1ull << G) - 1ull) << first;
  }
}

// ------------------------------------------------------------ wave scans
__device__ __forceinline__ int64_t wave_inclusive_sum(int64_t v) {
  int l = lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    int64_t o = __shfl_up(v, d, kWave);
    if (l >= d) v += o;
  }
  return v;
}

__device__ __forceinline__ int32_t wave_inclusive_sum32(int32_t v) {
  int l = lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    int32_t o = __shfl_up(v, d, kWave);
    if (l >= d) v += o;
  }
  return v;
}

__device__ __forceinline__ int64_t wave_sum(int64_t v) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

__device__ __forceinline__ int64_t wave_max64(int64_t v) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v = max(v, __shfl_xor(v, d, kWave));
  return v;
}

__device__ __forceinline__ int32_t wave_max32(int32_t v) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v = max(v, __shfl_xor(v, d, kWave));
  return v;
}

__device__ __forceinline__ int32_t wave_min32(int32_t v) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v = min(v, __shfl_xor(v, d, kWave));
  return v;
}

// Block-wide exclusive scan of one int64 per thread.  `wtot` is LDS scratch
// of kWavesPerBlock + 1 entries; returns the exclusive prefix and the total.
__device__ __forceinline__ int64_t block_exclusive_sum(int64_t v, int64_t *wtot, int64_t *total) {
  int w = threadIdx.x / kWave;
  int64_t inc = wave_inclusive_sum(v);
  if (lane_id() == kWave - 1) wtot[w] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int i = 0; i < kWavesPerBlock; ++i) {
      int64_t t = wtot[i];
      wtot[i] = run;
      run += t;
    }
    wtot[kWavesPerBlock] = run;
  }
  __syncthreads();
  int64_t r = wtot[w] + inc - v;
  *total = wtot[kWavesPerBlock];
  __syncthreads();
  return r;
}

// ------------------------------------------------- decoupled look-back
// A tile's status word: two flag bits over a 62-bit value.  Tiles are
// numbered by an atomic ticket in the order they start, so every tile waits
// only on tiles already running: the chain always makes progress.
constexpr uint64_t kFlagAgg = 1ull << 62;
constexpr uint64_t kFlagPre = 2ull << 62;
constexpr uint64_t kValMask = (1ull << 62) - 1ull;

// The status word carries everything a successor needs (flag and value in
// one 64-bit atomic), so relaxed agent-scope accesses suffice: they bypass
// the non-coherent caches without the L2 write-back (release) or
// invalidation (acquire) that stronger orderings cost on a multi-XCD part.
__device__ __forceinline__ void status_store(uint64_t *p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t status_load(uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Called by all 64 lanes of ONE wave.  Publishes the tile's aggregate, walks
// back over the predecessors' status words 64 at a time until an inclusive
// prefix is found, publishes this tile's inclusive prefix and returns the
// exclusive prefix (same value in every lane).
// A predecessor that never publishes (which would be a bug) must not hang
// the device: after kSpinLimit polls the wait gives up, returns what it has
// and raises *err so the host reports a failure.
constexpr int64_t kSpinLimit = 1ll << 24;

// abort_bit: give up at once when another workgroup has raised that flag in
// *err (the result is then discarded by the host).
__device__ inline int64_t lookback_exclusive(uint64_t *status, int64_t tile, int64_t aggregate,
                                             int64_t *err = nullptr, int64_t err_bit = 0,
                                             int64_t abort_bit = 0) {
  int l = lane_id();
  int64_t polls = 0;
  if (tile == 0) {
    if (l == 0) status_store(status, kFlagPre | (uint64_t)aggregate);
    return 0;
  }
  if (l == 0) status_store(status + tile, kFlagAgg | (uint64_t)aggregate);
  int64_t excl = 0;
  int64_t j = tile - 1;
  while (true) {
    int64_t idx = j - l;
    uint64_t s = idx >= 0 ? status_load(status + idx) : (kFlagPre | 0ull);
    uint64_t flag = s & ~kValMask;
    uint64_t have_pre = ballot(flag == kFlagPre);
    uint64_t invalid = ballot(flag == 0);
    // lanes up to and including the nearest inclusive prefix must be ready
    uint64_t upto = have_pre ? ((have_pre & (~have_pre + 1)) << 1) - 1ull : ~0ull;
    if (invalid & upto) {
      if (++polls > kSpinLimit) {
        if (l == 0 && err) atomicOr((unsigned long long *)err, (unsigned long long)err_bit);
        break;
      }
      if (abort_bit && (polls & 255) == 0) {
        const int64_t e = __shfl(l == 0 ? __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0, 0,
                                 kWave);
        if (e & abort_bit) break;
      }
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    int64_t mine = (upto >> l) & 1ull ? (int64_t)(s & kValMask) : 0;
    excl += wave_sum(mine);
    if (have_pre) break;
    j -= kWave;
  }
  if (l == 0) status_store(status + tile, kFlagPre | (uint64_t)(excl + aggregate));
  return excl;
}

}  // namespace spg
