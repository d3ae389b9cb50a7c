// Declarations shared by the host-side translation units of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/spgemm.h"
#include "spgemm_kernels.h"

namespace spg {

constexpr int kMlpHidden = 32;
constexpr int kMlpParams = kMlpHidden * 3 + kMlpHidden + kMlpHidden * kMlpHidden + kMlpHidden + kMlpHidden + 1;
constexpr int kMlpDevFloats = kMlpParams + 6;   // theta, mu[3], sd[3]

int device_cus();
int64_t *host_counters();

// Numeric pass of a plan as kernel launches only (no synchronisation), for
// graph capture; and access to the plan's device counters.
spgemm_status numeric_enqueue(spgemm_plan *p, void *scratch, size_t scratch_bytes, const double *av,
                              const double *bv, int64_t *c_row_ptr, int32_t *c_col, double *c_val,
                              int64_t c_capacity, hipStream_t s);
int64_t *plan_counters(spgemm_plan *p);
int plan_is_one_pass(const spgemm_plan *p);
size_t plan_workspace_bytes(int64_t rows, int64_t brows);
// workspace and scratch carry 256-byte aligned arrays (16-byte records among them)
inline bool aligned256(const void *p) { return ((uintptr_t)p & 255) == 0; }
spgemm_status plan_check_counters(spgemm_plan *p, const int64_t *h);

// Predicted nnz(C_row) for n rows; dev_params holds kMlpDevFloats floats
// (theta, mu, sd) already on the device.
hipError_t launch_mlp_predict(const float *dev_params, const int32_t *f1, const int32_t *f2,
                              const int32_t *f3, int64_t n, float *pred, hipStream_t s, float margin = 0.f,
                              int slack = 0, int64_t *partials = nullptr);
int64_t mlp_predict_blocks(int64_t n);
// Learned capacity of every row of A * B, its features computed from the
// operands: sums into counters[kCtrCapSum] (rows whose triple does not pack
// count 0; their summed bounds go to kCtrUnpacked), the largest sum over 64
// consecutive rows into kCtrWaveCap, and the multiplication count, longest
// row of A and empty rows into kCtrMults, kCtrMaxA and kCtrEmpty.  With a
// gate (the summed longest row of A) above gate_max only the longest row is
// passed on.
hipError_t launch_mlp_capacity(const float *dev_params, const Operands &op, int64_t *counters, int64_t *partials,
                               float margin, int slack, hipStream_t s, const int64_t *gate = nullptr,
                               int64_t gate_max = 0);

// Capacity of a row sized by the learned prediction: ceil(pred * (1 +
// margin)) + slack, clamped to [longest selected B row, multiplication
// count] (the bound itself for a prediction that is not a number in
// [0, bound]).  Shared by the sizing kernel and the prediction kernel.
__host__ __device__ inline int64_t learned_capacity(float pred, int32_t ub, int32_t maxb, float margin, int slack) {
  // a prediction that is not a number in [0, ub] gives the bound
  if (!(pred >= 0.0f && pred <= (float)ub)) return ub;
  double want = ceil((double)pred * (1.0 + (double)margin)) + (double)slack;
  double c = want < (double)maxb ? (double)maxb : want;
  return (int64_t)(c > (double)ub ? (double)ub : c);
}

}  // namespace spg

struct spgemm_model {
  float theta[spg::kMlpParams];
  float mu[3];
  float sd[3];
};
