// Declarations shared by the host-side translation units of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/spgemm.h"

namespace spg {

constexpr int kMlpHidden = 32;
constexpr int kMlpParams = kMlpHidden * 3 + kMlpHidden + kMlpHidden * kMlpHidden + kMlpHidden + kMlpHidden + 1;
constexpr int kMlpDevFloats = kMlpParams + 6;   // theta, mu[3], sd[3]

int device_cus();
int64_t *host_counters();

// Predicted nnz(C_row) for n rows; dev_params holds kMlpDevFloats floats
// (theta, mu, sd) already on the device.
hipError_t launch_mlp_predict(const float *dev_params, const int32_t *f1, const int32_t *f2,
                              const int32_t *f3, int64_t n, float *pred, hipStream_t s);

}  // namespace spg

struct spgemm_model {
  float theta[spg::kMlpParams];
  float mu[3];
  float sd[3];
};
