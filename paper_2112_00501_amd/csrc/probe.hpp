// Launch interface of the link-times-half-spinors measurement probe
// (probe.hip): kind 0 FP32 vector arithmetic, 1 bfloat16 MFMA with FP32
// accumulation.
#pragma once

#include <hip/hip_runtime.h>

namespace cs {

hipError_t launch_probe_link_product(int kind, long long nsites, int reps, const float* U, const float* H, float* V,
                                     hipStream_t s);

}  // namespace cs
