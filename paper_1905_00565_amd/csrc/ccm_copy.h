// ccm_copy.h -- the device forms' transfers of series in and results out,
// one launch each (defined in ccm_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ccmk {

// dst[0, n) = a, dst[n, 2n) = b (device arrays of doubles).
hipError_t launch_copy_pair(const double* a, const double* b, int64_t n, double* dst,
                            hipStream_t st);
// a = src[0, n), b = src[n, 2n).
hipError_t launch_split_pair(const double* src, int64_t n, double* a, double* b,
                             hipStream_t st);

}  // namespace ccmk
