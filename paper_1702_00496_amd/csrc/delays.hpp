// Device delay tables beyond the per-face one of launch_delays (step.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "atfd_internal.hpp"

namespace atfd {

// Delays of the second buffer point of every face (non-uniform-delay scheme)
// of steps n0 .. n0+count-1, after the start-up clamp: out[count][npe][2*ndim].
hipError_t launch_point_delays(const StepParams& p, int64_t n0, int64_t count, int8_t* out, hipStream_t st);

}  // namespace atfd
