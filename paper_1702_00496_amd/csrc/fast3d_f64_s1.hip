// Instantiation of the 32 x 32 3-D sweep: double, half-width s = 1.
#include "step3d_fast.hpp"

namespace atfd {
hipError_t launch_fast3d_f64_s1(const StepParams& p, hipStream_t st) {
  return fast3d::launch_fast_t<double, 1>(p, st);
}
}  // namespace atfd
