// Instantiation of the 32 x 32 3-D sweep: float, half-width s = 2.
#include "step3d_fast.hpp"

namespace atfd {
hipError_t launch_fast3d_f32_s2(const StepParams& p, hipStream_t st) {
  return fast3d::launch_fast_t<float, 2>(p, st);
}
}  // namespace atfd
