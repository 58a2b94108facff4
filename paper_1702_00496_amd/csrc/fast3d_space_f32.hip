// Instantiation of the 32 x 32 3-D sweep: float, space-expanded schemes.
#include "step3d_fast.hpp"

namespace atfd {
hipError_t launch_fast3d_space_f32(const StepParams& p, hipStream_t st) {
  return fast3d::launch_space_t<float>(p, st);
}
}  // namespace atfd
