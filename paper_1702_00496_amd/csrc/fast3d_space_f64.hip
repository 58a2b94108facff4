// Instantiation of the 32 x 32 3-D sweep: double, space-expanded schemes.
#include "step3d_fast.hpp"

namespace atfd {
hipError_t launch_fast3d_space_f64(const StepParams& p, hipStream_t st) {
  return fast3d::launch_space_t<double>(p, st);
}
}  // namespace atfd
