// Instantiation of the vector path of the generic sweep: float, 3-D.
#include "step_sweep.hpp"

namespace atfd {
hipError_t launch_step_vec_f32_d3(const StepParams& p, hipStream_t st, int blocks, int threads, size_t lds) {
  return sweep::launch_vec<float, 3>(p, st, blocks, threads, lds);
}
}  // namespace atfd
