// Instantiation of the vector path of the generic sweep: double, 1-D.
#include "step_sweep.hpp"

namespace atfd {
hipError_t launch_step_vec_f64_d1(const StepParams& p, hipStream_t st, int blocks, int threads, size_t lds) {
  return sweep::launch_vec<double, 1>(p, st, blocks, threads, lds);
}
}  // namespace atfd
