// Dispatcher of the 3-D sweep for 32 x 32 PE cross-sections; the kernel is
// in step3d_fast.hpp.

#include "step3d_fast.hpp"

namespace atfd {

int fast3d_default_depth(bool f64) { (void)f64; return 2; }

bool fast3d_valid_variant(int v) {
  return v == 1 || v == 2 || v == 4 || v == 9 || v == 10 || v == 12 || v == 17 || v == 18 || v == 20;
}

bool fast3d_shape(int ndim, int bx, int by, int scheme, int mode, int T, int s, int64_t field_bytes) {
  // the non-uniform-delay scheme runs the generic sweep in every mode, so
  // that its zero-delay and synchronous arms share one kernel
  if (scheme == AT_SCHEME_NONUNIFORM_212) return false;
  // the synchronous arm, time-expanded AT with T = s + 1 or the
  // space-expanded schemes (one level); other T take the generic sweep
  const bool space = mode != AT_SYNC && (scheme == AT_SCHEME_SPACE_212 || scheme == AT_SCHEME_SPACE_222);
  const bool levels_ok = mode == AT_SYNC || (scheme == AT_SCHEME_TIME && T == s + 1) || (space && T == 1);
  // 32-bit element offsets of the field
  return ndim == 3 && bx == fast3d::kB && by == fast3d::kB && levels_ok && field_bytes < (int64_t(1) << 32);
}

bool fast3d_applies(const StepParams& p, bool f64) {
  (void)f64;
  if (!p.pe_major || !fast3d_valid_variant(p.depth) || p.bz % (p.depth & 7) != 0) return false;
  // the space-expanded schemes have variants 1 and 2
  const bool space = p.mode != AT_SYNC && p.scheme != AT_SCHEME_TIME;
  return !space || p.depth == 1 || p.depth == 2;
}

hipError_t launch_step_fast3d(const StepParams& p, bool f64, int s, hipStream_t st) {
  if (p.mode != AT_SYNC && p.scheme == AT_SCHEME_NONUNIFORM_212) return hipErrorInvalidValue;
  if (p.mode != AT_SYNC && p.scheme != AT_SCHEME_TIME)
    return f64 ? launch_fast3d_space_f64(p, st) : launch_fast3d_space_f32(p, st);
  if (f64) {
    switch (s) {
      case 1: return launch_fast3d_f64_s1(p, st);
      case 2: return launch_fast3d_f64_s2(p, st);
      case 3: return launch_fast3d_f64_s3(p, st);
    }
  } else {
    switch (s) {
      case 1: return launch_fast3d_f32_s1(p, st);
      case 2: return launch_fast3d_f32_s2(p, st);
      case 3: return launch_fast3d_f32_s3(p, st);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace atfd
