// Discrete adjoint of the AT step: parameters and launchers shared by
// adjoint.hip and the host front end in atfd.cpp.
#pragma once

#include "atfd_internal.hpp"

namespace atfd {

constexpr int kAdjBlocks = 1024;   // fixed grid of the lambda kernel: its alpha partials

struct AdjParams {
  StepParams sp;                   // the forward problem (taps kad, c2; delays; ring layout)
  int64_t n;                       // the step being reversed (n -> n + 1)
  int64_t npts;
  double dt, beta0, beta1;         // mu^n = dt (beta0 lambda^{n+1} + beta1 lambda^{n+2})
  const void* lam1;                // lambda^{n+1}
  const void* lam2;                // lambda^{n+2}
  void* lam0;                      // lambda^n (output)
  void* mu;                        // mu^n (written by the first kernel of the step)
  void* hbuf;                      // forward halo values of step n [pe][face strips]
  void* aring;                     // adjoint ring, forward ring layout, anslots slots
  int anslots;
  const void* levels;              // forward levels seg_start .. seg_start + len, npts apart
  int64_t seg_start;
  const void* ring0;               // the forward ring at step seg_start
  double* partial;                 // [kAdjBlocks] alpha-gradient partial sums
};

int adj_blocks(int64_t npts);
hipError_t launch_adj_step(const AdjParams& q, bool f64, hipStream_t st);
hipError_t launch_adj_sum(const double* partial, int count, double* out, hipStream_t st);

}  // namespace atfd
