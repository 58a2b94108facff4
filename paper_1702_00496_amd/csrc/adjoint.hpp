// Discrete adjoint of the AT step: parameters and launchers shared by
// adjoint.hip and the host front end in atfd.cpp.
#pragma once

#include "atfd_internal.hpp"

namespace atfd {

constexpr int kAdjBlocks = 1024;   // fixed grid of the lambda kernel: its alpha partials

// One stage of the reversed step n (see adjoint.hip): mu = m0 y0 + m1 y1,
// out = b0 x0 + b1 x1 + (transposed stage) + drained adjoint ring.
struct AdjParams {
  StepParams sp;                   // the forward problem (taps, delays, ring layout)
  int64_t n;                       // the step being reversed (n -> n + 1)
  int64_t npts;
  int burgers;                     // Burgers right-hand side (taps depend on the stage field)
  const void* y0;
  const void* y1;
  double m0, m1;
  const void* x0;
  const void* x1;
  double b0, b1;
  void* out;                       // the stage's adjoint field
  const void* levels;              // stored levels of the stage field from seg_start, npts apart
  int64_t seg_start;
  const void* ring0;               // that field's ring at step seg_start
  void* hbuf;                      // forward halo values of this stage [pe][face strips]
  int64_t pfo[6];                  // offset of face f's strip inside one PE's pe_block values
  void* aring;                     // adjoint ring of the stage field, anslots slots
  int anslots;
  double* partial;                 // [adj_partials] alpha-gradient partial sums
  double wt[kMaxL][kMaxT];         // level weights c_m(k) of every delay k < L (host-computed)
};

int adj_blocks(int64_t npts);
// alpha-gradient partial sums the stage kernels write (>= kAdjBlocks; one per
// PE for the PE-tiled kernel)
int adj_partials(const StepParams& p);
hipError_t launch_adj_step(const AdjParams& q, bool f64, hipStream_t st);
hipError_t launch_adj_sum(const double* partial, int count, double* out, hipStream_t st);

}  // namespace atfd
