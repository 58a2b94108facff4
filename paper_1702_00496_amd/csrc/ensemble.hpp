// Delay ensembles: descriptors and launchers shared by ensemble.hip and the
// host front end ensemble_api.cpp.
#pragma once

#include "atfd_internal.hpp"

namespace atfd {

// One member of the ensemble: a periodic 1-D advection-diffusion problem.
struct EnsMember {
  int64_t off;                     // first point in the packed fields
  int64_t ring_off;                // first value of its ring in the packed ring
  int64_t hoff;                    // first value of its halo values in the packed halo buffer
  int64_t n;                       // points
  int b, npe, s, T, L, nslots;     // PE edge, PEs, half-width, levels, max delay, ring slots
  int integrator, mode;            // AT_EULER | AT_AB2; AT_DELAY_RNG | AT_DELAY_ZERO | AT_SYNC
  int vec;                         // 4-point vector sweep (b % 4 == 0 and off % 4 == 0)
  uint64_t key;                    // generator key
  uint64_t thr[kMaxL];             // delay bin thresholds
  double wt[kMaxL][kMaxT];         // level weights c_m(k) for every delay k < L
  double dt;
  double kad[2 * kMaxS + 1];       // alpha c2/dx^2 - c c1/dx per tap o = -s..s
  float kadf[2 * kMaxS + 1];
  double length, c, alpha;         // for the exact solution
};

struct EnsParams {
  const EnsMember* mem;            // [count]
  const int* bin_start;            // [nbins + 1] ranges of `order`
  const int* order;                // member ids, grouped by workgroup
  void* u[2];                      // packed fields, u^n in u[n & 1]
  void* f;                         // packed f^{n-1} (AB2 members)
  void* ring;                      // packed rings [member][slot][pe][face][s]
  void* hbuf;                      // packed halo values of the current step [member][pe][side][s]
  int64_t* counter;                // [0] = step n, [1] = finished workgroups
  int64_t nsteps;                  // steps of this launch
};

struct EnsNormParams {
  const EnsMember* mem;
  const void* u;                   // packed current fields
  const double* ref;               // packed reference (nmodes == 0)
  int64_t nstep;
  int nmodes;
  int kap[kMaxModes];
  double amp[kMaxModes];
  const double* phase;             // [count][nmodes], device
  double* out;                     // [count][4]: sum|E|, sum E^2, max|E|, non-finite count
};

struct EnsStatsParams {
  const EnsMember* mem;
  const double* sums;              // [count][4] from the norms kernel (sum E^2 at [1])
  const double* edges;             // [nbins + 1] ascending dx bin edges
  int count, nbins;
  double* out;                     // [3 groups][nbins][4]: count, mean dx, mean rms, unbiased variance
};

hipError_t launch_ens_stats(const EnsStatsParams& p, hipStream_t st);
hipError_t launch_ens_steps(const EnsParams& p, bool f64, int nbins, int threads, hipStream_t st);
hipError_t launch_ens_publish_all(const EnsParams& p, bool f64, int count, hipStream_t st);
hipError_t launch_ens_norms(const EnsNormParams& p, bool f64, int count, hipStream_t st);

}  // namespace atfd
