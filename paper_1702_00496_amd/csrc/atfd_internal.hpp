// Internal declarations of libatfd: device helpers shared by the kernels and
// the parameter blocks the host passes to them. Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/atfd.h"

namespace atfd {

constexpr int kMaxL = 8;
constexpr int kMaxT = 4;
constexpr int kMaxS = 3;
constexpr int kMaxModes = 16;
constexpr int kThreads = 256;          // workgroup size of the helper kernels
constexpr int kMaxSweepThreads = 1024; // largest workgroup of the generic sweep
constexpr int kMaxVec3Threads = 768;   // ... of its pipelined 3-D vector path (168 VGPRs per lane)
constexpr size_t kLdsLimit = 160 * 1024;

// ---------------------------------------------------------------- generator
// SplitMix64 output finaliser (Steele, Lea & Flood, OOPSLA 2014) used as a
// counter hash; golden-ratio increment.
constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

__host__ __device__ inline uint64_t mix64(uint64_t z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}

// Raw delay of (step n, face id) before the start-up clamp: the top 53 bits
// of the hash are binned by the cumulative thresholds thr[0..L-1]
// (thr[L-1] = 2^53), as in the bin matching of Sec. 5.1.
__host__ __device__ inline int raw_delay(uint64_t key, int64_t n, uint32_t face,
                                         const uint64_t* thr, int L) {
  const uint64_t ctr = ((static_cast<uint64_t>(n) << 32) | face) + 1ull;
  const uint64_t u53 = mix64(key + ctr * kGolden) >> 11;
  int k = 0;
  while (k < L - 1 && u53 >= thr[k]) ++k;
  return k;
}

// Ring slot of level n - back from r0 = n mod nslots, for 0 <= back < nslots
// (every delayed level k + m < L + T = nslots): no 64-bit division.
__host__ __device__ inline int slot_back(int r0, int back, int nslots) {
  const int s = r0 - back;
  return s < 0 ? s + nslots : s;
}

// No level before t = 0 exists: the delay is clamped so that the oldest level
// of the T-level combination, n - k - (T - 1), is not negative.
__host__ __device__ inline int clamp_startup(int k, int64_t n, int T) {
  const int64_t cap = n - T + 1 > 0 ? n - T + 1 : 0;
  return k < cap ? k : static_cast<int>(cap);
}

// Weights over delayed levels n-k-m, m = 0..T-1, of the time-expanded AT
// schemes (Sec. 3.4 Example 3, eq. cd4-at; Tables atschemes-left/right): the
// values that extrapolate T successive past levels back to level n, i.e. the
// Lagrange basis on nodes k, k+1, .., k+T-1 evaluated at 0:
//   w_m(k) = prod_{i != m} (k + i) / (i - m).
// For k = 0 this is (1, 0, .., 0): the scheme is the standard CD.
__host__ __device__ inline void level_weights(int k, int T, double* w) {
  for (int m = 0; m < T; ++m) {
    double num = 1.0, den = 1.0;
    for (int i = 0; i < T; ++i) {
      if (i == m) continue;
      num *= static_cast<double>(k + i);
      den *= static_cast<double>(i - m);
    }
    w[m] = num / den;
  }
}

// ---------------------------------------------------------------- kernels
// Workgroup -> PE map. Workgroups are handed to the 8 XCDs round-robin; this
// gives each XCD one contiguous range of PE ids (a slab of neighbouring PEs),
// so a halo row that one PE reads from its neighbour's field was most likely
// fetched into the same L2 by that neighbour.
__device__ inline int pe_of_workgroup(int b, int g) {
  return (g % 8 == 0) ? (b % 8) * (g / 8) + b / 8 : b;
}

// Step counter: counter[0] = step n, counter[1] = groups finished, then
// kCounterGroups group counters 128 bytes apart (zero between launches).
constexpr int kCounterGroups = 64;
constexpr int kCounterWords = 2 + 16 * kCounterGroups;

// Called by one thread of every workgroup after the step's last access to
// n = counter[0]: the last workgroup to arrive sets counter[0] = n + 1.
// Workgroup b counts in group b % 64 and the last one of a group in the top
// counter, so no address takes more than about gridDim / 64 atomics (one
// address taking one atomic per workgroup serialises them: about 12 ns each,
// 50 us for 4096 workgroups). Only the atomics order anything here; the field
// and ring stores need no fence because no workgroup of this launch reads
// them, and the launch boundary makes them visible to the next step.
__device__ inline void advance_counter(int64_t* counter, int64_t n) {
  unsigned long long* c = reinterpret_cast<unsigned long long*>(counter);
  const unsigned g = gridDim.x;
  const unsigned ng = g < kCounterGroups ? g : kCounterGroups;
  const unsigned gi = blockIdx.x % ng;
  const unsigned long long per = (g - gi + ng - 1) / ng;   // workgroups of group gi
  unsigned long long* cg = c + 2 + 16 * gi;
  if (atomicAdd(cg, 1ull) == per - 1ull) {
    atomicExch(cg, 0ull);
    if (atomicAdd(&c[1], 1ull) == static_cast<unsigned long long>(ng) - 1ull) {
      atomicExch(&c[1], 0ull);
      atomicExch(&c[0], static_cast<unsigned long long>(n + 1));
    }
  }
}

enum Stage : int { kStageSingle = 0, kStageRk1 = 1, kStageRk2 = 2 };

// Everything one sweep needs. Passed by value.
struct StepParams {
  // geometry
  int nx, ny, nz;              // global points
  int bx, by, bz;              // PE edge
  int px, py, pz;              // PEs per axis
  int ndim;
  int npe;
  int s;                       // stencil half-width (order / 2)
  int scheme;                  // AT_SCHEME_TIME | AT_SCHEME_SPACE_212 | AT_SCHEME_SPACE_222
  int sd;                      // depth of the face strips (s; 2 or 3 for the space-expanded schemes)
  // space-expanded schemes: taps of the point next to a low face, o = -3..3,
  // / dx and / dx^2 per axis (first derivative (1,2,2)a, second (2,1,2) or
  // (2,2,2)a); the high-face taps are the mirror images
  double sl1[3][2 * kMaxS + 1], sl2[3][2 * kMaxS + 1];
  // scheme
  double c1[3][2 * kMaxS + 1]; // first-derivative taps / dx (per axis)
  double c2[3][2 * kMaxS + 1]; // second-derivative taps / dx^2
  // folded taps for the 32 x 32 path: kad = alpha c2 - vel c1 (advection-
  // diffusion, one coefficient per tap), d2a = alpha c2 (Burgers), in double
  // and float
  double kad[3][2 * kMaxS + 1], d2a[3][2 * kMaxS + 1];
  float kadf[3][2 * kMaxS + 1], d2af[3][2 * kMaxS + 1], c1f[3][2 * kMaxS + 1];
  double vel[3];
  double alpha, dt;
  int equation, integrator, stage;
  // delays
  int mode, L, T;
  uint64_t key;
  uint64_t thr[kMaxL];
  const int8_t* host_delays;   // [host_nsteps][npe][ndim][2]
  // state (element type = bulk precision)
  void* ubuf[2];               // ping-pong solution, u^n in ubuf[n & 1]
  void* fbuf[2];               // f history (AB2: fbuf[0]; AB3: f^n -> fbuf[n & 1])
  void* ustar;                 // RK2 predictor
  void* ring;                  // u levels: slot, then face, then plane, then PE (see ring_index)
  void* sring;                 // RK2 predictor levels
  int nslots;
  int64_t pe_block;            // elements of all face strips of one PE (a slot holds npe of them)
  int64_t face_off[6];         // offset of face 2*axis+side's strips (all PEs) within a slot
  int64_t face_chunk[6];       // elements of one plane of one PE's strip of that face
  int64_t* counter;            // [0] = step n, [1] = finished workgroups
  int advance;                 // this launch ends the step: bump the counter
  int depth;                   // 3-D 32x32 path schedule: planes in flight D (1, 2, 4) with 4
                               // points per thread, or 8 + D with 2 points per thread; 16 + D:
                               // 4 points per thread, z sweep direction alternating per launch
  int sweep_down;              // this launch sweeps z downward (alternating variants)
  int pe_major;                // u, f and u* stored PE after PE (the 32 x 32 path), see pe_major_offset
  int yslices;                 // generic 3-D sweep: workgroups per PE along y (set per launch; 0, 1: one)
};

// Problems the 3-D path for 32 x 32 PE cross-sections takes store the
// solution, the integrator history and the RK2 predictor PE after PE:
// [pe][z][y][x] with the PE's own strides, so that a workgroup's z-plane is
// one contiguous block (4 KB in FP32) instead of 32 rows of 128 B at the
// global row pitch. Offset of global point (x, y, z) in that layout (PE edges
// 32 in x and y, bz in z; px, py PEs along x and y):
__host__ __device__ inline int64_t pe_major_offset(int x, int y, int z, int bz, int px, int py) {
  const int qz = z / bz;
  const int64_t pe = (x >> 5) + static_cast<int64_t>(px) * ((y >> 5) + static_cast<int64_t>(py) * qz);
  return ((pe * bz + (z - qz * bz)) << 10) + ((y & 31) << 5) + (x & 31);
}

// Ring layout. The strip of face f of a PE is a stack of planes (x and y
// faces: one per z-plane of the PE, [y][d] and [d][x] inside; z faces: one per
// depth d, [y][x] inside) of face_chunk[f] elements. A slot stores, face by
// face and plane by plane, the planes of all PEs side by side:
//   [slot][face][plane][pe][chunk].
// Workgroups sweep their PEs' z-planes in step, so the strips that all of them
// publish or read at one moment form one contiguous run of memory.
// PE-major problems (the 32 x 32 path) put the slots innermost instead:
//   [face][plane][pe][slot][chunk],
// so the T delayed levels a halo value combines (consecutive slots) are one
// contiguous run rather than T runs a slot apart; face f starts at nslots x
// face_off[f]. A ring of one slot (the adjoint ring of the synchronous arm,
// whose forward ring has none) takes nslots = 1.
__host__ __device__ inline int64_t ring_index(const StepParams& p, int slot, int pe, int f, int64_t plane,
                                              int64_t r) {
  if (p.pe_major) {
    const int64_t ns = p.nslots > 0 ? p.nslots : 1;
    return ns * p.face_off[f] + ((plane * p.npe + pe) * ns + slot) * p.face_chunk[f] + r;
  }
  return static_cast<int64_t>(slot) * p.npe * p.pe_block + p.face_off[f] +
         (plane * p.npe + pe) * p.face_chunk[f] + r;
}

// Same, for element q of the PE's strip counted plane after plane.
__host__ __device__ inline int64_t ring_index_q(const StepParams& p, int slot, int pe, int f, int64_t q) {
  const int64_t c = p.face_chunk[f];
  const int64_t plane = q / c;
  return ring_index(p, slot, pe, f, plane, q - plane * c);
}

struct NormParams {
  int nx, ny, nz, bx, by, bz, ndim, s;
  double length, alpha, dt;
  double vel[3];
  int nmodes;
  int kap[kMaxModes][3];
  double amp[kMaxModes], phase[kMaxModes];
  const void* u;
  const double* ref;
  double* partial;             // [nblocks][8]
  int64_t* counter;            // step n (time t = n dt)
  int pe_major, px, py;        // u stored PE after PE (pe_major_offset); ref is always [z][y][x]
};

// Launchers (step.hip / norms.hip). Return the HIP error of the launch.
hipError_t launch_step(const StepParams& p, bool f64, int s, hipStream_t st);
hipError_t launch_publish_all(const StepParams& p, bool f64, int s, hipStream_t st);
// Copy a field between the caller's [z][y][x] layout and the context's
// (PE-major where p.pe_major is set, else a plain copy).
hipError_t launch_field_copy(const StepParams& p, bool f64, const void* src, void* dst, bool to_internal,
                             hipStream_t st);
hipError_t launch_set_counter(int64_t* counter, int64_t n, hipStream_t st);
hipError_t launch_delays(const StepParams& p, int64_t n0, int64_t count, int8_t* out,
                         hipStream_t st);
// Workgroups of the allocation-free norm evaluation, and its device scratch
// (norms.hip: one array per GPU; `device` must be the current device).
constexpr int kNormStaticBlocks = 1024;
constexpr int kMaxDevices = 64;
hipError_t norms_static_scratch(int device, double** ptr);

hipError_t launch_norms(const NormParams& p, bool f64, int nblocks, double* result,
                        hipStream_t st);
size_t step_lds_bytes(const StepParams& p, bool f64, int s);
// 3-D sweep for 32 x 32 PE cross-sections (step3d_fast.hip). fast3d_shape:
// the problems it takes (with some schedule variant): 3-D, 32 x 32 PE
// cross-sections, a field below 4 GB, and the synchronous arm, the
// time-expanded schemes with T = s + 1 or the space-expanded ones with T = 1.
// Their fields are stored PE-major and only this path steps them.
bool fast3d_shape(int ndim, int bx, int by, int scheme, int mode, int T, int s, int64_t field_bytes);
// the schedule variant p.depth applies to p (a PE-major problem)
bool fast3d_applies(const StepParams& p, bool f64);
int fast3d_default_depth(bool f64);
bool fast3d_valid_variant(int v);
// Schedule variants of the generic 3-D sweep: kChunkVariant + c forces c
// z-chunks per PE (c in {1, 2, 4, 8, 16}, clamped to the PE depth; only where
// the sweep may split a PE), instead of the cost model.
constexpr int kChunkVariant = 32;
inline bool chunk_variant(int v) {
  return v == kChunkVariant + 1 || v == kChunkVariant + 2 || v == kChunkVariant + 4 || v == kChunkVariant + 8 ||
         v == kChunkVariant + 16;
}
// the generic sweep may split a PE's planes over several workgroups
bool sweep_can_chunk(const StepParams& p);

// Whether a 3-D PE, swept in y-slices of `rows` rows, is swept by the
// pipelined form of the generic sweep's vector path (where the instance has
// it): every thread owns at most one quad and one halo item (of the
// 2 sd (bx + rows)) of a slice's plane, at most kMaxVec3Threads threads.
inline bool vec_pipe(const StepParams& p, int sd, int rows) {
  if (p.ndim != 3) return false;
  const int64_t quads = static_cast<int64_t>(p.bx / 4) * rows;
  const int64_t halos = 2 * static_cast<int64_t>(sd) * (p.bx + rows);
  return quads <= kMaxVec3Threads && halos <= kMaxVec3Threads;
}

hipError_t launch_step_fast3d(const StepParams& p, bool f64, int s, hipStream_t st);

}  // namespace atfd
