// AT finite-difference sweep for gfx950.
//
// One workgroup owns one PE (a bx*by*bz brick) and streams its z-planes
// through a ring of LDS planes. Each LDS plane holds the PE's bx*by points
// plus an s-wide frame of x/y halo values; the z neighbours are the planes
// above and below in the LDS ring. Halo values across a PE face are the AT
// combination of T delayed levels of the neighbour's edge strip (computed in
// double, Sec. 3.4 eq. cd4-at), so every point then applies the standard
// central difference (Sec. 2 eq. general_deriv) to LDS data: interior points
// (set I_I) see only level-n values, buffer-adjacent points (set I_B) see the
// extrapolated halo exactly as in Tables atschemes-left/right.
//
// After the right-hand side (Sec. 5 eq. general) and the time update (Sec. 4.1
// eqs. time_disc, time_ab2; Heun), the new values of the s-deep edge layers
// are published into the neighbour-visible ring slot of the new level.
//
// Memory traffic per point and step: u^n read once, u^{n+1} written once,
// f^{n-1} read and f^n written (AB2), plus the face strips (1/b of the points
// per face and level).

#include <algorithm>

#include "step_sweep.hpp"

namespace atfd {
namespace {

using namespace sweep;

// Fill every ring slot (and the predictor ring) with the edge strips of the
// current field u^0.
template <typename Real, int DIM, int S>
__global__ __launch_bounds__(kThreads) void publish_all_kernel(StepParams p) {
  const int pid = blockIdx.x;
  const int qx = pid % p.px, qy = (pid / p.px) % p.py, qz = pid / (p.px * p.py);
  const int x0 = qx * p.bx, y0 = qy * p.by, z0 = qz * p.bz;
  const Real* u = static_cast<const Real*>(p.ubuf[0]);
  Real* R = static_cast<Real*>(p.ring);
  Real* SR = static_cast<Real*>(p.sring);
  const int64_t npts = static_cast<int64_t>(p.bx) * p.by * p.bz;
  for (int64_t i = threadIdx.x; i < npts; i += blockDim.x) {
    const int x = static_cast<int>(i % p.bx);
    const int y = static_cast<int>((i / p.bx) % p.by);
    const int z = static_cast<int>(i / (static_cast<int64_t>(p.bx) * p.by));
    int face[6];
    int64_t q[6];
    int nf = 0;
    if (x < S) { face[nf] = 0; q[nf++] = (static_cast<int64_t>(z) * p.by + y) * S + x; }
    if (x >= p.bx - S) { face[nf] = 1; q[nf++] = (static_cast<int64_t>(z) * p.by + y) * S + x - (p.bx - S); }
    if (DIM >= 2 && y < S) { face[nf] = 2; q[nf++] = (static_cast<int64_t>(z) * S + y) * p.bx + x; }
    if (DIM >= 2 && y >= p.by - S) { face[nf] = 3; q[nf++] = (static_cast<int64_t>(z) * S + y - (p.by - S)) * p.bx + x; }
    if (DIM == 3 && z < S) { face[nf] = 4; q[nf++] = (static_cast<int64_t>(z) * p.by + y) * p.bx + x; }
    if (DIM == 3 && z >= p.bz - S) { face[nf] = 5; q[nf++] = (static_cast<int64_t>(z - (p.bz - S)) * p.by + y) * p.bx + x; }
    if (!nf) continue;
    const Real v = p.pe_major ? u[pid * npts + i] : u[(static_cast<int64_t>(z0 + z) * p.ny + y0 + y) * p.nx + x0 + x];
    for (int j = 0; j < nf; ++j)
      for (int sl = 0; sl < p.nslots; ++sl) {
        const int64_t off = ring_index_q(p, sl, pid, face[j], q[j]);
        R[off] = v;
        if (SR) SR[off] = v;
      }
  }
}

// Copy between the [z][y][x] layout and the PE-major one, four consecutive x
// values (one quad) per thread; q counts quads in PE-major order. Word = a
// type of four values' size (vector path) or one value (any alignment).
template <typename Word, int WPQ>
__global__ __launch_bounds__(kThreads) void field_copy_kernel(const Word* src, Word* dst, uint32_t nquads,
                                                              int nx, int ny, int bz, int px, int py,
                                                              int to_pe_major) {
  for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < nquads; q += gridDim.x * blockDim.x) {
    // PE-major quad q: PE edges 32 x 32 x bz, 8 quads per row
    const uint32_t xq = q & 7, ly = (q >> 3) & 31, r = q >> 8;
    const uint32_t pe = r / bz, lz = r - pe * bz;
    const uint32_t qx = pe % px, qy = (pe / px) % py, qz = pe / (px * py);
    const uint32_t g = ((qz * bz + lz) * ny + qy * 32 + ly) * (nx / 4) + qx * 8 + xq;
    const uint32_t si = to_pe_major ? g : q, di = to_pe_major ? q : g;
#pragma unroll
    for (int w = 0; w < WPQ; ++w) dst[static_cast<size_t>(di) * WPQ + w] = src[static_cast<size_t>(si) * WPQ + w];
  }
}

__global__ void set_counter_kernel(int64_t* counter, int64_t n) {
  // step n; every other word (the group counters) zero
  for (int i = threadIdx.x; i < kCounterWords; i += blockDim.x) counter[i] = i == 0 ? n : 0;
}

// Delay table [count][npe][2*ndim] of steps n0.. with the sweep's routine.
__global__ void delays_kernel(StepParams p, int64_t n0, int64_t count, int8_t* out) {
  const int64_t per = static_cast<int64_t>(p.npe) * 2 * p.ndim;
  const int64_t total = count * per;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < total;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t n = n0 + i / per;
    const int r = static_cast<int>(i % per);
    const int pid = r / (2 * p.ndim), f = r % (2 * p.ndim);
    out[i] = p.mode == AT_SYNC ? 0 : static_cast<int8_t>(face_delay(p, pid, f, n));
  }
}

// Second-point delay table [count][npe][2*ndim] of steps n0.. (non-uniform scheme).
__global__ void point_delays_kernel(StepParams p, int64_t n0, int64_t count, int8_t* out) {
  const int64_t per = static_cast<int64_t>(p.npe) * 2 * p.ndim;
  const int64_t total = count * per;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < total;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t n = n0 + i / per;
    const int r = static_cast<int>(i % per);
    out[i] = static_cast<int8_t>(point_delay(p, r / (2 * p.ndim), r % (2 * p.ndim), n));
  }
}

// The vector path of the sweep takes PE x edges that are multiples of 4:
// each thread owns quads of consecutive points, and the field's PE rows then
// start on 16-byte boundaries. Its LDS rows hold bx + 8 values.
bool use_vec(const StepParams& p) { return p.bx % 4 == 0; }

template <typename Real, int DIM, int S, int SP>
size_t lds_bytes_t(const StepParams& p) {
  constexpr int SD = strip_depth<S, SP>();
  const int nsl = DIM == 3 ? 2 * SD + 2 : 1;
  const size_t row = use_vec(p) ? p.bx + 8 : p.bx + 2 * SD;
  const int rows = p.yslices > 1 ? p.by / p.yslices : p.by;   // a workgroup's y-slice
  const size_t plane = static_cast<size_t>(DIM >= 2 ? rows + 2 * SD : 1) * row;
  return nsl * plane * sizeof(Real);
}

// Workgroup size of the generic sweep: about four points of a plane per
// thread. A 3-D PE walks its planes with a barrier per plane, so it keeps up
// to 1024 threads (a 48 x 48 plane: 576). A 1-D or 2-D PE is a single plane
// loaded and computed once: when there are PEs enough for four workgroups per
// compute unit (256 CUs), at most 256 threads (16 points each for a 64 x 64
// PE) let several workgroups share a CU, one loading while another computes
// (4096^2 in 4096 PEs of 64^2: 78 us per step against 139 us with 1024
// threads, whose one workgroup per CU serialises the phases); with fewer PEs
// the larger groups keep the CUs filled (1024^2 in 256 PEs of 64^2: 14 us
// with 1024 threads, 20 us with 256).
int sweep_threads(const StepParams& p) {
  const int64_t pts = static_cast<int64_t>(p.bx) * (p.ndim >= 2 ? p.by : 1);
  int64_t t = (pts / 4 + 63) / 64 * 64;
  if (t < 64) t = 64;
  const int64_t cap = (p.ndim == 3 || p.npe < 4 * 256) ? kMaxSweepThreads : 256;
  if (t > cap) t = cap;
  return static_cast<int>(t);
}

// Workgroup size of the vector path: two quads of a plane per thread in 1-D
// and 2-D (their loads issued together), one in 3-D, with the same cap as
// above; where the 3-D sweep is pipelined, as many threads as the larger of
// the quad and halo item counts of a y-slice's plane.
int vec_threads(const StepParams& p, int sd) {
  const int rows = p.yslices > 1 ? p.by / p.yslices : p.by;
  const int64_t quads = static_cast<int64_t>(p.bx / 4) * (p.ndim >= 2 ? rows : 1);
  if (vec_pipe(p, sd, rows)) {
    const int64_t halos = 2 * static_cast<int64_t>(sd) * (p.bx + rows);
    const int64_t t = ((quads > halos ? quads : halos) + 63) / 64 * 64;
    return static_cast<int>(t < kMaxVec3Threads ? t : kMaxVec3Threads);
  }
  int64_t t = ((p.ndim == 3 ? quads : (quads + 1) / 2) + 63) / 64 * 64;
  if (t < 64) t = 64;
  const int64_t cap = (p.ndim == 3 || p.npe < 4 * 256) ? kMaxSweepThreads : 256;
  if (t > cap) t = cap;
  return static_cast<int>(t);
}

// Workgroups per PE along y of the 3-D vector sweep: two halves of the PE's
// rows where a whole cross-section is too large for the pipelined form but a
// half is not (more than 768 quads, e.g. 64 x 64: 256^3 in 4^3 PEs 99 -> 82
// us per step), the instance has that form and the planes may be split (as
// for z-chunks). Halving cross-sections that are pipelined already measured
// slower (192^3 in 4^3 PEs 43.9 -> 47.4 us).
template <typename Real, int S, int SP>
int sweep_yslices(const StepParams& p) {
  constexpr int sd = strip_depth<S, SP>();
  if (!pipe_form<Real, S, SP>() || p.ndim != 3 || !use_vec(p) || !sweep_can_chunk(p)) return 1;
  if (vec_pipe(p, sd, p.by) || p.by % 2 != 0 || p.by / 2 < sd || !vec_pipe(p, sd, p.by / 2)) return 1;
  return 2;
}

// Workgroups per PE of the generic sweep. A 3-D PE's planes are split into
// z-chunks (each reloads the SD planes around it) within one round of
// resident workgroups (256 CUs, each holding as many as its LDS and thread
// slots allow, at most four). Only where no chunk overwrites planes another
// one reads: the new level goes to the other solution buffer, or the stage
// writes the RK2 predictor / reads it (Heun). 1-D and 2-D PEs are a single
// plane.
constexpr int kNumCUs = 256;   // compute units of an MI355X

int sweep_chunks(const StepParams& p, size_t lds, int threads, int sd) {
  if (!sweep_can_chunk(p)) return 1;
  if (chunk_variant(p.depth)) {
    // a forced count (schedule variant), clamped to the depth, no empty chunk
    int nch = p.depth - kChunkVariant;
    if (nch > p.bz) nch = p.bz;
    const int zper = (p.bz + nch - 1) / nch;
    return (p.bz + zper - 1) / zper;
  }
  int per_cu = static_cast<int>((160 * 1024) / (lds > 0 ? lds : 1));
  const int by_threads = 2048 / threads;
  if (per_cu > by_threads) per_cu = by_threads;
  if (per_cu > 4) per_cu = 4;
  if (per_cu < 1) per_cu = 1;
  const int64_t slots = static_cast<int64_t>(kNumCUs) * per_cu;
  if (p.npe >= kNumCUs) {
    // every CU already has a PE: chunks only add co-resident workgroups,
    // as many as fill one resident round, of at least 8 planes each
    const int want = static_cast<int>(slots / (static_cast<int64_t>(p.npe) * (p.yslices > 1 ? p.yslices : 1)));
    if (want <= 1) return 1;
    int zper = (p.bz + want - 1) / want;
    if (zper < 8) zper = 8;
    return (p.bz + zper - 1) / zper;
  }
  // fewer PEs than CUs: a CU's time is about its workgroup count times the
  // planes each loads (its chunk plus sd reloaded on either side); take the
  // split with the smallest such product among those that stay in one
  // resident round and leave no chunk empty (the fewest chunks on a tie)
  int best = 1;
  int64_t best_cost = -1;
  const int nys = p.yslices > 1 ? p.yslices : 1;
  for (int nch = 1; nch <= p.bz; ++nch) {
    const int64_t wgs = static_cast<int64_t>(p.npe) * nch * nys;
    if (wgs > slots && nch > 1) break;
    const int zper = (p.bz + nch - 1) / nch;
    if ((p.bz + zper - 1) / zper != nch) continue;
    const int64_t cost = ((wgs + kNumCUs - 1) / kNumCUs) * (zper + 2 * sd);
    if (best_cost < 0 || cost < best_cost) {
      best_cost = cost;
      best = nch;
    }
  }
  return best;
}

}  // namespace

bool sweep_can_chunk(const StepParams& p) {
  return p.ndim == 3 && (p.ubuf[0] != p.ubuf[1] || p.integrator == AT_RK2);
}

namespace {

template <typename Real, int DIM>
hipError_t launch_vec_unit(const StepParams& p, hipStream_t st, int blocks, int threads, size_t lds) {
  if constexpr (sizeof(Real) == 4)
    return DIM == 1 ? launch_step_vec_f32_d1(p, st, blocks, threads, lds)
         : DIM == 2 ? launch_step_vec_f32_d2(p, st, blocks, threads, lds)
                    : launch_step_vec_f32_d3(p, st, blocks, threads, lds);
  else
    return DIM == 1 ? launch_step_vec_f64_d1(p, st, blocks, threads, lds)
         : DIM == 2 ? launch_step_vec_f64_d2(p, st, blocks, threads, lds)
                    : launch_step_vec_f64_d3(p, st, blocks, threads, lds);
}

// The launch parameters of one sweep: p with the y-slice count set.
template <typename Real, int DIM, int S, int SP>
StepParams launch_params(const StepParams& p) {
  StepParams q = p;
  q.yslices = DIM == 3 && use_vec(p) ? sweep_yslices<Real, S, SP>(p) : 1;
  return q;
}

template <typename Real, int DIM, int S, int SP>
hipError_t launch_t(const StepParams& p, hipStream_t st) {
  const bool vec = use_vec(p);
  const StepParams q = launch_params<Real, DIM, S, SP>(p);
  const size_t lds = lds_bytes_t<Real, DIM, S, SP>(q);
  const int threads = vec ? vec_threads(q, strip_depth<S, SP>()) : sweep_threads(q);
  const int blocks = p.npe * sweep_chunks(q, lds, threads, strip_depth<S, SP>()) * q.yslices;
  if (vec) return launch_vec_unit<Real, DIM>(q, st, blocks, threads, lds);
  hipLaunchKernelGGL((at_step_kernel<Real, DIM, S, SP>), dim3(blocks), dim3(threads), lds, st, q);
  return hipGetLastError();
}

template <typename Real, int DIM, int S>
hipError_t launch_pub_t(const StepParams& p, hipStream_t st) {
  hipLaunchKernelGGL((publish_all_kernel<Real, DIM, S>), dim3(p.npe), dim3(kThreads), 0, st, p);
  return hipGetLastError();
}

// Sweep launches by half-width s (and the space-expanded scheme, s = 1);
// publish_all launches by strip depth s.
template <typename Real, int DIM>
hipError_t dispatch_s(const StepParams& p, int s, hipStream_t st, bool pub) {
  if (!pub && p.scheme != AT_SCHEME_TIME) {
    if (s != 1) return hipErrorInvalidValue;
    if (p.scheme == AT_SCHEME_NONUNIFORM_212) return launch_t<Real, DIM, 1, 3>(p, st);
    return p.scheme == AT_SCHEME_SPACE_212 ? launch_t<Real, DIM, 1, 1>(p, st) : launch_t<Real, DIM, 1, 2>(p, st);
  }
  switch (s) {
    case 1: return pub ? launch_pub_t<Real, DIM, 1>(p, st) : launch_t<Real, DIM, 1, 0>(p, st);
    case 2: return pub ? launch_pub_t<Real, DIM, 2>(p, st) : launch_t<Real, DIM, 2, 0>(p, st);
    case 3: return pub ? launch_pub_t<Real, DIM, 3>(p, st) : launch_t<Real, DIM, 3, 0>(p, st);
  }
  return hipErrorInvalidValue;
}

template <typename Real>
hipError_t dispatch_dim(const StepParams& p, int s, hipStream_t st, bool pub) {
  switch (p.ndim) {
    case 1: return dispatch_s<Real, 1>(p, s, st, pub);
    case 2: return dispatch_s<Real, 2>(p, s, st, pub);
    case 3: return dispatch_s<Real, 3>(p, s, st, pub);
  }
  return hipErrorInvalidValue;
}

// LDS of one workgroup of the sweep as launch_t launches it
template <typename Real, int DIM, int S, int SP>
size_t lds_launch(const StepParams& p) {
  return lds_bytes_t<Real, DIM, S, SP>(launch_params<Real, DIM, S, SP>(p));
}

template <typename Real, int DIM>
size_t lds_s(const StepParams& p, int s) {
  if (p.scheme == AT_SCHEME_SPACE_212) return lds_launch<Real, DIM, 1, 1>(p);
  if (p.scheme == AT_SCHEME_SPACE_222) return lds_launch<Real, DIM, 1, 2>(p);
  if (p.scheme == AT_SCHEME_NONUNIFORM_212) return lds_launch<Real, DIM, 1, 3>(p);
  switch (s) {
    case 1: return lds_launch<Real, DIM, 1, 0>(p);
    case 2: return lds_launch<Real, DIM, 2, 0>(p);
    case 3: return lds_launch<Real, DIM, 3, 0>(p);
  }
  return ~size_t(0);
}

template <typename Real>
size_t lds_dim(const StepParams& p, int s) {
  switch (p.ndim) {
    case 1: return lds_s<Real, 1>(p, s);
    case 2: return lds_s<Real, 2>(p, s);
    case 3: return lds_s<Real, 3>(p, s);
  }
  return ~size_t(0);
}

}  // namespace

hipError_t launch_step(const StepParams& p, bool f64, int s, hipStream_t st) {
  // PE-major fields are stepped by the 32 x 32 path only (the host accepts
  // only schedule variants that apply)
  if (p.pe_major) return fast3d_applies(p, f64) ? launch_step_fast3d(p, f64, s, st) : hipErrorInvalidValue;
  return f64 ? dispatch_dim<double>(p, s, st, false) : dispatch_dim<float>(p, s, st, false);
}

hipError_t launch_field_copy(const StepParams& p, bool f64, const void* src, void* dst, bool to_internal,
                             hipStream_t st) {
  const size_t bytes = static_cast<size_t>(p.nx) * p.ny * p.nz * (f64 ? 8 : 4);
  if (!p.pe_major) return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st);
  const uint32_t nquads = static_cast<uint32_t>(static_cast<size_t>(p.nx) * p.ny * p.nz / 4);
  const int blocks = static_cast<int>(std::min<uint32_t>((nquads + kThreads - 1) / kThreads, 8192u));
  const bool vec = (reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16 == 0;
  const int tp = to_internal ? 1 : 0;
  if (vec && f64)
    hipLaunchKernelGGL((field_copy_kernel<uint4, 2>), dim3(blocks), dim3(kThreads), 0, st,
                       static_cast<const uint4*>(src), static_cast<uint4*>(dst), nquads, p.nx, p.ny, p.bz, p.px,
                       p.py, tp);
  else if (vec)
    hipLaunchKernelGGL((field_copy_kernel<uint4, 1>), dim3(blocks), dim3(kThreads), 0, st,
                       static_cast<const uint4*>(src), static_cast<uint4*>(dst), nquads, p.nx, p.ny, p.bz, p.px,
                       p.py, tp);
  else if (f64)
    hipLaunchKernelGGL((field_copy_kernel<uint64_t, 4>), dim3(blocks), dim3(kThreads), 0, st,
                       static_cast<const uint64_t*>(src), static_cast<uint64_t*>(dst), nquads, p.nx, p.ny, p.bz,
                       p.px, p.py, tp);
  else
    hipLaunchKernelGGL((field_copy_kernel<uint32_t, 4>), dim3(blocks), dim3(kThreads), 0, st,
                       static_cast<const uint32_t*>(src), static_cast<uint32_t*>(dst), nquads, p.nx, p.ny, p.bz,
                       p.px, p.py, tp);
  return hipGetLastError();
}

hipError_t launch_publish_all(const StepParams& p, bool f64, int s, hipStream_t st) {
  return f64 ? dispatch_dim<double>(p, s, st, true) : dispatch_dim<float>(p, s, st, true);
}

size_t step_lds_bytes(const StepParams& p, bool f64, int s) {
  return f64 ? lds_dim<double>(p, s) : lds_dim<float>(p, s);
}

hipError_t launch_set_counter(int64_t* counter, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(set_counter_kernel, dim3(1), dim3(64), 0, st, counter, n);
  return hipGetLastError();
}

hipError_t launch_delays(const StepParams& p, int64_t n0, int64_t count, int8_t* out,
                         hipStream_t st) {
  const int64_t total = count * p.npe * 2 * p.ndim;
  int blocks = static_cast<int>((total + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(delays_kernel, dim3(blocks), dim3(256), 0, st, p, n0, count, out);
  return hipGetLastError();
}

hipError_t launch_point_delays(const StepParams& p, int64_t n0, int64_t count, int8_t* out, hipStream_t st) {
  const int64_t total = count * p.npe * 2 * p.ndim;
  int blocks = static_cast<int>((total + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(point_delays_kernel, dim3(blocks), dim3(256), 0, st, p, n0, count, out);
  return hipGetLastError();
}

}  // namespace atfd
