// Delay ensembles: every member is a periodic 1-D advection-diffusion problem
// split into PEs that exchange edge values through a ring of past levels and
// see them with random delays (Sec. 2; Sec. 5.1 simulation of delays). A
// member never spans two workgroups, so one persistent launch can run all
// steps: each workgroup loops over the steps of its members with a workgroup
// barrier between steps (all members' data stay in L2 / Infinity Cache).
//
// Per point and step: the standard central difference on level n for taps
// inside the PE (Sec. 2 eq. general_deriv), the AT combination in double of
// T delayed levels of the neighbour's edge strip for taps across a PE face
// (Sec. 3.4 Example 3 eq. cd4-at and Tables atschemes-left/right), the
// advection-diffusion right-hand side (Sec. 5 eq. general) and Euler or AB2
// (Sec. 4.1 eqs. time_disc, time_ab2; AB2 starts with Euler). New edge values
// are published to the ring slot of level n + 1.

#include "ensemble.hpp"

namespace atfd {
namespace {

constexpr int kEnsMaxThreads = 1024;

template <typename Real>
__device__ inline Real ens_tap(const EnsMember& M, int o) {
  if constexpr (sizeof(Real) == 8) return M.kad[o];
  else return M.kadf[o];
}

// Phase 1 of a step: every halo value of member M at step n, i.e. for each
// PE, side (0: left of the PE, 1: right) and depth d the value that taps
// reaching across that face use: the combination in double of the live
// delayed levels of the neighbour's edge strip (the standard scheme: the
// neighbour's current value). Stored at hb[hoff + (pe * 2 + side) * s + d].
// One thread per face: one delay draw, its weights from the member's table,
// then all s * T reads of the face issued together.
template <typename Real, int S>
__device__ inline void ens_member_halos(const EnsMember& M, const Real* __restrict__ u,
                                        const Real* __restrict__ ring, Real* __restrict__ hb, int64_t n) {
  const int faces = M.npe * 2;
  const int64_t slot_stride = static_cast<int64_t>(M.npe) * 2 * S;
  for (int j = threadIdx.x; j < faces; j += blockDim.x) {
    const int pe = j >> 1, side = j & 1;
    const int q = side ? (pe + 1 == M.npe ? 0 : pe + 1) : (pe == 0 ? M.npe - 1 : pe - 1);
    Real v[S];
    if (M.mode == AT_SYNC) {
      const Real* src = u + M.off + static_cast<int64_t>(q) * M.b + (side ? 0 : M.b - S);
#pragma unroll
      for (int d = 0; d < S; ++d) v[d] = src[d];
    } else {
      int k = 0;
      if (M.mode == AT_DELAY_RNG)
        k = raw_delay(M.key, n, static_cast<uint32_t>(2 * pe + side), M.thr, M.L);
      k = clamp_startup(k, n, M.T);
      // the left neighbour's right strip (face 1) or the right neighbour's
      // left strip (face 0)
      const Real* strip = ring + M.ring_off + (static_cast<int64_t>(q) * 2 + (side ? 0 : 1)) * S;
      // all kMaxT levels are read (a level beyond T, or before t = 0, reads
      // an in-range slot that a zero weight then drops), so the reads of the
      // face are in flight together
      Real raw[kMaxT][S];
      const int r0 = static_cast<int>(n % M.nslots);
#pragma unroll
      for (int m = 0; m < kMaxT; ++m) {
        const Real* lv = strip + slot_back(r0, k + min(m, M.T - 1), M.nslots) * slot_stride;
#pragma unroll
        for (int d = 0; d < S; ++d) raw[m][d] = lv[d];
      }
      double acc[S];
#pragma unroll
      for (int d = 0; d < S; ++d) acc[d] = 0.0;
#pragma unroll
      for (int m = 0; m < kMaxT; ++m) {
        const double w = m < M.T ? M.wt[k][m] : 0.0;
#pragma unroll
        for (int d = 0; d < S; ++d) acc[d] += w != 0.0 ? w * static_cast<double>(raw[m][d]) : 0.0;
      }
#pragma unroll
      for (int d = 0; d < S; ++d) v[d] = static_cast<Real>(acc[d]);
    }
    Real* dst = hb + M.hoff + static_cast<int64_t>(j) * S;
#pragma unroll
    for (int d = 0; d < S; ++d) dst[d] = v[d];
  }
}

// V consecutive points of one PE with the S neighbours on each side, loaded.
template <typename Real, int S, int V>
struct EnsChunk {
  Real w[V + 2 * S];   // positions l0 - S .. l0 + V - 1 + S
  Real fo[V];          // f^{n-1} (AB2)
  int pe, l0;
  int64_t g0;
};

template <typename Real, int V>
__device__ inline void ens_load(const Real* p, Real* dst) {
  if constexpr (V == 4 && sizeof(Real) == 4) {
    const float4 t = *reinterpret_cast<const float4*>(p);
    dst[0] = t.x; dst[1] = t.y; dst[2] = t.z; dst[3] = t.w;
  } else if constexpr (V == 4) {
    const double2 a = *reinterpret_cast<const double2*>(p);
    const double2 b = *reinterpret_cast<const double2*>(p + 2);
    dst[0] = a.x; dst[1] = a.y; dst[2] = b.x; dst[3] = b.y;
  } else {
#pragma unroll
    for (int e = 0; e < V; ++e) dst[e] = p[e];
  }
}

template <typename Real, int V>
__device__ inline void ens_store(Real* p, const Real* src) {
  if constexpr (V == 4 && sizeof(Real) == 4) {
    *reinterpret_cast<float4*>(p) = make_float4(src[0], src[1], src[2], src[3]);
  } else if constexpr (V == 4) {
    *reinterpret_cast<double2*>(p) = make_double2(src[0], src[1]);
    *reinterpret_cast<double2*>(p + 2) = make_double2(src[2], src[3]);
  } else {
#pragma unroll
    for (int e = 0; e < V; ++e) p[e] = src[e];
  }
}

// Loads of chunk c (points V c .. V c + V - 1 of member M). A neighbour
// position outside the PE reads the halo value of that face instead: the
// address is selected, so no load sits behind a branch.
template <typename Real, int S, int V, bool AB2>
__device__ inline EnsChunk<Real, S, V> ens_chunk_load(const EnsMember& M, const Real* __restrict__ u,
                                                      const Real* __restrict__ f,
                                                      const Real* __restrict__ hb, int c) {
  EnsChunk<Real, S, V> k;
  const int i0 = V * c;
  k.pe = i0 / M.b;
  k.l0 = i0 - k.pe * M.b;
  k.g0 = M.off + i0;
  const Real* hl = hb + M.hoff + (k.pe * 2 + 0) * S;
  const Real* hr = hb + M.hoff + (k.pe * 2 + 1) * S;
  ens_load<Real, V>(u + k.g0, k.w + S);
#pragma unroll
  for (int o = 1; o <= S; ++o) {
    const int pl = k.l0 - o;
    const Real* al = pl >= 0 ? u + k.g0 - o : hl + (S + pl);
    k.w[S - o] = *al;
    const int pr = k.l0 + V - 1 + o;
    const Real* ar = pr < M.b ? u + k.g0 + V - 1 + o : hr + (pr - M.b);
    k.w[S + V - 1 + o] = *ar;
  }
  // f^{n-1} of an AB2 member (the sweep is instantiated per integrator, so
  // Euler members load nothing here; at n = 0 the update weights f, which
  // at_ens_set_state zeroes, by an exact zero)
  if constexpr (AB2) ens_load<Real, V>(f + k.g0, k.fo);
  return k;
}

// Right-hand side, update, stores and the publish of new edge values.
template <typename Real, int S, int V, bool AB2>
__device__ inline void ens_chunk_finish(const EnsMember& M, const EnsChunk<Real, S, V>& k, Real* __restrict__ un,
                                        Real* __restrict__ f, Real* __restrict__ ring, int64_t n) {
  const Real dt = static_cast<Real>(M.dt);
  // AB2 after its first step: u + dt (3/2 f^n - 1/2 f^{n-1}); Euler (and the
  // first AB2 step): u + dt f^n
  const bool ab2 = AB2 && n > 0;
  const Real b1 = ab2 ? Real(1.5) : Real(1), b2 = ab2 ? Real(-0.5) : Real(0);
  Real r[V], acc[V];
#pragma unroll
  for (int e = 0; e < V; ++e) {
    const Real u0 = k.w[S + e];
    // f = sum over taps of (alpha c2 - c c1) (v - u0): every neighbour enters
    // as a difference to u0, so float rounding stays relative to O(dx) terms
    Real a = Real(0);
#pragma unroll
    for (int o = 1; o <= S; ++o) {
      a += ens_tap<Real>(M, S - o) * (k.w[S + e - o] - u0);
      a += ens_tap<Real>(M, S + o) * (k.w[S + e + o] - u0);
    }
    acc[e] = a;
    if constexpr (AB2)
      r[e] = u0 + dt * (b1 * a + b2 * k.fo[e]);
    else
      r[e] = u0 + dt * (b1 * a);
  }
  ens_store<Real, V>(un + k.g0, r);
  if constexpr (AB2) ens_store<Real, V>(f + k.g0, acc);
  if (M.mode != AT_SYNC && (k.l0 < S || k.l0 + V - 1 >= M.b - S)) {
    const int pslot = static_cast<int>((n + 1) % M.nslots);
    Real* base = ring + M.ring_off + (static_cast<int64_t>(pslot) * M.npe + k.pe) * 2 * S;
#pragma unroll
    for (int e = 0; e < V; ++e) {
      const int l = k.l0 + e;
      if (l < S) base[l] = r[e];
      if (l >= M.b - S) base[S + (l - (M.b - S))] = r[e];
    }
  }
}

// Phase 2 of a step: the sweep over member M's points, V per chunk and U
// chunks per thread and iteration, all U chunks' loads issued before any
// result is stored so that they are in flight together.
template <typename Real, int S, int V, int U, bool AB2>
__device__ inline void ens_member_sweep(const EnsMember& M, const Real* __restrict__ u, Real* __restrict__ un,
                                        Real* __restrict__ f, Real* __restrict__ ring,
                                        const Real* __restrict__ hb, int64_t n) {
  const int nch = static_cast<int>(M.n / V);
  const int bd = blockDim.x;
  for (int c = threadIdx.x; c < nch; c += U * bd) {
    EnsChunk<Real, S, V> k[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      // chunks past the end re-load chunk c (in range) and are not stored
      const int cj = c + j * bd < nch ? c + j * bd : c;
      k[j] = ens_chunk_load<Real, S, V, AB2>(M, u, f, hb, cj);
    }
#pragma unroll
    for (int j = 0; j < U; ++j)
      if (c + j * bd < nch) ens_chunk_finish<Real, S, V, AB2>(M, k[j], un, f, ring, n);
  }
}

template <typename Real, int S, int UX>
__device__ inline void ens_member_sweep_s(const EnsMember& M, const Real* u, Real* un, Real* f, Real* ring,
                                          const Real* hb, int64_t n) {
  // as many chunks in flight as the 128 registers of a 1024-thread
  // workgroup hold without spilling; UX = 2 for workgroups of at most 512
  // threads (256 registers)
  constexpr int U = UX * (sizeof(Real) == 4 ? (S <= 2 ? 4 : 2) : (S <= 2 ? 2 : 1));
  constexpr int U1 = UX * (sizeof(Real) == 4 ? 2 : 1);
  // the integrator is uniform per member: one instantiation each
  if (M.integrator == AT_AB2) {
    if (M.vec)
      ens_member_sweep<Real, S, 4, U, true>(M, u, un, f, ring, hb, n);
    else
      ens_member_sweep<Real, S, 1, U1, true>(M, u, un, f, ring, hb, n);
  } else {
    if (M.vec)
      ens_member_sweep<Real, S, 4, U, false>(M, u, un, f, ring, hb, n);
    else
      ens_member_sweep<Real, S, 1, U1, false>(M, u, un, f, ring, hb, n);
  }
}

// Members whose descriptors a workgroup holds in LDS at a time.
constexpr int kEnsLdsMembers = AT_ENS_BATCH;

// All steps of `count` members whose descriptors are in LDS.
template <typename Real, int UX>
__device__ inline void ens_run(const EnsParams& p, int64_t n0, const EnsMember* mem, int count) {
  Real* f = static_cast<Real*>(p.f);
  Real* ring = static_cast<Real*>(p.ring);
  Real* hb = static_cast<Real*>(p.hbuf);
  for (int64_t st = 0; st < p.nsteps; ++st) {
    const int64_t n = n0 + st;
    const Real* u = static_cast<const Real*>(p.u[n & 1]);
    Real* un = static_cast<Real*>(p.u[(n + 1) & 1]);
    for (int i = 0; i < count; ++i) {
      const EnsMember& M = mem[i];
      switch (M.s) {
        case 1: ens_member_halos<Real, 1>(M, u, ring, hb, n); break;
        case 2: ens_member_halos<Real, 2>(M, u, ring, hb, n); break;
        default: ens_member_halos<Real, 3>(M, u, ring, hb, n); break;
      }
    }
    // halo values complete before the sweep reads them
    __syncthreads();
    for (int i = 0; i < count; ++i) {
      const EnsMember& M = mem[i];
      switch (M.s) {
        case 1: ens_member_sweep_s<Real, 1, UX>(M, u, un, f, ring, hb, n); break;
        case 2: ens_member_sweep_s<Real, 2, UX>(M, u, un, f, ring, hb, n); break;
        default: ens_member_sweep_s<Real, 3, UX>(M, u, un, f, ring, hb, n); break;
      }
    }
    // every member's level n+1 (field and ring) is complete, and the halo
    // values are consumed, before step n+1 starts
    __syncthreads();
  }
}

// One workgroup per bin of members. Members are independent problems, so a
// bin larger than the LDS descriptor cache runs all steps for one batch of
// members, then for the next.
template <typename Real, int MAXT, int UX>
__global__ __launch_bounds__(MAXT) void ens_steps_kernel(EnsParams p) {
  __shared__ EnsMember s_mem[kEnsLdsMembers];
  constexpr int kWords = sizeof(EnsMember) / sizeof(uint32_t);
  static_assert(sizeof(EnsMember) % sizeof(uint32_t) == 0, "descriptors are copied as words");
  const int m0 = p.bin_start[blockIdx.x], m1 = p.bin_start[blockIdx.x + 1];
  const int64_t n0 = p.counter[0];
  for (int b0 = m0; b0 < m1; b0 += kEnsLdsMembers) {
    const int count = min(kEnsLdsMembers, m1 - b0);
    __syncthreads();   // the previous batch is done with the descriptors
    uint32_t* dst = reinterpret_cast<uint32_t*>(s_mem);
    for (int i = threadIdx.x; i < count * kWords; i += blockDim.x) {
      const int j = i / kWords;
      dst[i] = reinterpret_cast<const uint32_t*>(p.mem + p.order[b0 + j])[i - j * kWords];
    }
    __syncthreads();
    ens_run<Real, UX>(p, n0, s_mem, count);
  }
  if (threadIdx.x == 0) advance_counter(p.counter, n0 + p.nsteps - 1);
}

// Every ring slot of every member holds the edge strips of u^0.
template <typename Real>
__global__ __launch_bounds__(256) void ens_publish_all_kernel(EnsParams p) {
  const EnsMember& M = p.mem[blockIdx.x];
  if (M.mode == AT_SYNC) return;
  const Real* u = static_cast<const Real*>(p.u[0]);
  Real* ring = static_cast<Real*>(p.ring);
  const int s = M.s;
  const int64_t per_slot = static_cast<int64_t>(M.npe) * 2 * s;
  for (int64_t j = threadIdx.x; j < per_slot * M.nslots; j += blockDim.x) {
    const int64_t e = j % per_slot;
    const int pe = static_cast<int>(e / (2 * s));
    const int face = static_cast<int>((e / s) % 2);
    const int d = static_cast<int>(e % s);
    const int64_t src = static_cast<int64_t>(pe) * M.b + (face ? M.b - s + d : d);
    ring[M.ring_off + j] = u[M.off + src];
  }
}

// One workgroup per member. The exact solution at point i = 1024 q + j is
// sum_m Im(lo_m[j] hi_m[q]) with lo_m[j] = exp(i kappa_m dx j) and
// hi_m[q] = A_m e^{-alpha kappa_m^2 t} exp(i (kappa_m dx 1024 q + phi_m -
// kappa_m c t)), both tabulated in LDS, so a point costs two multiply-adds per
// mode instead of a sine.
constexpr int kEnsNormThreads = 1024;
constexpr int kEnsNormTable = 60 * 1024;   // LDS bytes for the two tables

template <typename Real>
__global__ __launch_bounds__(kEnsNormThreads) void ens_norms_kernel(EnsNormParams p) {
  extern __shared__ double2 etab[];   // lo[m][1024], then hi[m][nq]
  __shared__ double dec[kMaxModes], sh[kMaxModes];
  const EnsMember& M = p.mem[blockIdx.x];
  const Real* u = static_cast<const Real*>(p.u) + M.off;
  const double t = static_cast<double>(p.nstep) * M.dt;
  const double dx = M.length / static_cast<double>(M.n);
  const int nm = p.nmodes;
  const double* ph = p.phase + static_cast<int64_t>(blockIdx.x) * nm;
  if (static_cast<int>(threadIdx.x) < nm) {
    const int m = threadIdx.x;
    dec[m] = p.amp[m] * exp(-M.alpha * double(p.kap[m]) * p.kap[m] * t);
    sh[m] = ph[m] - double(p.kap[m]) * M.c * t;
  }
  __syncthreads();
  const int n = static_cast<int>(M.n);   // members are validated below 2^31 points
  const int nq = (n + kEnsNormThreads - 1) / kEnsNormThreads;
  const bool table = nm > 0 && static_cast<size_t>(nm) * (kEnsNormThreads + nq) * sizeof(double2) <=
                                   static_cast<size_t>(kEnsNormTable);
  double2* lo = etab;
  double2* hi = etab + nm * kEnsNormThreads;
  if (table) {
    for (int i = threadIdx.x; i < nm * (kEnsNormThreads + nq); i += blockDim.x) {
      double arg, scale = 1.0;
      if (i < nm * kEnsNormThreads) {
        arg = double(p.kap[i / kEnsNormThreads]) * dx * (i % kEnsNormThreads);
      } else {
        const int r = i - nm * kEnsNormThreads, m = r / nq, q = r % nq;
        arg = double(p.kap[m]) * dx * (static_cast<double>(q) * kEnsNormThreads) + sh[m];
        scale = dec[m];
      }
      double sv, cv;
      sincos(arg, &sv, &cv);
      etab[i] = make_double2(scale * cv, scale * sv);
    }
    __syncthreads();
  }
  double s1 = 0.0, s2 = 0.0, mx = 0.0, bad = 0.0;
  for (int q = 0; q < nq; ++q) {
    const int j = threadIdx.x, i = q * kEnsNormThreads + j;
    if (i >= n) break;
    double ref = 0.0;
    if (table) {
      for (int m = 0; m < nm; ++m) {
        const double2 a = lo[m * kEnsNormThreads + j], b = hi[m * nq + q];
        ref += a.y * b.x + a.x * b.y;
      }
    } else if (nm > 0) {
      for (int m = 0; m < nm; ++m) ref += dec[m] * sin(double(p.kap[m]) * dx * i + sh[m]);
    } else {
      ref = p.ref[M.off + i];
    }
    const double e = static_cast<double>(u[i]) - ref;
    if (!isfinite(e)) {
      bad += 1.0;
      continue;
    }
    s1 += fabs(e);
    s2 += e * e;
    mx = fmax(mx, fabs(e));
  }
  // wave64 tree, then the waves in order: a fixed summation order
  for (int off = 32; off > 0; off >>= 1) {
    s1 += __shfl_down(s1, off, 64);
    s2 += __shfl_down(s2, off, 64);
    mx = fmax(mx, __shfl_down(mx, off, 64));
    bad += __shfl_down(bad, off, 64);
  }
  __shared__ double part[kEnsNormThreads / 64][4];
  const int wave = threadIdx.x / 64;
  if ((threadIdx.x & 63) == 0) {
    part[wave][0] = s1;
    part[wave][1] = s2;
    part[wave][2] = mx;
    part[wave][3] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double r[4] = {0.0, 0.0, 0.0, 0.0};
    for (int w = 0; w < static_cast<int>(blockDim.x) / 64; ++w) {
      r[0] += part[w][0];
      r[1] += part[w][1];
      r[2] = fmax(r[2], part[w][2]);
      r[3] += part[w][3];
    }
    for (int j = 0; j < 4; ++j) p.out[blockIdx.x * 4 + j] = r[j];
  }
}

// Binned ensemble statistics of the per-member RMS error (Sec. 4 ensemble
// averages): one workgroup per (order group, dx bin). Two passes over the
// members in index order (mean, then the sum of squared deviations), each
// thread's partial sums combined by a wave64 shuffle tree and then wave by
// wave: a fixed summation order.
constexpr int kEnsStatsThreads = 256;

__device__ inline void ens_stats_reduce(double* v, int nv, double (*part)[3]) {
  for (int off = 32; off > 0; off >>= 1)
    for (int q = 0; q < nv; ++q) v[q] += __shfl_down(v[q], off, 64);
  const int wave = threadIdx.x / 64;
  __syncthreads();   // earlier readers of `part` are done
  if ((threadIdx.x & 63) == 0)
    for (int q = 0; q < nv; ++q) part[wave][q] = v[q];
  __syncthreads();
  for (int q = 0; q < nv; ++q) {
    double t = 0.0;
    for (int w = 0; w < kEnsStatsThreads / 64; ++w) t += part[w][q];
    v[q] = t;
  }
}

__global__ __launch_bounds__(kEnsStatsThreads) void ens_stats_kernel(EnsStatsParams p) {
  __shared__ double part[kEnsStatsThreads / 64][3];
  const int g = blockIdx.x / p.nbins, j = blockIdx.x % p.nbins;
  const double lo = p.edges[j], hi = p.edges[j + 1];
  double v[3] = {0.0, 0.0, 0.0};   // count, sum dx, sum rms
  for (int i = threadIdx.x; i < p.count; i += kEnsStatsThreads) {
    const EnsMember& M = p.mem[i];
    const double dx = M.length / static_cast<double>(M.n);
    if (M.s - 1 == g && dx >= lo && dx < hi) {
      v[0] += 1.0;
      v[1] += dx;
      v[2] += sqrt(p.sums[4 * i + 1] / static_cast<double>(M.n));
    }
  }
  ens_stats_reduce(v, 3, part);
  const double cnt = v[0];
  const double mean = cnt > 0.0 ? v[2] / cnt : 0.0;
  double d[1] = {0.0};
  for (int i = threadIdx.x; i < p.count; i += kEnsStatsThreads) {
    const EnsMember& M = p.mem[i];
    const double dx = M.length / static_cast<double>(M.n);
    if (M.s - 1 == g && dx >= lo && dx < hi) {
      const double e = sqrt(p.sums[4 * i + 1] / static_cast<double>(M.n)) - mean;
      d[0] += e * e;
    }
  }
  ens_stats_reduce(d, 1, part);
  if (threadIdx.x == 0) {
    double* o = p.out + static_cast<int64_t>(blockIdx.x) * 4;
    o[0] = cnt;
    o[1] = cnt > 0.0 ? v[1] / cnt : 0.0;
    o[2] = mean;
    o[3] = cnt > 1.0 ? d[0] / (cnt - 1.0) : 0.0;
  }
}

}  // namespace

hipError_t launch_ens_stats(const EnsStatsParams& p, hipStream_t st) {
  if (p.nbins < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(ens_stats_kernel, dim3(3 * p.nbins), dim3(kEnsStatsThreads), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_ens_steps(const EnsParams& p, bool f64, int nbins, int threads, hipStream_t st) {
  if (threads < 64 || threads > kEnsMaxThreads || threads % 64) return hipErrorInvalidValue;
  // workgroups of up to 512 threads have twice the registers: twice the
  // chunks in flight
  if (f64) {
    if (threads > 512)
      hipLaunchKernelGGL((ens_steps_kernel<double, 1024, 1>), dim3(nbins), dim3(threads), 0, st, p);
    else
      hipLaunchKernelGGL((ens_steps_kernel<double, 512, 2>), dim3(nbins), dim3(threads), 0, st, p);
  } else {
    if (threads > 512)
      hipLaunchKernelGGL((ens_steps_kernel<float, 1024, 1>), dim3(nbins), dim3(threads), 0, st, p);
    else
      hipLaunchKernelGGL((ens_steps_kernel<float, 512, 2>), dim3(nbins), dim3(threads), 0, st, p);
  }
  return hipGetLastError();
}

hipError_t launch_ens_publish_all(const EnsParams& p, bool f64, int count, hipStream_t st) {
  if (f64)
    hipLaunchKernelGGL(ens_publish_all_kernel<double>, dim3(count), dim3(256), 0, st, p);
  else
    hipLaunchKernelGGL(ens_publish_all_kernel<float>, dim3(count), dim3(256), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_ens_norms(const EnsNormParams& p, bool f64, int count, hipStream_t st) {
  if (f64)
    hipLaunchKernelGGL(ens_norms_kernel<double>, dim3(count), dim3(kEnsNormThreads), kEnsNormTable, st, p);
  else
    hipLaunchKernelGGL(ens_norms_kernel<float>, dim3(count), dim3(kEnsNormThreads), kEnsNormTable, st, p);
  return hipGetLastError();
}

}  // namespace atfd
