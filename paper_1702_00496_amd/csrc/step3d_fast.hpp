// 3-D AT sweep specialised for 32 x 32 PE cross-sections (gfx950): kernel
// template, instantiated per precision and half-width in fast3d_*.hip.
//
// Same scheme as the generic sweep in step.hip, organised for HBM bandwidth:
//  - one PE per workgroup; each thread owns V consecutive x points of one row
//    (V = 4: 256 threads, V = 2: 512 threads) and streams the PE's z-planes,
//    so every bulk global access is an 8- or 16-byte vector access; the
//    fields are stored PE-major, so a plane is one contiguous block (a
//    streaming copy's access pattern, not 32 rows at the global pitch);
//  - the z neighbours of a thread's points live in a register queue of 2s+1
//    vectors; x/y neighbours come from a double-buffered LDS plane (row
//    stride 40 with the x halo at columns 4-s..3 and 36..35+s, so vectors stay
//    aligned), one barrier per plane;
//  - reads of u^n, of the integrator history and of the halo values (the AT
//    combination of T delayed ring levels, in double) are issued D planes
//    ahead in a rotating set of registers: the slot consumed for plane z is
//    refilled with plane z + D, so no register copies stall the pipeline;
//  - the z sweep alternates direction from launch to launch (multistep
//    methods: by step parity; Heun: up in the first stage, down in the
//    second), so that a launch starts on the planes the previous one touched
//    last, which the Infinity Cache still holds when the working set is
//    larger than it; the arithmetic per point is the same either way;
//  - the integrator stage and the equation are template parameters and the
//    stencil taps arrive pre-folded with velocity and diffusivity; every
//    neighbour enters as (v - u0), which keeps float rounding relative to the
//    O(dx) differences instead of the O(1/dx^2) taps; each axis accumulates
//    into its own partial sum (three independent FMA chains per point).
// Halo items are quads (x faces are stored [z][y][d], y faces [z][d][x]); the
// ring slot and weight of every live delayed level of a face sit in LDS, and
// a level with zero weight re-reads level n-k with weight 0 so that no read
// sits behind a branch.
#pragma once

#include <type_traits>

#include "atfd_internal.hpp"

namespace atfd {
namespace fast3d {

constexpr int kB = 32;           // PE edge in x and y for this path
constexpr int kRS = 40;          // LDS row stride (elements)
constexpr int kHO = 4;           // LDS column of x = 0

enum Kind : int { kEuler = 0, kAb2 = 1, kAb3 = 2, kRk1 = 3, kRk2 = 4 };

template <typename Real, int V>
struct Vec {
  Real v[V];
};

// Vector loads/stores through a 32-bit byte offset from a uniform base, so the
// compiler can address with a scalar base register plus one VGPR.
template <typename Real, int V>
__device__ inline Vec<Real, V> ldv(const Real* base, uint32_t elem) {
  const char* p = reinterpret_cast<const char*>(base) + elem * static_cast<uint32_t>(sizeof(Real));
  Vec<Real, V> r;
  if constexpr (sizeof(Real) * V == 16) {
    if constexpr (sizeof(Real) == 4) {
      const float4 t = *reinterpret_cast<const float4*>(p);
      r.v[0] = t.x; r.v[1] = t.y; r.v[2] = t.z; r.v[3] = t.w;
    } else {
      const double2 t = *reinterpret_cast<const double2*>(p);
      r.v[0] = t.x; r.v[1] = t.y;
    }
  } else if constexpr (sizeof(Real) * V == 8) {
    const float2 t = *reinterpret_cast<const float2*>(p);
    r.v[0] = t.x; r.v[1] = t.y;
  } else {   // 32 bytes: two 16-byte halves
    const double2 a = *reinterpret_cast<const double2*>(p);
    const double2 b = *reinterpret_cast<const double2*>(p + 16);
    r.v[0] = a.x; r.v[1] = a.y; r.v[2] = b.x; r.v[3] = b.y;
  }
  return r;
}
template <typename Real, int V>
__device__ inline void stv(Real* base, uint32_t elem, const Vec<Real, V>& q) {
  char* p = reinterpret_cast<char*>(base) + elem * static_cast<uint32_t>(sizeof(Real));
  if constexpr (sizeof(Real) * V == 16) {
    if constexpr (sizeof(Real) == 4)
      *reinterpret_cast<float4*>(p) = make_float4(q.v[0], q.v[1], q.v[2], q.v[3]);
    else
      *reinterpret_cast<double2*>(p) = make_double2(q.v[0], q.v[1]);
  } else if constexpr (sizeof(Real) * V == 8) {
    *reinterpret_cast<float2*>(p) = make_float2(q.v[0], q.v[1]);
  } else {
    *reinterpret_cast<double2*>(p) = make_double2(q.v[0], q.v[1]);
    *reinterpret_cast<double2*>(p + 16) = make_double2(q.v[2], q.v[3]);
  }
}
// Same through a full pointer (ring strips may exceed 4 GB).
template <typename Real, int V>
__device__ inline Vec<Real, V> ldp(const Real* p) {
  return ldv<Real, V>(p, 0u);
}
template <typename Real, int V>
__device__ inline Vec<Real, V> zerov() {
  Vec<Real, V> r;
#pragma unroll
  for (int i = 0; i < V; ++i) r.v[i] = Real(0);
  return r;
}

// Store a run of N consecutive values (N = s <= 3; s = 2 as one 8- or
// 16-byte vector store: its offset is even).
template <typename Real, int N>
__device__ inline void st_run(Real* p, const Real* w) {
  if constexpr (N == 2 && sizeof(Real) == 4) {
    *reinterpret_cast<float2*>(p) = make_float2(w[0], w[1]);
  } else if constexpr (N == 2) {
    *reinterpret_cast<double2*>(p) = make_double2(w[0], w[1]);
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) p[i] = w[i];
  }
}

__device__ inline int neighbour_pe(const StepParams& p, int pid, int f) {
  int q[3] = {pid % p.px, (pid / p.px) % p.py, pid / (p.px * p.py)};
  const int ext[3] = {p.px, p.py, p.pz};
  const int a = f >> 1;
  q[a] = (q[a] + ((f & 1) ? 1 : ext[a] - 1)) % ext[a];
  return q[0] + p.px * (q[1] + p.py * q[2]);
}

__device__ inline int face_delay_fast(const StepParams& p, int pid, int f, int64_t n) {
  int k = 0;
  if (p.mode == AT_DELAY_RNG) {
    k = raw_delay(p.key, n, static_cast<uint32_t>(pid * 2 * p.ndim + f), p.thr, p.L);
  } else if (p.mode == AT_DELAY_HOST) {
    k = p.host_delays[(n * p.npe + pid) * (2 * p.ndim) + f];
  }
  return clamp_startup(k, n, p.T);
}

template <typename Real>
struct Taps;
template <>
struct Taps<double> {
  __device__ static double kad(const StepParams& p, int a, int o) { return p.kad[a][o]; }
  __device__ static double d2a(const StepParams& p, int a, int o) { return p.d2a[a][o]; }
  __device__ static double d1(const StepParams& p, int a, int o) { return p.c1[a][o]; }
};
template <>
struct Taps<float> {
  __device__ static float kad(const StepParams& p, int a, int o) { return p.kadf[a][o]; }
  __device__ static float d2a(const StepParams& p, int a, int o) { return p.d2af[a][o]; }
  __device__ static float d1(const StepParams& p, int a, int o) { return p.c1f[a][o]; }
};

// combine raw level values (already loaded) in double
template <typename Real, int W, int TT>
__device__ inline Vec<Real, W> combine_levels(const double* w, const Vec<Real, W>* raw, bool sync) {
  if (sync) return raw[0];
  Vec<Real, W> r;
#pragma unroll
  for (int j = 0; j < W; ++j) {
    double acc = 0.0;
#pragma unroll
    for (int m = 0; m < TT; ++m) acc += w[m] * static_cast<double>(raw[m].v[j]);
    r.v[j] = static_cast<Real>(acc);
  }
  return r;
}

// SP = 0: time-expanded AT (TT = T levels) or the synchronous arm (TT = 1).
// SP = 1, 2: the space-expanded single-level schemes of the second-order CD
// (first derivative (1,2,2)a, second (2,1,2) or (2,2,2)a), TT = 1, S = the
// strip depth (2 or 3): the CD2 stencil everywhere plus, at a point next to a
// face whose delay is positive, the difference between that scheme's stencil
// and the CD2 one over the S buffer points of level n-k and the own points.
template <typename Real, int S, int V, int D, int KIND, int EQ, int TT, int SP = 0, bool REV = false>
__global__ __launch_bounds__(kB * kB / V) void at_step3d_fast_kernel(StepParams p) {
  static_assert(S <= kHO, "the x halo must fit left of column kHO");
  static_assert(SP == 0 || TT == 1, "the space-expanded schemes combine one level");
  static_assert(TT >= 1 && TT <= kMaxT, "levels per halo value");
  using VR = Vec<Real, V>;
  using Q = Vec<Real, 4>;
  constexpr int NT = kB * kB / V;         // threads
  constexpr int VPR = kB / V;             // vectors per row
  constexpr int ROWS = kB + 2 * S;
  constexpr bool kHist = KIND == kAb2 || KIND == kAb3 || KIND == kRk2;
  constexpr bool kSync = TT == 1 && SP == 0;   // synchronous arm: neighbours' u^n directly
  constexpr int SS = SP != 0 ? 1 : S;     // half-width of the bulk central difference
  __shared__ __align__(16) Real buf[2][ROWS * kRS];
  __shared__ __align__(16) Real zhi_lds[S * kB * kB];   // planes bz .. bz+S-1
  __shared__ double s_w[6 * kMaxT];
  __shared__ int s_slot[6 * kMaxT];
  __shared__ int s_nbr[6];
  __shared__ int s_kpos[6];               // face delay k > 0 (space-expanded stencils apply)

  const int tid = threadIdx.x;
  const int vi = tid % VPR, y = tid / VPR;
  const int x = V * vi;
  const int64_t n = p.counter[0];
  // a downward sweep also takes the PEs in the opposite order, so that when
  // there are more PEs than resident workgroups the launch starts on the PEs
  // the previous one finished last
  const int wg = REV ? static_cast<int>(gridDim.x) - 1 - static_cast<int>(blockIdx.x) : static_cast<int>(blockIdx.x);
  const int pid = pe_of_workgroup(wg, gridDim.x);
  const int bz = p.bz;

  if (tid < 6) {
    const int f = tid;
    s_nbr[f] = neighbour_pe(p, pid, f);
    s_kpos[f] = 0;
    if (!kSync) {
      const int k = face_delay_fast(p, pid, f, n);
      s_kpos[f] = k > 0;
      double w[kMaxT];
      level_weights(k, TT, w);
      // a level whose weight is zero re-reads level n-k (same lines, cache
      // hits) and is multiplied by an exact zero, so every read is issued
      // without a branch
      const int r0 = static_cast<int>(n % p.nslots);
      const int s0 = slot_back(r0, k, p.nslots);
      for (int m = 0; m < kMaxT; ++m) {
        const bool live = m < TT && w[m] != 0.0;
        s_w[f * kMaxT + m] = live ? w[m] : 0.0;
        s_slot[f * kMaxT + m] = live ? slot_back(r0, k + m, p.nslots) : s0;
      }
    }
  }
  __syncthreads();

  const Real* centre = static_cast<const Real*>(KIND == kRk2 ? p.ustar : p.ubuf[n & 1]);
  const Real* ring = static_cast<const Real*>(KIND == kRk2 ? p.sring : p.ring);
  // The field is PE-major ([pe][z][y][x], 32 x 32 x bz values per PE): each
  // plane of the PE is one contiguous block. Offsets fit 32 bits (the host
  // checks the field size).
  const uint32_t pe_size = static_cast<uint32_t>(kB * kB) * bz;
  constexpr uint32_t zstride = kB * kB;
  const uint32_t col = static_cast<uint32_t>(pid) * pe_size + y * kB + x;
  // ring_index of PE-major problems: [face][plane][pe][slot][chunk]
  const int64_t nsl = p.nslots > 0 ? p.nslots : 1;

  // A halo source: one pointer per level to the element of plane 0, a
  // per-plane stride and the level weights. AT: the neighbour's strip in the
  // ring slots of the delayed levels; SYNC: the neighbour's u^n (sync_g: the
  // offset of the value at the PE's plane 0 in the neighbour's block).
  struct Src {
    const Real* lvl[TT];
    double w[TT];
    int64_t stride;
  };
  auto make_src = [&](int f, int64_t q0, int64_t qstride, int64_t sync_g) -> Src {
    Src r;
    if (kSync) {
      r.lvl[0] = centre + sync_g;
      r.w[0] = 1.0;
      r.stride = zstride;
      return r;
    }
    // producer face f ^ 1 of the neighbour (uniform offsets selected, not
    // indexed per lane)
    const int pf = f ^ 1;
    const int64_t foff = pf == 0 ? p.face_off[0] : pf == 1 ? p.face_off[1] : pf == 2 ? p.face_off[2]
                       : pf == 3 ? p.face_off[3] : pf == 4 ? p.face_off[4] : p.face_off[5];
    const int64_t chunk = pf < 4 ? p.face_chunk[0] : p.face_chunk[4];
    const Real* strip = ring + nsl * foff + static_cast<int64_t>(s_nbr[f]) * nsl * chunk + q0;
#pragma unroll
    for (int m = 0; m < TT; ++m) {
      r.lvl[m] = strip + s_slot[f * kMaxT + m] * chunk;
      r.w[m] = s_w[f * kMaxT + m];
    }
    // the next plane of the same strip is npe groups of nslots chunks further
    r.stride = static_cast<int64_t>(p.npe) * nsl * chunk;
    (void)qstride;
    return r;
  };

  // Halo items, all quads so that every thread issues the same reads:
  // x items (side and four consecutive values of the producer strip [z][y][d],
  // i.e. rows and depths (e / S, e % S); the synchronous arm reads rows
  // yq..yq+3 at one depth of the neighbour's field instead) and y items (side,
  // depth d, columns xq..xq+3; strip [z][d][x]). FP32: the items fill the
  // first threads (one wave for s <= 2), so that the other waves skip the
  // FP64 combination (256^3 AT 69.4 -> 68.6 us); FP64: each wave owns a
  // contiguous share of the items in its low lanes (the first form measured
  // 130.3 -> 132.2 us there). Other threads alias item 0 (their reads hit the
  // same lines and are discarded).
  constexpr int QPR = kB / 4;
  constexpr int NHX = 2 * S * QPR;
  constexpr int NH = 2 * NHX;
  constexpr bool kFirst = sizeof(Real) == 4;
  constexpr int NW = NT / 64;
  constexpr int NHW = NH / NW;
  static_assert(kFirst ? NH <= NT : (NH % NW == 0 && NHW <= 64), "halo items per wave");
  const int lane = tid & 63;
  const bool is_h = kFirst ? tid < NH : lane < NHW;
  const int hid = is_h ? (kFirst ? tid : (tid >> 6) * NHW + lane) : 0;
  Src hs;
  int hp[4];                        // LDS positions of the 4 values
  int estride;                      // element stride of the synchronous arm's reads
  if (hid < NHX) {
    const int side = hid / (S * QPR), r = hid % (S * QPR);
    if (kSync) {
      // column xl of this PE's frame is column lx of the x neighbour
      const int d = r / QPR, yq = 4 * (r % QPR);
      const int xl = side ? kB + d : d - S;
      const int lx = side ? d : kB - S + d;
#pragma unroll
      for (int i = 0; i < 4; ++i) hp[i] = (yq + i + S) * kRS + kHO + xl;
      estride = kB;
      hs = make_src(side, 0, 0, static_cast<int64_t>(s_nbr[side]) * pe_size + yq * kB + lx);
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int e = 4 * r + i, y = e / S, d = e - (e / S) * S;
        hp[i] = (y + S) * kRS + kHO + (side ? kB + d : d - S);
      }
      estride = 1;
      hs = make_src(side, static_cast<int64_t>(4) * r, static_cast<int64_t>(S) * kB, 0);
    }
  } else {
    const int h = hid - NHX;
    const int side = h / (S * QPR), r = h % (S * QPR), d = r / QPR, xq = 4 * (r % QPR);
    const int yl = side ? kB + d : d - S;
    const int ly = side ? d : kB - S + d;          // row of the y neighbour
#pragma unroll
    for (int i = 0; i < 4; ++i) hp[i] = (yl + S) * kRS + kHO + xq + i;
    estride = 1;
    hs = make_src(2 + side, static_cast<int64_t>(d) * kB + xq, static_cast<int64_t>(S) * kB,
                  static_cast<int64_t>(s_nbr[2 + side]) * pe_size + ly * kB + xq);
  }
  // raw read of level m of this thread's halo item at plane zz
  auto halo_raw = [&](int zz, int m) -> Q {
    if (!kSync) return ldp<Real, 4>(hs.lvl[m] + zz * hs.stride);
    const Real* b = hs.lvl[0] + zz * hs.stride;
    return Q{{b[0], b[estride], b[2 * estride], b[3 * estride]}};
  };

  // integrator history: f^{n-1} (AB2, AB3), u^n (second RK2 stage). AB3 keeps
  // f^{n-1} in fbuf[(n-1)&1] and f^{n-2} in fbuf[n&1]; f^n overwrites f^{n-2}.
  // The reads are issued unconditionally (a value the formula does not use at
  // start-up is never touched).
  Real* fb0 = static_cast<Real*>(p.fbuf[0]);
  Real* fm1 = KIND == kAb3 ? static_cast<Real*>(p.fbuf[(n + 1) & 1]) : nullptr;
  Real* fm2 = KIND == kAb3 ? static_cast<Real*>(p.fbuf[n & 1]) : nullptr;
  const Real* hist = KIND == kAb2 ? fb0 : KIND == kAb3 ? fm1
                   : KIND == kRk2 ? static_cast<const Real*>(p.ubuf[n & 1]) : nullptr;
  // where f^n goes
  Real* fout = KIND == kAb2 ? fb0
             : KIND == kAb3 ? (n == 0 ? fb0 : n == 1 ? static_cast<Real*>(p.fbuf[1]) : fm2) : nullptr;
  auto hist1 = [&](int z) -> VR { return kHist ? ldv<Real, V>(hist, col + z * zstride) : zerov<Real, V>(); };
  auto hist2 = [&](int z) -> VR { return KIND == kAb3 ? ldv<Real, V>(fm2, col + z * zstride) : zerov<Real, V>(); };

  const Real dt = static_cast<Real>(p.dt);
  Real* unext = static_cast<Real*>(KIND == kRk1 ? p.ustar : p.ubuf[(n + 1) & 1]);
  Real* pub = static_cast<Real*>(KIND == kRk1 ? p.sring : p.ring);
  const int pslot = static_cast<int>((KIND == kRk1 ? n : n + 1) % (p.nslots > 0 ? p.nslots : 1));
  // this PE's strips in the ring slot of the new level (ring_index): plane
  // z of an x or y face at nslots face_off + ((z npe + pid) nslots + slot)
  // chunk, depth d of a z face likewise with plane d
  const int64_t cxy = p.face_chunk[0];             // s * 32 (x and y faces)
  const int64_t cz = p.face_chunk[4];              // 32 * 32 (z faces)
  auto pub_xy = [&](int64_t fo, int zz) -> Real* {
    return pub + nsl * fo + ((static_cast<int64_t>(zz) * p.npe + pid) * nsl + pslot) * cxy;
  };
  auto pub_z = [&](int64_t fo, int d) -> Real* {
    return pub + nsl * fo + ((static_cast<int64_t>(d) * p.npe + pid) * nsl + pslot) * cz;
  };

  // space-expanded schemes: low-face taps minus the CD2 taps, o = -S..S
  Real dl1[3][2 * S + 1], dl2[3][2 * S + 1];
  const Real alpha_r = static_cast<Real>(p.alpha);
  const Real vel[3] = {static_cast<Real>(p.vel[0]), static_cast<Real>(p.vel[1]), static_cast<Real>(p.vel[2])};
  if constexpr (SP != 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int o = -S; o <= S; ++o) {
        const bool in_cd = o >= -1 && o <= 1;
        dl1[a][o + S] = static_cast<Real>(p.sl1[a][o + kMaxS] - (in_cd ? p.c1[a][o + 1] : 0.0));
        dl2[a][o + S] = static_cast<Real>(p.sl2[a][o + kMaxS] - (in_cd ? p.c2[a][o + 1] : 0.0));
      }
  }
  const bool kpos0 = SP != 0 && s_kpos[0], kpos1 = SP != 0 && s_kpos[1], kpos2 = SP != 0 && s_kpos[2],
             kpos3 = SP != 0 && s_kpos[3], kpos4 = SP != 0 && s_kpos[4], kpos5 = SP != 0 && s_kpos[5];
  const int c_at = (y + S) * kRS + kHO + x;     // LDS index of this thread's first point

  // The sweep over the PE's z-planes, upward (REV = false) or downward (the
  // alternating variants: the host alternates the direction from launch to
  // launch, so that a launch starts on the planes the previous one touched
  // last, which are still in the Infinity Cache when the working set exceeds
  // it). Per point the arithmetic is the same in both directions (the z
  // neighbours are taken from the queue by their physical offset), so
  // results are bit-identical.
  {
    // physical plane of sweep position zs
    auto phys = [&](int zs) { return REV ? bz - 1 - zs : zs; };
    // The 2S planes beyond the PE's z faces (strip [d][y][x]) are loaded and
    // combined once, before the sweep: the S planes the sweep starts beyond
    // into registers, the S planes it ends beyond into LDS (picked by a
    // run-time plane index). Sweep position -S + i holds depth i of the low
    // strip (upward) or depth S-1-i of the high strip (downward); position
    // bz + e holds depth e of the high strip or depth S-1-e of the low one.
    VR zst[S];
    {
      // synchronous arm: the last S planes of the low z neighbour, the first
      // S of the high one (bz >= 2s, checked at creation)
      const int64_t q0 = static_cast<int64_t>(y) * kB + x;
      const Src lo = make_src(4, q0, static_cast<int64_t>(kB) * kB,
                              static_cast<int64_t>(s_nbr[4]) * pe_size + (bz - S) * zstride + q0);
      const Src hi = make_src(5, q0, static_cast<int64_t>(kB) * kB, static_cast<int64_t>(s_nbr[5]) * pe_size + q0);
#pragma unroll
      for (int d = 0; d < S; ++d) {
        VR rl[TT], rh[TT];
#pragma unroll
        for (int m = 0; m < TT; ++m) {
          rl[m] = ldp<Real, V>(lo.lvl[m] + d * lo.stride);
          rh[m] = ldp<Real, V>(hi.lvl[m] + d * hi.stride);
        }
        const VR cl = combine_levels<Real, V, TT>(lo.w, rl, kSync);
        const VR ch = combine_levels<Real, V, TT>(hi.w, rh, kSync);
        zst[REV ? S - 1 - d : d] = REV ? ch : cl;
        stv<Real, V>(zhi_lds, static_cast<uint32_t>(((REV ? S - 1 - d : d) * kB + y) * kB + x), REV ? cl : ch);
      }
    }
    // values of sweep position zs in [0, bz + S): the PE's planes from u^n,
    // the last S from LDS (each thread reads back what it wrote)
    auto plane_vec = [&](int zs) -> VR {
      if (zs < bz) return ldv<Real, V>(centre, col + phys(zs) * zstride);
      return ldv<Real, V>(zhi_lds, static_cast<uint32_t>(((zs - bz) * kB + y) * kB + x));
    };

    // z queue (sweep positions zs-S .. zs+S) and the rotating prefetch slots
    VR qz[2 * S + 1];
#pragma unroll
    for (int i = 0; i < S; ++i) qz[i] = zst[i];
#pragma unroll
    for (int i = 0; i < S; ++i) qz[S + i] = plane_vec(i);
    VR A[D], F1[D], F2[D];
    Q HR[D][TT];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      A[j] = plane_vec(j + S);
      F1[j] = hist1(phys(j));
      F2[j] = hist2(phys(j));
#pragma unroll
      for (int m = 0; m < TT; ++m) HR[j][m] = halo_raw(phys(j), m);
    }
    // z neighbour at physical offset -o / +o of the current plane
    auto zlow = [&](int o) -> const VR& { return REV ? qz[S + o] : qz[S - o]; };
    auto zhigh = [&](int o) -> const VR& { return REV ? qz[S - o] : qz[S + o]; };

    for (int zb = 0; zb < bz; zb += D) {
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const int zs = zb + j;
        const int z = phys(zs);
        qz[2 * S] = A[j];
        const VR fo1 = F1[j], fo2 = F2[j];
        Real* Lp = buf[zs & 1];
        stv<Real, V>(Lp, static_cast<uint32_t>(c_at), qz[S]);
        if (is_h) {
          const Q hv = combine_levels<Real, 4, TT>(hs.w, HR[j], kSync);
#pragma unroll
          for (int i = 0; i < 4; ++i) Lp[hp[i]] = hv.v[i];
        }
        // refill the slot with what sweep position zs + D consumes
        if (zs + D < bz) {
          A[j] = plane_vec(zs + D + S);
          F1[j] = hist1(phys(zs + D));
          F2[j] = hist2(phys(zs + D));
#pragma unroll
          for (int m = 0; m < TT; ++m) HR[j][m] = halo_raw(phys(zs + D), m);
        }
        __syncthreads();
        // x row segment [x - S, x + V - 1 + S] and the y neighbour vectors
        Real row[V + 2 * S];
#pragma unroll
        for (int i = 0; i < V + 2 * S; ++i) row[i] = Lp[c_at - S + i];
        VR ym[S], yp[S];
#pragma unroll
        for (int o = 1; o <= S; ++o) {
          ym[o - 1] = ldv<Real, V>(Lp, static_cast<uint32_t>(c_at - o * kRS));
          yp[o - 1] = ldv<Real, V>(Lp, static_cast<uint32_t>(c_at + o * kRS));
        }
        VR un, fq;
#pragma unroll
        for (int e = 0; e < V; ++e) {
          const Real u0 = qz[S].v[e];
          Real fval;
          if (EQ == AT_ADVDIFF) {
            // f = sum over axes and taps of (alpha c2 - vel c1) (v - u0), one
            // partial sum per axis
            Real ax = 0, ay = 0, az = 0;
#pragma unroll
            for (int o = 1; o <= SS; ++o) {
              ax += Taps<Real>::kad(p, 0, SS - o) * (row[S + e - o] - u0);
              ay += Taps<Real>::kad(p, 1, SS - o) * (ym[o - 1].v[e] - u0);
              az += Taps<Real>::kad(p, 2, SS - o) * (zlow(o).v[e] - u0);
              ax += Taps<Real>::kad(p, 0, SS + o) * (row[S + e + o] - u0);
              ay += Taps<Real>::kad(p, 1, SS + o) * (yp[o - 1].v[e] - u0);
              az += Taps<Real>::kad(p, 2, SS + o) * (zhigh(o).v[e] - u0);
            }
            fval = (ax + ay) + az;
          } else {
            // f = alpha lap u - u (sum_d du/dx_d)
            Real lx = 0, ly = 0, lz = 0, gx = 0, gy = 0, gz = 0;
#pragma unroll
            for (int o = 1; o <= SS; ++o) {
              const Real xm = row[S + e - o] - u0, xp = row[S + e + o] - u0;
              const Real ymv = ym[o - 1].v[e] - u0, ypv = yp[o - 1].v[e] - u0;
              const Real zm = zlow(o).v[e] - u0, zp = zhigh(o).v[e] - u0;
              lx += Taps<Real>::d2a(p, 0, SS - o) * xm + Taps<Real>::d2a(p, 0, SS + o) * xp;
              ly += Taps<Real>::d2a(p, 1, SS - o) * ymv + Taps<Real>::d2a(p, 1, SS + o) * ypv;
              lz += Taps<Real>::d2a(p, 2, SS - o) * zm + Taps<Real>::d2a(p, 2, SS + o) * zp;
              gx += Taps<Real>::d1(p, 0, SS - o) * xm + Taps<Real>::d1(p, 0, SS + o) * xp;
              gy += Taps<Real>::d1(p, 1, SS - o) * ymv + Taps<Real>::d1(p, 1, SS + o) * ypv;
              gz += Taps<Real>::d1(p, 2, SS - o) * zm + Taps<Real>::d1(p, 2, SS + o) * zp;
            }
            fval = ((lx + ly) + lz) - u0 * ((gx + gy) + gz);
          }
          if constexpr (SP != 0) {
            // space-expanded stencils at points next to a face with k > 0: the
            // difference to the CD2 taps, over o = -S..S (the high face mirrors
            // the low-face taps: first derivative odd, second even)
            Real c1s = 0, c2s = 0, adv = 0;
            auto add_axis = [&](int a, bool lo, bool hi, auto val) {
              if (!(lo || hi)) return;
              Real t1 = 0, t2 = 0;
#pragma unroll
              for (int o = -S; o <= S; ++o) {
                if (o == 0) continue;
                const Real v = val(o) - u0;
                t1 += (lo ? dl1[a][o + S] : -dl1[a][S - o]) * v;
                t2 += (lo ? dl2[a][o + S] : dl2[a][S - o]) * v;
              }
              c1s += EQ == AT_ADVDIFF ? Real(0) : t1;
              adv += EQ == AT_ADVDIFF ? vel[a] * t1 : Real(0);
              c2s += t2;
            };
            add_axis(0, e == 0 && x == 0 && kpos0, e == V - 1 && x + e == kB - 1 && kpos1,
                     [&](int o) { return row[S + e + o]; });
            add_axis(1, y == 0 && kpos2, y == kB - 1 && kpos3,
                     [&](int o) { return o < 0 ? ym[-o - 1].v[e] : yp[o - 1].v[e]; });
            add_axis(2, z == 0 && kpos4, z == bz - 1 && kpos5,
                     [&](int o) { return o < 0 ? zlow(-o).v[e] : o > 0 ? zhigh(o).v[e] : qz[S].v[e]; });
            fval += EQ == AT_ADVDIFF ? alpha_r * c2s - adv : alpha_r * c2s - u0 * c1s;
          }
          fq.v[e] = fval;
          Real r;
          if (KIND == kRk1 || KIND == kEuler) {
            r = u0 + dt * fval;
          } else if (KIND == kRk2) {
            r = Real(0.5) * (fo1.v[e] + u0) + (Real(0.5) * dt) * fval;
          } else if (KIND == kAb2) {
            r = n == 0 ? u0 + dt * fval : u0 + dt * (Real(1.5) * fval - Real(0.5) * fo1.v[e]);
          } else {   // AB3: Euler, then AB2, then AB3
            r = n == 0 ? u0 + dt * fval
              : n == 1 ? u0 + dt * (Real(1.5) * fval - Real(0.5) * fo1.v[e])
                       : u0 + dt * ((Real(23) * fval - Real(16) * fo1.v[e] + Real(5) * fo2.v[e]) / Real(12));
          }
          un.v[e] = r;
        }
        const uint32_t g = col + z * zstride;
        stv<Real, V>(unext, g, un);
        if (KIND == kAb2 || KIND == kAb3) stv<Real, V>(fout, g, fq);
        if (!kSync) {
          // publish the new edge values into the ring slot of their level;
          // x faces: plane [y][d], one run of s values per row
          const int xrow = y * S;
          if constexpr (V == 4) {
            // the first quad of a row holds the low-face depths, the last one
            // the high-face depths: one store of s values for both faces
            const bool lo = vi == 0, hi = vi == VPR - 1;
            if (lo || hi) {
              Real w[S];
#pragma unroll
              for (int d = 0; d < S; ++d) w[d] = hi ? un.v[V - S + d] : un.v[d];
              // (select between the two uniform offsets: an index that varies
              // per lane would turn the kernel-argument read into a memory load)
              const int64_t fo = hi ? p.face_off[1] : p.face_off[0];
              st_run<Real, S>(pub_xy(fo, z) + xrow, w);
            }
          } else {
#pragma unroll
            for (int e = 0; e < V; ++e) {
              if (x + e < S) pub_xy(p.face_off[0], z)[xrow + x + e] = un.v[e];
              if (x + e >= kB - S) pub_xy(p.face_off[1], z)[xrow + x + e - (kB - S)] = un.v[e];
            }
          }
          // y faces: plane [d][x]; rows 0..s-1 and kB-s..kB-1, one store
          if (y < S || y >= kB - S) {
            const int64_t fo = y < S ? p.face_off[2] : p.face_off[3];
            const int d = y < S ? y : y - (kB - S);
            stv<Real, V>(pub_xy(fo, z), static_cast<uint32_t>(d * kB + x), un);
          }
          // z faces: depth plane [y][x]
          if (z < S) stv<Real, V>(pub_z(p.face_off[4], z), static_cast<uint32_t>(y * kB + x), un);
          if (z >= bz - S) stv<Real, V>(pub_z(p.face_off[5], z - (bz - S)), static_cast<uint32_t>(y * kB + x), un);
        }
#pragma unroll
        for (int i = 0; i < 2 * S; ++i) qz[i] = qz[i + 1];
      }
    }
  }

  if (KIND != kRk1) {
    // every workgroup has read n before its own increment
    __syncthreads();
    if (tid == 0) advance_counter(p.counter, n);
  }
}

template <typename Real, int S, int V, int D, int KIND, int TT, int SP, bool REV>
hipError_t launch_dir(const StepParams& p, hipStream_t st) {
  constexpr int NT = kB * kB / V;
  if (p.equation == AT_ADVDIFF)
    hipLaunchKernelGGL((at_step3d_fast_kernel<Real, S, V, D, KIND, AT_ADVDIFF, TT, SP, REV>), dim3(p.npe),
                       dim3(NT), 0, st, p);
  else
    hipLaunchKernelGGL((at_step3d_fast_kernel<Real, S, V, D, KIND, AT_BURGERS, TT, SP, REV>), dim3(p.npe),
                       dim3(NT), 0, st, p);
  return hipGetLastError();
}

// ALT: the launch's sweep direction comes from p.sweep_down.
template <typename Real, int S, int V, int D, int KIND, int TT, int SP = 0, bool ALT = false>
hipError_t launch_eq(const StepParams& p, hipStream_t st) {
  if (ALT && p.sweep_down) return launch_dir<Real, S, V, D, KIND, TT, SP, true>(p, st);
  return launch_dir<Real, S, V, D, KIND, TT, SP, false>(p, st);
}

// The synchronous arm reads one value per halo point; the AT schemes read the
// T = s + 1 delayed levels of the time-expanded family.
template <typename Real, int S, int V, int D, int KIND, bool ALT>
hipError_t launch_kind(const StepParams& p, hipStream_t st) {
  if (p.mode == AT_SYNC) return launch_eq<Real, S, V, D, KIND, 1, 0, ALT>(p, st);
  return launch_eq<Real, S, V, D, KIND, S + 1, 0, ALT>(p, st);
}

template <typename Real, int S, int V, int D, bool ALT = false>
hipError_t launch_fast_d(const StepParams& p, hipStream_t st) {
  if (p.stage == kStageRk1) return launch_kind<Real, S, V, D, kRk1, ALT>(p, st);
  if (p.stage == kStageRk2) return launch_kind<Real, S, V, D, kRk2, ALT>(p, st);
  switch (p.integrator) {
    case AT_EULER: return launch_kind<Real, S, V, D, kEuler, ALT>(p, st);
    case AT_AB2: return launch_kind<Real, S, V, D, kAb2, ALT>(p, st);
    case AT_AB3: return launch_kind<Real, S, V, D, kAb3, ALT>(p, st);
  }
  return hipErrorInvalidValue;
}

// Schedule variants (the tunables of this path): planes of reads in flight
// D in {1, 2, 4} and points per thread V in {2, 4}, encoded as
// variant = D for V = 4 and 8 + D for V = 2, and 16 + D for V = 4 with the
// z sweep direction alternating from launch to launch. All variants compute
// bit-identical results.
template <typename Real, int S>
hipError_t launch_fast_t(const StepParams& p, hipStream_t st) {
  switch (p.depth) {
    case 1: return launch_fast_d<Real, S, 4, 1>(p, st);
    case 2: return launch_fast_d<Real, S, 4, 2>(p, st);
    case 4: return launch_fast_d<Real, S, 4, 4>(p, st);
    case 9: return launch_fast_d<Real, S, 2, 1>(p, st);
    case 10: return launch_fast_d<Real, S, 2, 2>(p, st);
    case 12: return launch_fast_d<Real, S, 2, 4>(p, st);
    case 17: return launch_fast_d<Real, S, 4, 1, true>(p, st);
    case 18: return launch_fast_d<Real, S, 4, 2, true>(p, st);
    case 20: return launch_fast_d<Real, S, 4, 4, true>(p, st);
  }
  return hipErrorInvalidValue;
}

// The space-expanded schemes (one level, strips S = 2 or 3 deep): schedule
// variants 1 and 2 (V = 4, D = 1 or 2).
template <typename Real, int S, int SP, int D>
hipError_t launch_space_d(const StepParams& p, hipStream_t st) {
  if (p.stage == kStageRk1) return launch_eq<Real, S, 4, D, kRk1, 1, SP>(p, st);
  if (p.stage == kStageRk2) return launch_eq<Real, S, 4, D, kRk2, 1, SP>(p, st);
  switch (p.integrator) {
    case AT_EULER: return launch_eq<Real, S, 4, D, kEuler, 1, SP>(p, st);
    case AT_AB2: return launch_eq<Real, S, 4, D, kAb2, 1, SP>(p, st);
    case AT_AB3: return launch_eq<Real, S, 4, D, kAb3, 1, SP>(p, st);
  }
  return hipErrorInvalidValue;
}

template <typename Real>
hipError_t launch_space_t(const StepParams& p, hipStream_t st) {
  const int key = p.scheme * 10 + p.depth;
  switch (key) {
    case 11: return launch_space_d<Real, 2, 1, 1>(p, st);
    case 12: return launch_space_d<Real, 2, 1, 2>(p, st);
    case 21: return launch_space_d<Real, 3, 2, 1>(p, st);
    case 22: return launch_space_d<Real, 3, 2, 2>(p, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace fast3d

// one instantiation per translation unit (fast3d_*.hip), built in parallel
hipError_t launch_fast3d_f32_s1(const StepParams& p, hipStream_t st);
hipError_t launch_fast3d_f32_s2(const StepParams& p, hipStream_t st);
hipError_t launch_fast3d_f32_s3(const StepParams& p, hipStream_t st);
hipError_t launch_fast3d_f64_s1(const StepParams& p, hipStream_t st);
hipError_t launch_fast3d_f64_s2(const StepParams& p, hipStream_t st);
hipError_t launch_fast3d_f64_s3(const StepParams& p, hipStream_t st);
hipError_t launch_fast3d_space_f32(const StepParams& p, hipStream_t st);
hipError_t launch_fast3d_space_f64(const StepParams& p, hipStream_t st);

}  // namespace atfd
