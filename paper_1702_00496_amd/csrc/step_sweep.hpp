// Device side of the generic AT sweep (any PE shape, 1-D/2-D/3-D): the
// per-workgroup sweep state, face set-up and the kernels. Shared by the
// scalar instantiations in step.hip and the vector ones in step_vec_*.hip.
#pragma once

#include "atfd_internal.hpp"
#include "delays.hpp"

namespace atfd {
namespace sweep {

// LDS plane slot of z-plane zz (zz >= -S). 3-D sweeps keep 2S+2 planes: the
// 2S+1 planes of the current stencil plus the one being filled, so a single
// barrier per plane separates reads from overwrites.
template <int DIM, int S>
__device__ inline int slot_of(int zz) {
  return DIM == 3 ? (zz + S) % (2 * S + 2) : 0;
}

// Parts of an LDS plane: the PE's own values and the x/y halo frame.
constexpr int kPlaneCentre = 1, kPlaneHalos = 2;

// SP: 0 = time-expanded AT (or the standard scheme); 1, 2 = the
// space-expanded single-level schemes with the second derivative (2,1,2) or
// (2,2,2)a and the first (1,2,2)a (second-order CD only); 3 = the
// non-uniform-delay scheme (Sec. 3.4 Example 1) whose two buffer points carry
// their own delays. SD = depth of the face strips and of the LDS halo frame:
// s, or the 2 or 3 buffer points the single-level stencils reach.
template <int S, int SP>
constexpr int strip_depth() {
  return SP == 0 ? S : SP == 2 ? 3 : 2;
}

// Part of a PE a workgroup of the sweep takes: PE pid, z-chunk ci of nch,
// y-slice ys. 3-D grids whose size is a multiple of the 8 XCDs are
// renumbered so that consecutive logical indices run on one XCD (the
// dispatcher places workgroup b on XCD b mod 8) and the chunks of a PE come
// first, then its neighbours along x: the planes a chunk reloads from the
// next one, and the cache lines PEs share at their x edges when a PE row is
// not a multiple of 128 bytes, stay in one L2.
struct SweepPart {
  int pid, ci, ys, nch;
};
template <int DIM>
__device__ inline SweepPart sweep_part(const StepParams& p) {
  const int g = static_cast<int>(gridDim.x), b = static_cast<int>(blockIdx.x);
  const int nys = p.yslices > 1 ? p.yslices : 1;
  SweepPart r;
  r.nch = g / (p.npe * nys);
  const int L = DIM == 3 && g % 8 == 0 ? (b % 8) * (g / 8) + b / 8 : b;
  r.ci = L % r.nch;
  r.pid = (L / r.nch) % p.npe;
  r.ys = L / (r.nch * p.npe);
  return r;
}

// Per-face taps of the non-uniform scheme, [face][derivative][o + 2]
constexpr int kNuTaps = 10;

// Per-face table of the vector path's face correction: [face][o + 3] first
// derivative, [face][7 + o + 3] second, o = -3..3
constexpr int kDtaps = 14;

// Stage of the time integrator a vector-path kernel is specialised on.
enum VKind : int { kVEuler = 0, kVAb2 = 1, kVAb3 = 2, kVRk1 = 3, kVRk2 = 4 };

// Four consecutive values (one thread's points of a row in the vector path).
template <typename Real>
struct Vec4 {
  Real v[4];
};
template <typename Real>
__device__ inline Vec4<Real> ld4(const Real* p) {
  Vec4<Real> r;
  if constexpr (sizeof(Real) == 4) {
    const float4 t = *reinterpret_cast<const float4*>(p);
    r.v[0] = t.x; r.v[1] = t.y; r.v[2] = t.z; r.v[3] = t.w;
  } else {
    const double2 a = *reinterpret_cast<const double2*>(p);
    const double2 b = *reinterpret_cast<const double2*>(p + 2);
    r.v[0] = a.x; r.v[1] = a.y; r.v[2] = b.x; r.v[3] = b.y;
  }
  return r;
}
template <typename Real>
__device__ inline void st4(Real* p, const Vec4<Real>& q) {
  if constexpr (sizeof(Real) == 4) {
    *reinterpret_cast<float4*>(p) = make_float4(q.v[0], q.v[1], q.v[2], q.v[3]);
  } else {
    *reinterpret_cast<double2*>(p) = make_double2(q.v[0], q.v[1]);
    *reinterpret_cast<double2*>(p + 2) = make_double2(q.v[2], q.v[3]);
  }
}

// VEC: the vector layout and path (PE x edge a multiple of 4): LDS rows of
// bx + 8 values with x = 0 at column 4, so that the 4 consecutive points a
// thread owns are one aligned LDS vector and one 16-byte global access.
template <typename Real, int DIM, int S, int SP, bool VEC = false>
struct Sweep {
  static constexpr int SD = strip_depth<S, SP>();
  static constexpr int NSL = DIM == 3 ? 2 * SD + 2 : 1;
  static constexpr int kBatch = 4;   // points per thread whose loads are issued together

  const StepParams& p;
  Real* lds;
  int pid, qx, qy, qz, x0, y0, z0;
  int px_stride, plane;     // LDS row stride and plane size
  int co;                   // LDS column of x = 0
  int yl0, rows_sl;         // the workgroup's y-slice of the PE: first row, rows
  int64_t n;
  const Real* centre;       // field whose level-n values feed the stencil
  const Real* ring_rd;      // ring the halos come from
  // per-face delay data (AT) in LDS
  const double* w;          // [6][kMaxT]
  const int* lev_slot;      // [6][kMaxT] ring slot of level n-k-m, -1 if weight 0
  const int* nbr;           // [6] neighbour PE of face
  const int* kpos;          // [6] face delay k > 0 (space-expanded stencils apply)
  const Real* nut;          // [6][kNuTaps] non-uniform taps (SP = 3), in the storage type
  const Real* dtap;         // [6][kDtaps] face stencil minus the CD2 taps (SP != 0, faces with kpos)

  __device__ Sweep(const StepParams& p_, Real* lds_, int64_t n_, const double* w_,
                   const int* ls_, const int* nb_, const int* kp_, const Real* nu_, const Real* dt_)
      : p(p_), lds(lds_), n(n_), w(w_), lev_slot(ls_), nbr(nb_), kpos(kp_), nut(nu_), dtap(dt_) {
    pid = sweep_part<DIM>(p).pid;
    qx = pid % p.px;
    qy = (pid / p.px) % p.py;
    qz = pid / (p.px * p.py);
    x0 = qx * p.bx;
    y0 = qy * p.by;
    z0 = qz * p.bz;
    co = VEC ? 4 : SD;
    px_stride = VEC ? p.bx + 8 : p.bx + 2 * SD;
    yl0 = 0;
    rows_sl = p.by;
    plane = (DIM >= 2 ? p.by + 2 * SD : 1) * px_stride;
    const bool rk2 = p.stage == kStageRk2;
    centre = static_cast<const Real*>(rk2 ? p.ustar : p.ubuf[n & 1]);
    ring_rd = static_cast<const Real*>(rk2 ? p.sring : p.ring);
  }

  // Slice ys of nys equal y-slices (3-D pipelined sweep): the workgroup's
  // LDS planes then hold its rows and the SD rows on either side, which come
  // from the PE's own level-n values where the slice edge is inside the PE.
  __device__ void set_slice(int ys, int nys) {
    rows_sl = p.by / nys;
    yl0 = ys * rows_sl;
    plane = (rows_sl + 2 * SD) * px_stride;
  }

  // v mod n for v in [-n, 2n): a periodic index one strip depth outside the box
  static __device__ int wrap(int v, int n) {
    v = v < 0 ? v + n : v;
    return v >= n ? v - n : v;
  }

  __device__ int64_t gidx(int x, int y, int z) const {
    return (static_cast<int64_t>(z) * p.ny + y) * p.nx + x;
  }

  // Offset of element r of plane `plane` of face `face`'s strip of PE `pe`
  // in ring slot `slot` (x and y strips: plane z; z strips: plane d). The
  // face may differ between lanes: its offset and chunk are selected from
  // the uniform values rather than indexed.
  __device__ int64_t ring_off(int slot, int pe, int face, int plane, int r) const {
    const int64_t fo = face == 0 ? p.face_off[0] : face == 1 ? p.face_off[1] : face == 2 ? p.face_off[2]
                     : face == 3 ? p.face_off[3] : face == 4 ? p.face_off[4] : p.face_off[5];
    const int64_t ch = face < 2 ? p.face_chunk[0] : face < 4 ? p.face_chunk[2] : p.face_chunk[4];
    return static_cast<int64_t>(slot) * p.npe * p.pe_block + fo + (static_cast<int64_t>(plane) * p.npe + pe) * ch + r;
  }

  // Halo value across face f = 2*axis + side, element r of plane `plane` of
  // the producer strip; m = the buffer point's distance from the face - 1.
  // AT: sum over the T delayed levels, in double. SYNC: the neighbour's
  // level-n value at global position (gx, gy, gz). Non-uniform scheme: the
  // single level of buffer point m. halo_raw issues the loads, halo_sum
  // combines them, so that a pipelined sweep can load a plane's halo values
  // one plane ahead of their combination.
  __device__ void halo_raw(int f, int plane, int r, int m, int gx, int gy, int gz, Real (&v)[kMaxT]) const {
    if (p.mode == AT_SYNC) {
      v[0] = centre[gidx(gx, gy, gz)];
      return;
    }
    const int pf = f ^ 1;   // producer face: the opposite side
    const int nb = nbr[f];
    if constexpr (SP == 3) {
      v[0] = ring_rd[ring_off(lev_slot[f * kMaxT + m], nb, pf, plane, r)];
      return;
    }
    // every level is loaded from an in-range slot so that the T loads are in
    // flight together; a level beyond T or of weight zero (k = 0: exact
    // synchronous value) re-reads level 0 (a cache hit) and is then dropped
    // by the select
    const int64_t base = ring_off(0, nb, pf, plane, r);
    const int64_t slot_stride = static_cast<int64_t>(p.npe) * p.pe_block;
    const int s0 = lev_slot[f * kMaxT] > 0 ? lev_slot[f * kMaxT] : 0;
#pragma unroll
    for (int mm = 0; mm < kMaxT; ++mm) {
      const int sl = lev_slot[f * kMaxT + mm];
      v[mm] = ring_rd[base + (mm < p.T && sl >= 0 ? sl : s0) * slot_stride];
    }
  }
  __device__ Real halo_sum(int f, const Real (&v)[kMaxT]) const {
    if (p.mode == AT_SYNC || SP == 3) return v[0];
    double acc = 0.0;
#pragma unroll
    for (int m = 0; m < kMaxT; ++m) {
      const int sl = lev_slot[f * kMaxT + m];
      if (m < p.T && sl >= 0) acc += w[f * kMaxT + m] * static_cast<double>(v[m]);
    }
    return static_cast<Real>(acc);
  }
  __device__ Real halo(int f, int plane, int r, int m, int gx, int gy, int gz) const {
    Real v[kMaxT];
    halo_raw(f, plane, r, m, gx, gy, gz, v);
    return halo_sum(f, v);
  }

  // Item h < 2 SD (by + bx) of an in-box plane's x/y halo frame: the x halos
  // (producer strip [z][y][d]) first, then the y halos (producer strip
  // [z][d][x]). at = LDS offset in the plane, f = face, r = element of the
  // producer strip's plane, m = distance from the face - 1, (gx, gy) = the
  // global position (synchronous arm; and the y halos of a y-slice whose edge
  // is inside the PE, inner: the PE's own level-n values). Rows are those of
  // the workgroup's y-slice.
  struct HaloItem {
    int at, f, r, m, gx, gy;
    bool inner;
  };
  __device__ HaloItem halo_item(int h) const {
    const int bx = p.bx, by = rows_sl;
    const int nxh = 2 * SD * by;
    HaloItem it;
    it.inner = false;
    if (h < nxh) {
      const int side = h >= SD * by ? 1 : 0, r = side ? h - SD * by : h, d = r % SD, y = r / SD;
      const int xl = side ? bx + d : d - SD;
      it.at = (DIM >= 2 ? y + SD : 0) * px_stride + xl + co;
      it.f = side;
      it.r = (yl0 + y) * SD + d;
      it.m = side ? d : SD - 1 - d;
      it.gx = wrap(x0 + xl, p.nx);
      it.gy = y0 + yl0 + y;
    } else {
      const int hy = h - nxh;
      const int side = hy >= SD * bx ? 1 : 0;
      int x = side ? hy - SD * bx : hy, d = 0;   // x = r % bx, d = r / bx < SD
#pragma unroll
      for (int i = 1; i < SD; ++i) {
        if (x >= bx) {
          x -= bx;
          ++d;
        }
      }
      const int yl = side ? by + d : d - SD;
      it.at = (yl + SD) * px_stride + x + co;
      it.f = 2 + side;
      it.r = d * bx + x;
      it.m = side ? d : SD - 1 - d;
      it.gx = x0 + x;
      it.gy = wrap(y0 + yl0 + yl, p.ny);
      it.inner = side ? yl0 + by < p.by : yl0 > 0;
    }
    return it;
  }

  // Point i = tid + k nt of a bx * by plane as (x, y), stepped from k to k + 1
  // without a division.
  struct PlaneIter {
    int x, y, dx, dy, bx;
    __device__ PlaneIter(int tid, int nt, int bx_) : bx(bx_) {
      x = tid % bx;
      y = tid / bx;
      dx = nt % bx;
      dy = nt / bx;
    }
    __device__ void next() {
      x += dx;
      y += dy;
      if (x >= bx) {
        x -= bx;
        ++y;
      }
    }
  };

  __device__ __forceinline__ void load_plane(int zz, int parts = kPlaneCentre | kPlaneHalos) {
    Real* P = lds + slot_of<DIM, SD>(zz) * plane;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int bx = p.bx, by = rows_sl, bz = p.bz;
    if (zz >= 0 && zz < bz) {
      const int gz = z0 + zz;
      // kBatch loads per thread are issued before any LDS write, from
      // clamped (in-range) addresses
      if (VEC && (parts & kPlaneCentre)) {
        // quads: one aligned 16-byte (FP32) or 32-byte (FP64) access each,
        // kBatch of them in flight per thread before the LDS stores
        const Real* cz = centre + gidx(x0, y0 + yl0, gz);
        const int qpr = bx >> 2;
        PlaneIter it(tid, nt, qpr);
        const int rows = DIM >= 2 ? by : 1;
        while (it.y < rows) {
          Vec4<Real> v[kBatch];
          int at[kBatch];
#pragma unroll
          for (int k = 0; k < kBatch; ++k) {
            const bool in = it.y < rows;
            v[k] = ld4<Real>(cz + static_cast<int64_t>(in ? it.y : rows - 1) * p.nx + 4 * (in ? it.x : qpr - 1));
            at[k] = in ? (DIM >= 2 ? it.y + SD : 0) * px_stride + 4 * it.x + co : -1;
            it.next();
          }
#pragma unroll
          for (int k = 0; k < kBatch; ++k)
            if (at[k] >= 0) st4<Real>(P + at[k], v[k]);
        }
      } else if (parts & kPlaneCentre) {
        const Real* cz = centre + gidx(x0, y0 + yl0, gz);
        PlaneIter it(tid, nt, bx);
        while (it.y < by) {
          Real v[kBatch];
          int at[kBatch];
#pragma unroll
          for (int k = 0; k < kBatch; ++k) {
            const bool in = it.y < by;
            v[k] = cz[static_cast<int64_t>(in ? it.y : by - 1) * p.nx + (in ? it.x : bx - 1)];
            at[k] = in ? (DIM >= 2 ? it.y + SD : 0) * px_stride + it.x + co : -1;
            it.next();
          }
#pragma unroll
          for (int k = 0; k < kBatch; ++k)
            if (at[k] >= 0) P[at[k]] = v[k];
        }
      }
      // x halos and y halos in one pass, so that their loads overlap
      const int nh = (parts & kPlaneHalos) ? 2 * SD * by + (DIM >= 2 ? 2 * SD * bx : 0) : 0;
      for (int h = tid; h < nh; h += nt) {
        const HaloItem hi = halo_item(h);
        P[hi.at] = hi.inner ? centre[gidx(hi.gx, hi.gy, gz)] : halo(hi.f, zz, hi.r, hi.m, hi.gx, hi.gy, gz);
      }
    } else {
      // z halo plane: producer strip [d][y][x]
      const int side = zz < 0 ? 0 : 1;
      const int d = side ? zz - bz : zz + SD;
      const int gz = wrap(z0 + zz, p.nz);
      for (PlaneIter it(tid, nt, bx); it.y < by; it.next()) {
        const int x = it.x, y = it.y;
        P[(y + SD) * px_stride + x + co] =
            halo(4 + side, d, (yl0 + y) * bx + x, side ? d : SD - 1 - d, x0 + x, y0 + yl0 + y, gz);
      }
    }
  }

  // Previous-level fields the update of a vector-path stage reads: pre_a
  // (f^{n-1}, or u^n for the second Heun stage), pre_b (f^{n-2}, AB3 from
  // n = 2); any = whether the stage reads one at all.
  template <int KIND>
  __device__ void history(const Real*& pre_a, const Real*& pre_b, bool& any, bool& ab3) const {
    const bool ab = (KIND == kVAb2 || KIND == kVAb3) && n > 0;
    ab3 = KIND == kVAb3 && n >= 2;
    any = KIND == kVRk2 || ab;
    pre_a = static_cast<const Real*>(KIND == kVRk2 ? p.ubuf[n & 1] : ab3 ? p.fbuf[(n - 1) & 1] : p.fbuf[0]);
    pre_b = static_cast<const Real*>(p.fbuf[n & 1]);
  }

  // Pipelined 3-D vector sweep. The global loads of a plane (the thread's
  // quad of u, the kMaxT raw delayed levels of its halo item, its history
  // quads) are issued one plane ahead into registers and written to LDS
  // (the halo levels combined) when the plane enters the stencil, so that
  // their latency overlaps the stencil work of the plane before. Every
  // thread owns at most one quad and one halo item of a plane (the 3-D
  // workgroup has as many threads as the larger count, up to 768: cross-
  // sections, or y-slices of them, of up to 768 quads). Addresses are fixed
  // per thread and advance
  // by a plane stride; loads go to clamped in-box planes and lanes, with no
  // branch around them (a level beyond T or of weight zero re-reads level
  // 0, a cache hit, and is dropped by the combination), and a load whose
  // plane lies beyond the PE's high z face is not used (that plane comes
  // from the z strips).
  struct PipeAddr {
    const Real* c;           // the thread's quad of u at plane 0
    const Real* h[kMaxT];    // its halo item's levels at plane 0
    int64_t hstride;         // halo plane stride
    const Real* a;           // history quads at plane 0
    const Real* b;
    int c_at, h_at;          // LDS offsets (-1: none)
    int hf;                  // the halo item's face (-1: a single level-n value)
  };
  struct Prefetch {
    Vec4<Real> c, pa, pb;
    Real hv[kMaxT];
  };
  template <int KIND>
  __device__ void pipe_setup(PipeAddr& pa) const {
    const int tid = threadIdx.x;
    const int qpr = p.bx >> 2, quads = qpr * rows_sl;
    const int q = tid < quads ? tid : quads - 1;
    const int qy = q / qpr, qx = q - qy * qpr;
    const int64_t g0 = gidx(x0 + 4 * qx, y0 + yl0 + qy, z0);
    pa.c = centre + g0;
    pa.c_at = tid < quads ? (qy + SD) * px_stride + 4 * qx + co : -1;
    const Real *ha, *hb;
    bool any, ab3;
    history<KIND>(ha, hb, any, ab3);
    pa.a = ha + g0;
    pa.b = hb + g0;
    const int nh = 2 * SD * (rows_sl + p.bx);
    const HaloItem hi = halo_item(tid < nh ? tid : nh - 1);
    pa.h_at = tid < nh ? hi.at : -1;
    pa.hf = hi.f;
    if (p.mode == AT_SYNC || hi.inner) {
      // the neighbour's (or the PE's own) level-n value
      const Real* src = centre + gidx(hi.gx, hi.gy, z0);
#pragma unroll
      for (int m = 0; m < kMaxT; ++m) pa.h[m] = src;
      pa.hstride = static_cast<int64_t>(p.nx) * p.ny;
      pa.hf = -1;
      return;
    }
    const int nb = nbr[hi.f], pf = hi.f ^ 1;
    pa.hstride = static_cast<int64_t>(p.npe) * (hi.f < 2 ? p.face_chunk[0] : p.face_chunk[2]);
    if constexpr (SP == 3) {
      const Real* src = ring_rd + ring_off(lev_slot[hi.f * kMaxT + hi.m], nb, pf, 0, hi.r);
#pragma unroll
      for (int m = 0; m < kMaxT; ++m) pa.h[m] = src;
    } else {
      const int64_t base = ring_off(0, nb, pf, 0, hi.r);
      const int64_t slot_stride = static_cast<int64_t>(p.npe) * p.pe_block;
      const int s0 = lev_slot[hi.f * kMaxT] > 0 ? lev_slot[hi.f * kMaxT] : 0;
#pragma unroll
      for (int m = 0; m < kMaxT; ++m) {
        const int sl = lev_slot[hi.f * kMaxT + m];
        pa.h[m] = ring_rd + base + (m < p.T && sl >= 0 ? sl : s0) * slot_stride;
      }
    }
  }
  // Loads of in-box plane zz (u and halo) and, with hist, of the history of
  // plane zh. The history fields of the multistep and second Heun stages
  // exist from the first step on (a value loaded before the history is
  // written is not used), so their loads need no branch.
  template <int KIND>
  __device__ __forceinline__ void pipe_load(const PipeAddr& pa, int zz, int zh, bool hist, Prefetch& pf) const {
    const int64_t ps = static_cast<int64_t>(p.nx) * p.ny;
    pf.c = ld4<Real>(pa.c + zz * ps);
    const int64_t ho = zz * pa.hstride;
#pragma unroll
    for (int m = 0; m < kMaxT; ++m) pf.hv[m] = pa.h[m][ho];
    if (hist && (KIND == kVAb2 || KIND == kVAb3 || KIND == kVRk2)) {
      pf.pa = ld4<Real>(pa.a + zh * ps);
      if (KIND == kVAb3) pf.pb = ld4<Real>(pa.b + zh * ps);
    }
  }
  // The values loaded for plane zz into its LDS slot.
  __device__ __forceinline__ void pipe_commit(const PipeAddr& pa, const Prefetch& pf, int zz) {
    Real* P = lds + slot_of<DIM, SD>(zz) * plane;
    if (pa.c_at >= 0) st4<Real>(P + pa.c_at, pf.c);
    if (pa.h_at >= 0) P[pa.h_at] = pa.hf < 0 ? pf.hv[0] : halo_sum(pa.hf, pf.hv);
  }

  __device__ __forceinline__ void compute_plane(int z) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int bx = p.bx, by = p.by, bz = p.bz;
    const Real* C = lds + slot_of<DIM, SD>(z) * plane;
    Real c1[3][2 * S + 1], c2[3][2 * S + 1];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int o = 0; o <= 2 * S; ++o) {
        c1[a][o] = static_cast<Real>(p.c1[a][o]);
        c2[a][o] = static_cast<Real>(p.c2[a][o]);
      }
    // space-expanded schemes: taps at a point next to a low face (o = -SD..SD);
    // the high-face stencils are their mirror images
    Real l1[3][2 * SD + 1], l2[3][2 * SD + 1];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int o = -SD; o <= SD; ++o) {
        l1[a][o + SD] = SP != 0 ? static_cast<Real>(p.sl1[a][o + kMaxS]) : Real(0);
        l2[a][o + SD] = SP != 0 ? static_cast<Real>(p.sl2[a][o + kMaxS]) : Real(0);
      }
    const Real dt = static_cast<Real>(p.dt), alpha = static_cast<Real>(p.alpha);
    const Real vx = static_cast<Real>(p.vel[0]), vy = static_cast<Real>(p.vel[1]),
               vz = static_cast<Real>(p.vel[2]);
    const int gz = z0 + z;
    const int64_t gbase = gidx(x0, y0, gz);   // the plane's first point in the field
    // the previous-level values the update reads (f^{n-1}, f^{n-2} or u^n)
    // are loaded for kBatch points before any of them is computed
    const bool rk2 = p.stage == kStageRk2;
    const bool ab = p.stage != kStageRk1 && p.stage != kStageRk2 && p.integrator != AT_EULER && n > 0;
    const bool ab3 = ab && p.integrator == AT_AB3 && n >= 2;
    const Real* pre_a = static_cast<const Real*>(
        rk2 ? p.ubuf[n & 1] : (ab3 ? p.fbuf[(n - 1) & 1] : p.fbuf[0]));
    const Real* pre_b = static_cast<const Real*>(p.fbuf[n & 1]);
    set_publish_plane(z);
    PlaneIter it(tid, nt, bx);
    while (it.y < by) {
      Real pa[kBatch], pb[kBatch];
      int px[kBatch], py[kBatch];
#pragma unroll
      for (int k = 0; k < kBatch; ++k) {
        px[k] = it.x;
        py[k] = it.y;
        pa[k] = pb[k] = Real(0);
        it.next();
      }
      if (rk2 || ab) {   // uniform: Euler steps and the first RK2 stage read no previous level
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
          const bool in = py[k] < by;
          const int64_t g = gbase + static_cast<int64_t>(in ? py[k] : by - 1) * p.nx + (in ? px[k] : bx - 1);
          pa[k] = pre_a[g];
          if (ab3) pb[k] = pre_b[g];
        }
      }
#pragma unroll
      for (int k = 0; k < kBatch; ++k) {
        const int x = px[k], y = py[k];
        if (y >= by) break;
        const int ly = DIM >= 2 ? y + SD : 0;
        const int c_at = ly * px_stride + x + co;
        const Real u0 = C[c_at];
        // difference form: the taps of each derivative sum to zero, so each
        // neighbour enters as (v - u0), which keeps float rounding small
        Real g1 = 0, g2 = 0;
        if constexpr (SP == 3) {
          // per axis the CD2; at the point next to a face whose delays are
          // not both zero, the four-point stencil with the face's taps
          const Real vel[3] = {vx, vy, vz};
          const bool at_lo[3] = {x == 0, y == 0, z == 0};
          const bool at_hi[3] = {x == bx - 1, y == by - 1, z == bz - 1};
#pragma unroll
          for (int a = 0; a < DIM; ++a) {
            auto nb = [&](int o) -> Real {
              return a == 0 ? C[c_at + o] : a == 1 ? C[c_at + o * px_stride]
                                          : lds[slot_of<DIM, SD>(z + o) * plane + c_at];
            };
            const Real vm = nb(-1) - u0, vp = nb(1) - u0;
            Real d1 = c1[a][0] * vm + c1[a][2] * vp;
            Real d2 = c2[a][0] * vm + c2[a][2] * vp;
            const int f = 2 * a + (at_hi[a] ? 1 : 0);
            if ((at_lo[a] || at_hi[a]) && kpos[f] != 0) {
              const Real* t = nut + f * kNuTaps;
              const Real v2m = nb(-2) - u0, v2p = nb(2) - u0;
              d1 = t[0] * v2m + t[1] * vm + t[3] * vp + t[4] * v2p;
              d2 = t[5] * v2m + t[6] * vm + t[8] * vp + t[9] * v2p;
            }
            g1 += p.equation == AT_ADVDIFF ? vel[a] * d1 : d1;
            g2 += d2;
          }
        } else if constexpr (SP != 0) {
          // per axis: the standard taps, or at the point next to a face whose
          // delay is positive the space-expanded stencil over the own points
          // and the 2 or 3 buffer points of level n - k in the halo frame
          const Real vel[3] = {vx, vy, vz};
          const bool at_lo[3] = {x == 0, y == 0, z == 0};
          const bool at_hi[3] = {x == bx - 1, y == by - 1, z == bz - 1};
#pragma unroll
          for (int a = 0; a < DIM; ++a) {
            const bool lo = at_lo[a] && kpos[2 * a] != 0, hi = at_hi[a] && kpos[2 * a + 1] != 0;
            Real d1 = 0, d2 = 0;
#pragma unroll
            for (int o = -SD; o <= SD; ++o) {
              if (o == 0) continue;
              const Real nv = a == 0 ? C[c_at + o] : a == 1 ? C[c_at + o * px_stride]
                                                     : lds[slot_of<DIM, SD>(z + o) * plane + c_at];
              const Real v = nv - u0;
              const Real s1 = (o >= -S && o <= S) ? c1[a][o + S] : Real(0);
              const Real s2 = (o >= -S && o <= S) ? c2[a][o + S] : Real(0);
              const Real t1 = lo ? l1[a][o + SD] : hi ? -l1[a][SD - o] : s1;
              const Real t2 = lo ? l2[a][o + SD] : hi ? l2[a][SD - o] : s2;
              d1 += t1 * v;
              d2 += t2 * v;
            }
            g1 += p.equation == AT_ADVDIFF ? vel[a] * d1 : d1;
            g2 += d2;
          }
        } else {
          {
            Real d1 = 0, d2 = 0;
#pragma unroll
            for (int o = -S; o <= S; ++o) {
              if (o == 0) continue;
              const Real v = C[c_at + o] - u0;
              d1 += c1[0][o + S] * v;
              d2 += c2[0][o + S] * v;
            }
            g1 = p.equation == AT_ADVDIFF ? vx * d1 : d1;
            g2 = d2;
          }
          if (DIM >= 2) {
            Real d1 = 0, d2 = 0;
#pragma unroll
            for (int o = -S; o <= S; ++o) {
              if (o == 0) continue;
              const Real v = C[c_at + o * px_stride] - u0;
              d1 += c1[1][o + S] * v;
              d2 += c2[1][o + S] * v;
            }
            g1 += p.equation == AT_ADVDIFF ? vy * d1 : d1;
            g2 += d2;
          }
          if (DIM == 3) {
            Real d1 = 0, d2 = 0;
#pragma unroll
            for (int o = -S; o <= S; ++o) {
              if (o == 0) continue;
              const Real v = lds[slot_of<DIM, SD>(z + o) * plane + c_at] - u0;
              d1 += c1[2][o + S] * v;
              d2 += c2[2][o + S] * v;
            }
            g1 += p.equation == AT_ADVDIFF ? vz * d1 : d1;
            g2 += d2;
          }
        }
        const Real f = p.equation == AT_ADVDIFF ? alpha * g2 - g1 : alpha * g2 - u0 * g1;
        const int64_t g = gbase + static_cast<int64_t>(y) * p.nx + x;
        Real un;
        if (p.stage == kStageRk1) {
          un = u0 + dt * f;
          static_cast<Real*>(p.ustar)[g] = un;
        } else if (rk2) {
          un = Real(0.5) * (pa[k] + u0) + (Real(0.5) * dt) * f;
          static_cast<Real*>(p.ubuf[(n + 1) & 1])[g] = un;
        } else {
          if (!ab) {
            un = u0 + dt * f;
            if (p.integrator == AT_AB2 || p.integrator == AT_AB3) static_cast<Real*>(p.fbuf[0])[g] = f;
          } else if (!ab3) {
            // AB2, or AB3 at n = 1 (an AB2 step); f^{n-1} is in fbuf[0] either way
            un = u0 + dt * (Real(1.5) * f - Real(0.5) * pa[k]);
            if (p.integrator == AT_AB2) {
              static_cast<Real*>(p.fbuf[0])[g] = f;
            } else {
              static_cast<Real*>(p.fbuf[1])[g] = f;   // f^1 -> fbuf[1]
            }
          } else {
            // AB3, n >= 2: f^{n-1} in fbuf[(n-1)&1], f^{n-2} in fbuf[n&1]
            un = u0 + dt * ((Real(23) * f - Real(16) * pa[k] + Real(5) * pb[k]) / Real(12));
            static_cast<Real*>(p.fbuf[n & 1])[g] = f;
          }
          static_cast<Real*>(p.ubuf[(n + 1) & 1])[g] = un;
        }
        if (p.mode != AT_SYNC) publish(x, y, z, un);
      }
    }
  }

  // Vector path of one plane (VEC): every thread owns quads of 4 consecutive
  // x points (aligned LDS vectors, 16- or 32-byte global accesses). The stage
  // of the time integrator (KIND) and the equation (EQ) are template
  // parameters, the taps arrive folded (alpha c2 - vel c1 for advection-
  // diffusion), and the space-expanded / non-uniform stencils of Sec. 3.4 and
  // Tables atschemes-left/right are added as a correction (their taps minus
  // the CD2 ones) only on the quads next to a face whose delay calls for them,
  // so the common quad runs no face logic.
  // hist: the thread's history quads (pa, pb) when they were prefetched (one
  // quad per thread), else nullptr.
  template <int KIND, int EQ>
  __device__ __forceinline__ void compute_plane_vec(int z, const Vec4<Real>* hist = nullptr) {
    static_assert(VEC, "vector layout only");
    using Q = Vec4<Real>;
    constexpr int QB = 2;   // quads per thread whose loads are issued together
    const int tid = threadIdx.x, nt = blockDim.x;
    const int bx = p.bx, by = p.by, bz = p.bz;
    const int rows = DIM >= 2 ? rows_sl : 1;   // the workgroup's y-slice
    const int qpr = bx >> 2;
    const Real* C = lds + slot_of<DIM, SD>(z) * plane;
    const Real* Zlo[S];   // z neighbour planes z - o and z + o, o = 1..S
    const Real* Zhi[S];
#pragma unroll
    for (int o = 1; o <= S; ++o) {
      Zlo[o - 1] = DIM == 3 ? lds + slot_of<DIM, SD>(z - o) * plane : C;
      Zhi[o - 1] = DIM == 3 ? lds + slot_of<DIM, SD>(z + o) * plane : C;
    }
    Real kad[3][2 * S + 1], lap[3][2 * S + 1], grd[3][2 * S + 1];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int o = 0; o <= 2 * S; ++o) {
        kad[a][o] = static_cast<Real>(p.kad[a][o]);
        lap[a][o] = static_cast<Real>(p.d2a[a][o]);
        grd[a][o] = static_cast<Real>(p.c1[a][o]);
      }
    const Real dt = static_cast<Real>(p.dt), alpha = static_cast<Real>(p.alpha);
    const Real vel[3] = {static_cast<Real>(p.vel[0]), static_cast<Real>(p.vel[1]), static_cast<Real>(p.vel[2])};
    const int64_t gbase = gidx(x0, y0 + yl0, z0 + z);
    // history and destinations of this stage
    const bool ab = (KIND == kVAb2 || KIND == kVAb3) && n > 0;
    const Real *pre_a, *pre_b;
    bool any_hist, ab3;
    history<KIND>(pre_a, pre_b, any_hist, ab3);
    Real* uout = static_cast<Real*>(KIND == kVRk1 ? p.ustar : p.ubuf[(n + 1) & 1]);
    Real* fout = static_cast<Real*>(KIND == kVAb3 ? (n == 0 ? p.fbuf[0] : n == 1 ? p.fbuf[1] : p.fbuf[n & 1])
                                                  : p.fbuf[0]);
    const bool sync = p.mode == AT_SYNC;
    const bool kp0 = SP != 0 && kpos[0], kp1 = SP != 0 && kpos[1];
    const bool kp2 = SP != 0 && DIM >= 2 && kpos[2], kp3 = SP != 0 && DIM >= 2 && kpos[3];
    const bool kp4 = SP != 0 && DIM == 3 && kpos[4], kp5 = SP != 0 && DIM == 3 && kpos[5];
    set_publish_plane(z);
    // pipelined form (hist given): exactly one quad per thread, the threads
    // beyond the plane's quads repeating the last one (the same values to
    // the same addresses), so that the body runs once with no branch
    // around its stores and the compiler can leave them in flight past the
    // next plane's wait for its loads
    const bool one = hist != nullptr;
    const int quads = qpr * rows;
    PlaneIter it(one && tid >= quads ? quads - 1 : tid, nt, qpr);
    bool more = one || it.y < rows;
    while (more) {
      int qxs[QB], ys[QB];
      Q pa[QB], pb[QB];
#pragma unroll
      for (int j = 0; j < QB; ++j) {
        qxs[j] = it.x;
        ys[j] = it.y;
        it.next();
      }
      more = !one && it.y < rows;
      if (hist != nullptr) {
        // one quad per thread: the only live one is j = 0
        pa[0] = hist[0];
        pb[0] = hist[1];
      } else if (any_hist) {   // uniform
#pragma unroll
        for (int j = 0; j < QB; ++j) {
          const bool in = ys[j] < rows;
          const int64_t g = gbase + static_cast<int64_t>(in ? ys[j] : rows - 1) * p.nx + 4 * (in ? qxs[j] : qpr - 1);
          pa[j] = ld4<Real>(pre_a + g);
          if (KIND == kVAb3 && ab3) pb[j] = ld4<Real>(pre_b + g);
        }
      }
#pragma unroll
      for (int j = 0; j < QB; ++j) {
        const int y = ys[j];
        if (one ? j > 0 : y >= rows) break;
        const int ype = y + yl0;   // row within the PE
        const int qx = qxs[j], x = 4 * qx;
        const int ly = DIM >= 2 ? y + SD : 0;
        const int c_at = ly * px_stride + x + co;
        // x row segment [x - 4, x + 8): the quad and the 4 values on either side
        Real row[12];
        {
          const Q a = ld4<Real>(C + c_at - 4), b = ld4<Real>(C + c_at), c = ld4<Real>(C + c_at + 4);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            row[e] = a.v[e];
            row[4 + e] = b.v[e];
            row[8 + e] = c.v[e];
          }
        }
        Q ym[S], yp[S], zm[S], zp[S];
#pragma unroll
        for (int o = 1; o <= S; ++o) {
          if (DIM >= 2) {
            ym[o - 1] = ld4<Real>(C + c_at - o * px_stride);
            yp[o - 1] = ld4<Real>(C + c_at + o * px_stride);
          }
          if (DIM == 3) {
            zm[o - 1] = ld4<Real>(Zlo[o - 1] + c_at);
            zp[o - 1] = ld4<Real>(Zhi[o - 1] + c_at);
          }
        }
        Q un, fq;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const Real u0 = row[4 + e];
          Real fval;
          if constexpr (EQ == AT_ADVDIFF) {
            Real ax = 0, ay = 0, az = 0;
#pragma unroll
            for (int o = 1; o <= S; ++o) {
              ax += kad[0][S - o] * (row[4 + e - o] - u0);
              if (DIM >= 2) ay += kad[1][S - o] * (ym[o - 1].v[e] - u0);
              if (DIM == 3) az += kad[2][S - o] * (zm[o - 1].v[e] - u0);
              ax += kad[0][S + o] * (row[4 + e + o] - u0);
              if (DIM >= 2) ay += kad[1][S + o] * (yp[o - 1].v[e] - u0);
              if (DIM == 3) az += kad[2][S + o] * (zp[o - 1].v[e] - u0);
            }
            fval = (ax + ay) + az;
          } else {
            Real lx = 0, ly_ = 0, lz = 0, gx = 0, gy = 0, gz = 0;
#pragma unroll
            for (int o = 1; o <= S; ++o) {
              const Real xm = row[4 + e - o] - u0, xp = row[4 + e + o] - u0;
              lx += lap[0][S - o] * xm + lap[0][S + o] * xp;
              gx += grd[0][S - o] * xm + grd[0][S + o] * xp;
              if (DIM >= 2) {
                const Real a_ = ym[o - 1].v[e] - u0, b_ = yp[o - 1].v[e] - u0;
                ly_ += lap[1][S - o] * a_ + lap[1][S + o] * b_;
                gy += grd[1][S - o] * a_ + grd[1][S + o] * b_;
              }
              if (DIM == 3) {
                const Real a_ = zm[o - 1].v[e] - u0, b_ = zp[o - 1].v[e] - u0;
                lz += lap[2][S - o] * a_ + lap[2][S + o] * b_;
                gz += grd[2][S - o] * a_ + grd[2][S + o] * b_;
              }
            }
            fval = ((lx + ly_) + lz) - u0 * ((gx + gy) + gz);
          }
          fq.v[e] = fval;
        }
        if constexpr (SP != 0) {
          // points next to a face whose delay calls for the face stencil:
          // add its difference from the CD2 taps (per-face table in LDS) times
          // the differences (v_o - u0) along the face's axis
          auto corr = [&](int f, Real u0, const Real (&v)[2 * SD + 1]) -> Real {
            const Real* t = dtap + f * kDtaps;
            Real d1 = 0, d2 = 0;
#pragma unroll
            for (int o = -SD; o <= SD; ++o) {
              if (o == 0) continue;
              const Real dv = v[o + SD] - u0;
              d1 += t[o + 3] * dv;
              d2 += t[7 + o + 3] * dv;
            }
            return EQ == AT_ADVDIFF ? alpha * d2 - vel[f >> 1] * d1 : alpha * d2 - u0 * d1;
          };
          // x faces: the first point of a row's first quad, the last of its last
          if (qx == 0 && kp0) {
            Real v[2 * SD + 1];
#pragma unroll
            for (int o = -SD; o <= SD; ++o) v[o + SD] = row[4 + o];
            fq.v[0] += corr(0, row[4], v);
          }
          if (qx == qpr - 1 && kp1) {
            Real v[2 * SD + 1];
#pragma unroll
            for (int o = -SD; o <= SD; ++o) v[o + SD] = row[7 + o];
            fq.v[3] += corr(1, row[7], v);
          }
          // y and z faces: all four points of the quad
          auto face_quad = [&](int f, const Real* base, int stride) {
            Q nq[2 * SD + 1];
#pragma unroll
            for (int o = -SD; o <= SD; ++o) nq[o + SD] = ld4<Real>(base + o * stride);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              Real v[2 * SD + 1];
#pragma unroll
              for (int o = -SD; o <= SD; ++o) v[o + SD] = nq[o + SD].v[e];
              fq.v[e] += corr(f, row[4 + e], v);
            }
          };
          if (DIM >= 2 && ((ype == 0 && kp2) || (ype == by - 1 && kp3)))
            face_quad(ype == 0 && kp2 ? 2 : 3, C + c_at, px_stride);
          if constexpr (DIM == 3) {
            if ((z == 0 && kp4) || (z == bz - 1 && kp5)) {
              // planes z - SD .. z + SD of the LDS ring, at this quad
              const int f = z == 0 && kp4 ? 4 : 5;
              Q nq[2 * SD + 1];
#pragma unroll
              for (int o = -SD; o <= SD; ++o) nq[o + SD] = ld4<Real>(lds + slot_of<DIM, SD>(z + o) * plane + c_at);
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                Real v[2 * SD + 1];
#pragma unroll
                for (int o = -SD; o <= SD; ++o) v[o + SD] = nq[o + SD].v[e];
                fq.v[e] += corr(f, row[4 + e], v);
              }
            }
          }
        }
        const int64_t g = gbase + static_cast<int64_t>(y) * p.nx + x;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const Real u0 = row[4 + e], f = fq.v[e];
          Real r;
          if (KIND == kVEuler || KIND == kVRk1) {
            r = u0 + dt * f;
          } else if (KIND == kVRk2) {
            r = Real(0.5) * (pa[j].v[e] + u0) + (Real(0.5) * dt) * f;
          } else if (!ab) {
            r = u0 + dt * f;
          } else if (!ab3) {
            r = u0 + dt * (Real(1.5) * f - Real(0.5) * pa[j].v[e]);
          } else {
            r = u0 + dt * ((Real(23) * f - Real(16) * pa[j].v[e] + Real(5) * pb[j].v[e]) / Real(12));
          }
          un.v[e] = r;
        }
        if (!sync) {
          // the new edge values of this quad into the strips they lie in
          if (qx == 0)
#pragma unroll
            for (int e = 0; e < SD; ++e) pub[0][ype * SD + e] = un.v[e];
          if (qx == qpr - 1)
#pragma unroll
            for (int e = 4 - SD; e < 4; ++e) pub[1][ype * SD + e - (4 - SD)] = un.v[e];
          if (DIM >= 2) {
            if (ype < SD)
#pragma unroll
              for (int e = 0; e < 4; ++e) pub[2][ype * bx + x + e] = un.v[e];
            if (ype >= by - SD)
#pragma unroll
              for (int e = 0; e < 4; ++e) pub[3][(ype - (by - SD)) * bx + x + e] = un.v[e];
          }
          if (DIM == 3) {
            if (z < SD) {
              Real* zs = slot_base + p.face_off[4] + (static_cast<int64_t>(z) * p.npe + pid) * p.face_chunk[4] + ype * bx + x;
#pragma unroll
              for (int e = 0; e < 4; ++e) zs[e] = un.v[e];
            }
            if (z >= bz - SD) {
              Real* zs = slot_base + p.face_off[5] + (static_cast<int64_t>(z - (bz - SD)) * p.npe + pid) * p.face_chunk[5] +
                         ype * bx + x;
#pragma unroll
              for (int e = 0; e < 4; ++e) zs[e] = un.v[e];
            }
          }
        }
        // the bulk stores last: in the pipelined form they are the newest
        // memory operations of the plane, which the next plane's wait for
        // its loads may leave in flight
        st4<Real>(uout + g, un);
        if (KIND == kVAb2 || KIND == kVAb3) st4<Real>(fout + g, fq);
      }
    }
  }

  // This PE's x and y strips of plane z in the ring slot of the new level:
  // u^{n+1} after a full step, u*^n after the first RK2 stage (z strips are
  // addressed in publish, for the few planes that have them).
  Real* slot_base;
  Real* pub[4];
  __device__ void set_publish_plane(int z) {
    if (p.mode == AT_SYNC) return;
    const bool rk1 = p.stage == kStageRk1;
    Real* R = static_cast<Real*>(rk1 ? p.sring : p.ring);
    const int slot = static_cast<int>((rk1 ? n : n + 1) % p.nslots);
    slot_base = R + static_cast<int64_t>(slot) * p.npe * p.pe_block;
#pragma unroll
    for (int f = 0; f < (DIM >= 2 ? 4 : 2); ++f)
      pub[f] = slot_base + p.face_off[f] + (static_cast<int64_t>(z) * p.npe + pid) * p.face_chunk[f];
  }

  // Write a new edge value into the strips (of the plane set last) it lies in.
  __device__ void publish(int x, int y, int z, Real v) const {
    const int bx = p.bx, by = p.by, bz = p.bz;
    if (x < SD) pub[0][y * SD + x] = v;
    if (x >= bx - SD) pub[1][y * SD + x - (bx - SD)] = v;
    if (DIM >= 2) {
      if (y < SD) pub[2][y * bx + x] = v;
      if (y >= by - SD) pub[3][(y - (by - SD)) * bx + x] = v;
    }
    if (DIM == 3) {
      // z strips: depth plane z (low face) or z - (bz - s) (high face)
      if (z < SD)
        slot_base[p.face_off[4] + (static_cast<int64_t>(z) * p.npe + pid) * p.face_chunk[4] + y * bx + x] = v;
      if (z >= bz - SD)
        slot_base[p.face_off[5] + (static_cast<int64_t>(z - (bz - SD)) * p.npe + pid) * p.face_chunk[5] +
                  y * bx + x] = v;
    }
  }
};

// Neighbour PE across face f = 2*axis + side (periodic).
__device__ inline int neighbour(const StepParams& p, int pid, int f) {
  int q[3] = {pid % p.px, (pid / p.px) % p.py, pid / (p.px * p.py)};
  const int ext[3] = {p.px, p.py, p.pz};
  const int a = f >> 1;
  q[a] = (q[a] + ((f & 1) ? 1 : ext[a] - 1)) % ext[a];
  return q[0] + p.px * (q[1] + p.py * q[2]);
}

// Delay of face f at step n (after the clamp), from the generator, zero or the
// host table.
__device__ inline int face_delay(const StepParams& p, int pid, int f, int64_t n) {
  int k = 0;
  if (p.mode == AT_DELAY_RNG) {
    k = raw_delay(p.key, n, static_cast<uint32_t>(pid * 2 * p.ndim + f), p.thr, p.L);
  } else if (p.mode == AT_DELAY_HOST) {
    k = p.host_delays[(n * p.npe + pid) * (2 * p.ndim) + f];
  }
  return clamp_startup(k, n, p.T);
}

// Delay of the second buffer point of face f (non-uniform-delay scheme): a
// draw of the generator with the face index shifted by the number of faces,
// clamped like every delay; 0 unless the delays are drawn.
__device__ inline int point_delay(const StepParams& p, int pid, int f, int64_t n) {
  if (p.mode != AT_DELAY_RNG) return 0;
  const uint32_t nfaces = static_cast<uint32_t>(p.npe * 2 * p.ndim);
  return clamp_startup(raw_delay(p.key, n, nfaces + static_cast<uint32_t>(pid * 2 * p.ndim + f), p.thr, p.L), n,
                       p.T);
}

// Non-uniform-delay scheme, face f of PE pid at step n (Sec. 3.4 Example 1):
// delays k1 (nearest buffer point: the face's draw) and k2 (second point: a
// draw with the face index shifted by the number of faces), both clamped as
// any delay. On the singular set 3 k1 = k2 (k1 >= 1) the nearest point takes
// the next older level k1 + 1, which the ring still holds. Writes the use
// flag, the two ring slots and the taps by offset o = -2..2 of both
// derivatives, scaled by 1/dx and 1/dx^2: at a high face, for points (i-1,
// i+1, i+2) the first derivative ((k2 - 4k1), -k2, k1) / (2 (3k1 - k2)) and
// the second ((2k1 - k2), -k2, k1) / (3k1 - k2) (the centre tap is implied:
// each row sums to zero); a low face takes the mirror image.
__device__ inline void nonuniform_face(const StepParams& p, int pid, int f, int64_t n, int* kpos, int* slot,
                                       double* nu) {
  int k1 = face_delay(p, pid, f, n);
  const int k2 = point_delay(p, pid, f, n);
  const bool use = k1 != 0 || k2 != 0;
  if (use && 3 * k1 == k2) ++k1;
  kpos[f] = use;
  const int r0 = static_cast<int>(n % p.nslots);
  slot[f * kMaxT + 0] = slot_back(r0, k1, p.nslots);
  slot[f * kMaxT + 1] = slot_back(r0, k2, p.nslots);
  const int a = f >> 1;
  const double den = use ? static_cast<double>(3 * k1 - k2) : 1.0;
  // taps at j = -1, +1, +2 of a high face
  const double t1[3] = {(k2 - 4 * k1) / (2.0 * den), -k2 / (2.0 * den), k1 / (2.0 * den)};
  const double t2[3] = {(2 * k1 - k2) / den, -k2 / den, k1 / den};
  const int jj[3] = {-1, 1, 2};
  const bool hi = f & 1;
  for (int i = 0; i < kNuTaps; ++i) nu[f * kNuTaps + i] = 0.0;
  for (int i = 0; i < 3; ++i) {
    const int o = hi ? jj[i] : -jj[i];
    nu[f * kNuTaps + o + 2] = (hi ? t1[i] : -t1[i]) * p.sl1[a][kMaxS];
    nu[f * kNuTaps + 5 + o + 2] = t2[i] * p.sl2[a][kMaxS];
  }
}

// The face stencil of face f (the space-expanded single-level taps of
// Sec. 3.4 and Tables atschemes-left/right, mirrored for a high face, or the
// non-uniform taps nu of Example 1) minus the CD2 taps it replaces, by
// offset o = -3..3 along the face's axis, into dt[kDtaps]: the vector path
// adds their product with the differences (v_o - u0) at the points next to a
// face whose delay calls for the face stencil.
template <typename Real, int SP>
__device__ inline void face_delta_taps(const StepParams& p, int f, const double* nu, Real* dt) {
  const int a = f >> 1;
  const bool lo = (f & 1) == 0;
  auto cd1 = [&](int o) { return o >= -1 && o <= 1 ? p.c1[a][o + 1] : 0.0; };
  auto cd2 = [&](int o) { return o >= -1 && o <= 1 ? p.c2[a][o + 1] : 0.0; };
  for (int o = -3; o <= 3; ++o) {
    double t1 = 0.0, t2 = 0.0;
    if constexpr (SP == 3) {
      if (o >= -2 && o <= 2) {
        t1 = nu[f * kNuTaps + o + 2] - cd1(o);
        t2 = nu[f * kNuTaps + 5 + o + 2] - cd2(o);
      }
    } else {
      t1 = lo ? p.sl1[a][o + kMaxS] - cd1(o) : -(p.sl1[a][-o + kMaxS] - cd1(-o));
      t2 = lo ? p.sl2[a][o + kMaxS] - cd2(o) : p.sl2[a][-o + kMaxS] - cd2(-o);
    }
    dt[o + 3] = static_cast<Real>(t1);
    dt[7 + o + 3] = static_cast<Real>(t2);
  }
}

// Whether a 3-D vector-path instance has the pipelined form (the space-
// expanded and non-uniform stencils, whose face corrections take more
// registers, and sixth order in FP64 do not).
template <typename Real, int S, int SP>
constexpr bool pipe_form() {
  return SP == 0 && (sizeof(Real) == 4 || S < 3);
}

// VEC: the vector layout and path, specialised on the integrator stage KIND
// and the equation EQ (the scalar path reads both at run time).
// PIPE (3-D vector path only): the pipelined sweep, at most kMaxVec3Threads
// threads, so that it may hold 168 VGPRs per lane.
template <typename Real, int DIM, int S, int SP, bool VEC = false, int KIND = 0, int EQ = 0, bool PIPE = false>
__global__ __launch_bounds__(PIPE ? kMaxVec3Threads : kMaxSweepThreads) void at_step_kernel(StepParams p) {
  constexpr int SD = strip_depth<S, SP>();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Real* lds = reinterpret_cast<Real*>(smem_raw);
  __shared__ double s_w[6 * kMaxT];
  __shared__ int s_slot[6 * kMaxT];
  __shared__ int s_nbr[6];
  __shared__ int s_kpos[6];
  __shared__ double s_nu[SP == 3 ? 6 * kNuTaps : 1];
  __shared__ Real s_nur[SP == 3 ? 6 * kNuTaps : 1];
  __shared__ Real s_dt[SP != 0 ? 6 * kDtaps : 1];

  const int64_t n = p.counter[0];
  const int pid = sweep_part<DIM>(p).pid;
  const int tid = threadIdx.x;
  // neighbours, delays and level weights of the 2 * DIM faces
  auto faces = [&]() {
    if (tid >= 2 * DIM) return;
    const int f = tid;
    s_nbr[f] = neighbour(p, pid, f);
    s_kpos[f] = 0;
    if constexpr (SP == 3) {
      if (p.mode != AT_SYNC) {
        nonuniform_face(p, pid, f, n, s_kpos, s_slot, s_nu);
        // the stencil multiplies in the storage type: convert once per face
        for (int i = 0; i < kNuTaps; ++i) s_nur[f * kNuTaps + i] = static_cast<Real>(s_nu[f * kNuTaps + i]);
        if (VEC && s_kpos[f]) face_delta_taps<Real, SP>(p, f, s_nu, s_dt + f * kDtaps);
      }
      return;
    }
    if (p.mode != AT_SYNC) {
      const int k = face_delay(p, pid, f, n);
      s_kpos[f] = k > 0;
      if constexpr (SP != 0)
        if (VEC && k > 0) face_delta_taps<Real, SP>(p, f, nullptr, s_dt + f * kDtaps);
      const int r0 = static_cast<int>(n % p.nslots);
      double w[kMaxT];
      level_weights(k, p.T, w);
      for (int m = 0; m < kMaxT; ++m) {
        const bool live = m < p.T && w[m] != 0.0;
        s_w[f * kMaxT + m] = live ? w[m] : 0.0;
        s_slot[f * kMaxT + m] = live ? slot_back(r0, k + m, p.nslots) : -1;
      }
    }
  };

  Sweep<Real, DIM, S, SP, VEC> sw(p, lds, n, s_w, s_slot, s_nbr, s_kpos, s_nur, s_dt);
  auto compute = [&](int z) {
    if constexpr (VEC)
      sw.template compute_plane_vec<KIND, EQ>(z);
    else
      sw.compute_plane(z);
  };
  if (DIM == 3) {
    // the workgroup sweeps z-chunk ci, [zc0, zc1), of y-slice ys of its PE
    // (y-slices: pipelined form only); the SD planes on either side come
    // from the PE (or across its z faces)
    const SweepPart part = sweep_part<DIM>(p);
    const int nys = PIPE && p.yslices > 1 ? p.yslices : 1;
    const int nch = part.nch;
    const int ci = part.ci;
    if (nys > 1) sw.set_slice(part.ys, nys);
    const int zper = (p.bz + nch - 1) / nch;
    const int zc0 = ci * zper;
    const int zc1 = zc0 + zper < p.bz ? zc0 + zper : p.bz;
    faces();
    __syncthreads();
    if constexpr (PIPE) {
      static_assert(VEC && DIM == 3 && pipe_form<Real, S, SP>(), "pipelined form");
      // plane z + 1 + SD (u, halo) and the history of plane z + 1 are loaded
      // while plane z is computed, issued after the barrier (two planes ahead
      // measured no faster and takes more registers; issuing them before the
      // barrier, slower). The host launches this form only where every
      // thread owns at most one quad and one halo item of a slice's plane.
      using SW = Sweep<Real, DIM, S, SP, VEC>;
      if (zc0 < zc1) {
        typename SW::PipeAddr pa;
        sw.template pipe_setup<KIND>(pa);
        const int bz = p.bz;
        auto cl = [&](int zz) { return zz < 0 ? 0 : zz < bz ? zz : bz - 1; };
        // the 2 SD planes before the first one computed: their loads, then
        // those of the first iteration, are issued together
        typename SW::Prefetch pro[2 * SD], pf;
#pragma unroll
        for (int i = 0; i < 2 * SD; ++i) sw.template pipe_load<KIND>(pa, cl(zc0 - SD + i), 0, false, pro[i]);
#pragma unroll
        for (int e = 0; e < 4; ++e) pf.pa.v[e] = pf.pb.v[e] = Real(0);
        sw.template pipe_load<KIND>(pa, cl(zc0 + SD), zc0, true, pf);
#pragma unroll
        for (int i = 0; i < 2 * SD; ++i) {
          const int zz = zc0 - SD + i;
          if (zz < 0 || zz >= bz)
            sw.load_plane(zz);
          else
            sw.pipe_commit(pa, pro[i], zz);
        }
        // planes z whose plane z + SD lies in the PE: every load is
        // unconditional (no register copies that would wait for them)
        const int zm = zc1 < bz - SD ? zc1 : bz - SD;
        int z = zc0;
        for (; z < zm; ++z) {
          sw.pipe_commit(pa, pf, z + SD);
          const Vec4<Real> hq[2] = {pf.pa, pf.pb};
          __syncthreads();
          sw.template pipe_load<KIND>(pa, cl(z + 1 + SD), cl(z + 1), true, pf);
          sw.template compute_plane_vec<KIND, EQ>(z, hq);
        }
        // the last SD planes of the PE (last chunk): plane z + SD comes
        // from the z strips beyond the high face
        for (; z < zc1; ++z) {
          sw.load_plane(z + SD);
          __syncthreads();
          sw.template compute_plane_vec<KIND, EQ>(z);
        }
      }
    } else if (zc0 < zc1) {
      for (int zz = zc0 - SD; zz < zc0 + SD; ++zz) sw.load_plane(zz);
      for (int z = zc0; z < zc1; ++z) {
        sw.load_plane(z + SD);
        __syncthreads();
        compute(z);
      }
    }
  } else {
    // the PE's own values do not depend on the delays: their loads are in
    // flight while the first wave derives the face weights
    sw.load_plane(0, kPlaneCentre);
    faces();
    __syncthreads();
    sw.load_plane(0, kPlaneHalos);
    __syncthreads();
    compute(0);
  }

  if (p.advance) {
    // every workgroup has read n before its own increment
    __syncthreads();
    if (tid == 0) advance_counter(p.counter, n);
  }
}

// Vector-path launches for one precision and dimension (instantiated in
// step_vec_*.hip): dispatch on the scheme (half-width, space-expanded or
// non-uniform family), the integrator stage and the equation.
template <typename Real, int DIM, int S, int SP, int KIND, bool PIPE>
hipError_t launch_vec_e(const StepParams& p, hipStream_t st, int blocks, int threads, size_t lds) {
  if (p.equation == AT_ADVDIFF)
    hipLaunchKernelGGL((at_step_kernel<Real, DIM, S, SP, true, KIND, AT_ADVDIFF, PIPE>), dim3(blocks), dim3(threads),
                       lds, st, p);
  else
    hipLaunchKernelGGL((at_step_kernel<Real, DIM, S, SP, true, KIND, AT_BURGERS, PIPE>), dim3(blocks), dim3(threads),
                       lds, st, p);
  return hipGetLastError();
}

template <typename Real, int DIM, int S, int SP, int KIND>
hipError_t launch_vec_k(const StepParams& p, hipStream_t st, int blocks, int threads, size_t lds) {
  const int nys = p.yslices > 1 ? p.yslices : 1;
  if constexpr (DIM == 3 && pipe_form<Real, S, SP>()) {
    if (vec_pipe(p, strip_depth<S, SP>(), p.by / nys)) {
      // one quad and one halo item of a slice's plane per thread (see
      // vec_threads); slices of equal rows, at least SD each
      const int rows = p.by / nys;
      const int quads = (p.bx / 4) * rows, halos = 2 * strip_depth<S, SP>() * (p.bx + rows);
      if (threads < quads || threads < halos || threads > kMaxVec3Threads || rows * nys != p.by ||
          rows < strip_depth<S, SP>() || blocks % (p.npe * nys) != 0)
        return hipErrorInvalidConfiguration;
      return launch_vec_e<Real, DIM, S, SP, KIND, true>(p, st, blocks, threads, lds);
    }
  }
  if (nys != 1) return hipErrorInvalidConfiguration;   // y-slices: pipelined form only
  return launch_vec_e<Real, DIM, S, SP, KIND, false>(p, st, blocks, threads, lds);
}

template <typename Real, int DIM, int S, int SP>
hipError_t launch_vec_s(const StepParams& p, hipStream_t st, int blocks, int threads, size_t lds) {
  if (p.stage == kStageRk1) return launch_vec_k<Real, DIM, S, SP, kVRk1>(p, st, blocks, threads, lds);
  if (p.stage == kStageRk2) return launch_vec_k<Real, DIM, S, SP, kVRk2>(p, st, blocks, threads, lds);
  switch (p.integrator) {
    case AT_EULER: return launch_vec_k<Real, DIM, S, SP, kVEuler>(p, st, blocks, threads, lds);
    case AT_AB2: return launch_vec_k<Real, DIM, S, SP, kVAb2>(p, st, blocks, threads, lds);
    case AT_AB3: return launch_vec_k<Real, DIM, S, SP, kVAb3>(p, st, blocks, threads, lds);
  }
  return hipErrorInvalidValue;
}

template <typename Real, int DIM>
hipError_t launch_vec(const StepParams& p, hipStream_t st, int blocks, int threads, size_t lds) {
  if (p.scheme == AT_SCHEME_NONUNIFORM_212) return launch_vec_s<Real, DIM, 1, 3>(p, st, blocks, threads, lds);
  if (p.scheme == AT_SCHEME_SPACE_212) return launch_vec_s<Real, DIM, 1, 1>(p, st, blocks, threads, lds);
  if (p.scheme == AT_SCHEME_SPACE_222) return launch_vec_s<Real, DIM, 1, 2>(p, st, blocks, threads, lds);
  switch (p.s) {
    case 1: return launch_vec_s<Real, DIM, 1, 0>(p, st, blocks, threads, lds);
    case 2: return launch_vec_s<Real, DIM, 2, 0>(p, st, blocks, threads, lds);
    case 3: return launch_vec_s<Real, DIM, 3, 0>(p, st, blocks, threads, lds);
  }
  return hipErrorInvalidValue;
}

}  // namespace sweep

hipError_t launch_step_vec_f32_d1(const StepParams& p, hipStream_t st, int blocks, int threads, size_t lds);
hipError_t launch_step_vec_f32_d2(const StepParams& p, hipStream_t st, int blocks, int threads, size_t lds);
hipError_t launch_step_vec_f32_d3(const StepParams& p, hipStream_t st, int blocks, int threads, size_t lds);
hipError_t launch_step_vec_f64_d1(const StepParams& p, hipStream_t st, int blocks, int threads, size_t lds);
hipError_t launch_step_vec_f64_d2(const StepParams& p, hipStream_t st, int blocks, int threads, size_t lds);
hipError_t launch_step_vec_f64_d3(const StepParams& p, hipStream_t st, int blocks, int threads, size_t lds);
}  // namespace atfd
