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

#include "atfd_internal.hpp"
#include "delays.hpp"

namespace atfd {
namespace {

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

// Per-face taps of the non-uniform scheme, [face][derivative][o + 2]
constexpr int kNuTaps = 10;

template <typename Real, int DIM, int S, int SP>
struct Sweep {
  static constexpr int SD = strip_depth<S, SP>();
  static constexpr int NSL = DIM == 3 ? 2 * SD + 2 : 1;
  static constexpr int kBatch = 4;   // points per thread whose loads are issued together

  const StepParams& p;
  Real* lds;
  int pid, qx, qy, qz, x0, y0, z0;
  int px_stride, plane;     // LDS row stride and plane size
  int64_t n;
  const Real* centre;       // field whose level-n values feed the stencil
  const Real* ring_rd;      // ring the halos come from
  // per-face delay data (AT) in LDS
  const double* w;          // [6][kMaxT]
  const int* lev_slot;      // [6][kMaxT] ring slot of level n-k-m, -1 if weight 0
  const int* nbr;           // [6] neighbour PE of face
  const int* kpos;          // [6] face delay k > 0 (space-expanded stencils apply)
  const Real* nut;          // [6][kNuTaps] non-uniform taps (SP = 3), in the storage type

  __device__ Sweep(const StepParams& p_, Real* lds_, int64_t n_, const double* w_,
                   const int* ls_, const int* nb_, const int* kp_, const Real* nu_)
      : p(p_), lds(lds_), n(n_), w(w_), lev_slot(ls_), nbr(nb_), kpos(kp_), nut(nu_) {
    pid = blockIdx.x % p.npe;   // workgroups beyond npe take further z-chunks of the PEs
    qx = pid % p.px;
    qy = (pid / p.px) % p.py;
    qz = pid / (p.px * p.py);
    x0 = qx * p.bx;
    y0 = qy * p.by;
    z0 = qz * p.bz;
    px_stride = p.bx + 2 * SD;
    plane = (DIM >= 2 ? p.by + 2 * SD : 1) * px_stride;
    const bool rk2 = p.stage == kStageRk2;
    centre = static_cast<const Real*>(rk2 ? p.ustar : p.ubuf[n & 1]);
    ring_rd = static_cast<const Real*>(rk2 ? p.sring : p.ring);
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
  // single level of buffer point m.
  __device__ Real halo(int f, int plane, int r, int m, int gx, int gy, int gz) const {
    if (p.mode == AT_SYNC) return centre[gidx(gx, gy, gz)];
    const int pf = f ^ 1;   // producer face: the opposite side
    const int nb = nbr[f];
    if constexpr (SP == 3) return ring_rd[ring_off(lev_slot[f * kMaxT + m], nb, pf, plane, r)];
    // every level is loaded from an in-range slot so that the T loads are in
    // flight together; a level of weight zero (k = 0: exact synchronous
    // value) is then dropped by the select
    const int64_t base = ring_off(0, nb, pf, plane, r);
    const int64_t slot_stride = static_cast<int64_t>(p.npe) * p.pe_block;
    Real v[kMaxT];
#pragma unroll
    for (int m = 0; m < kMaxT; ++m) {
      const int sl = lev_slot[f * kMaxT + m];
      v[m] = ring_rd[base + (m < p.T && sl > 0 ? sl : 0) * slot_stride];
    }
    double acc = 0.0;
#pragma unroll
    for (int m = 0; m < kMaxT; ++m) {
      const int sl = lev_slot[f * kMaxT + m];
      if (m < p.T && sl >= 0) acc += w[f * kMaxT + m] * static_cast<double>(v[m]);
    }
    return static_cast<Real>(acc);
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

  __device__ void load_plane(int zz, int parts = kPlaneCentre | kPlaneHalos) {
    Real* P = lds + slot_of<DIM, SD>(zz) * plane;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int bx = p.bx, by = p.by, bz = p.bz;
    if (zz >= 0 && zz < bz) {
      const int gz = z0 + zz;
      // kBatch loads per thread are issued before any LDS write, from
      // clamped (in-range) addresses
      if (parts & kPlaneCentre) {
        const Real* cz = centre + gidx(x0, y0, gz);
        PlaneIter it(tid, nt, bx);
        while (it.y < by) {
          Real v[kBatch];
          int at[kBatch];
#pragma unroll
          for (int k = 0; k < kBatch; ++k) {
            const bool in = it.y < by;
            v[k] = cz[static_cast<int64_t>(in ? it.y : by - 1) * p.nx + (in ? it.x : bx - 1)];
            at[k] = in ? (DIM >= 2 ? it.y + SD : 0) * px_stride + it.x + SD : -1;
            it.next();
          }
#pragma unroll
          for (int k = 0; k < kBatch; ++k)
            if (at[k] >= 0) P[at[k]] = v[k];
        }
      }
      // x halos (producer strip [z][y][d]) and y halos (producer strip
      // [z][d][x]) in one pass, so that their loads overlap
      const int nxh = 2 * SD * by, nh = (parts & kPlaneHalos) ? nxh + (DIM >= 2 ? 2 * SD * bx : 0) : 0;
      for (int h = tid; h < nh; h += nt) {
        if (h < nxh) {
          const int side = h >= SD * by ? 1 : 0, r = side ? h - SD * by : h, d = r % SD, y = r / SD;
          const int xl = side ? bx + d : d - SD;
          const int gx = wrap(x0 + xl, p.nx);
          P[(DIM >= 2 ? y + SD : 0) * px_stride + xl + SD] =
              halo(side, zz, y * SD + d, side ? d : SD - 1 - d, gx, y0 + y, gz);
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
          const int gy = wrap(y0 + yl, p.ny);
          P[(yl + SD) * px_stride + x + SD] = halo(2 + side, zz, d * bx + x, side ? d : SD - 1 - d, x0 + x, gy, gz);
        }
      }
    } else {
      // z halo plane: producer strip [d][y][x]
      const int side = zz < 0 ? 0 : 1;
      const int d = side ? zz - bz : zz + SD;
      const int gz = wrap(z0 + zz, p.nz);
      for (PlaneIter it(tid, nt, bx); it.y < by; it.next()) {
        const int x = it.x, y = it.y;
        P[(y + SD) * px_stride + x + SD] = halo(4 + side, d, y * bx + x, side ? d : SD - 1 - d, x0 + x, y0 + y, gz);
      }
    }
  }

  __device__ void compute_plane(int z) {
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
        const int c_at = ly * px_stride + x + SD;
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

template <typename Real, int DIM, int S, int SP>
__global__ __launch_bounds__(kMaxSweepThreads) void at_step_kernel(StepParams p) {
  constexpr int SD = strip_depth<S, SP>();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Real* lds = reinterpret_cast<Real*>(smem_raw);
  __shared__ double s_w[6 * kMaxT];
  __shared__ int s_slot[6 * kMaxT];
  __shared__ int s_nbr[6];
  __shared__ int s_kpos[6];
  __shared__ double s_nu[SP == 3 ? 6 * kNuTaps : 1];
  __shared__ Real s_nur[SP == 3 ? 6 * kNuTaps : 1];

  const int64_t n = p.counter[0];
  const int pid = blockIdx.x % p.npe;
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
      }
      return;
    }
    if (p.mode != AT_SYNC) {
      const int k = face_delay(p, pid, f, n);
      s_kpos[f] = k > 0;
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

  Sweep<Real, DIM, S, SP> sw(p, lds, n, s_w, s_slot, s_nbr, s_kpos, s_nur);
  if (DIM == 3) {
    // workgroup blockIdx.x / npe sweeps z-chunk [zc0, zc1) of its PE; the
    // SD planes on either side come from the PE (or across its z faces)
    const int nch = gridDim.x / p.npe;
    const int zper = (p.bz + nch - 1) / nch;
    const int zc0 = static_cast<int>(blockIdx.x / p.npe) * zper;
    const int zc1 = zc0 + zper < p.bz ? zc0 + zper : p.bz;
    faces();
    __syncthreads();
    if (zc0 < zc1) {
      for (int zz = zc0 - SD; zz < zc0 + SD; ++zz) sw.load_plane(zz);
      for (int z = zc0; z < zc1; ++z) {
        sw.load_plane(z + SD);
        __syncthreads();
        sw.compute_plane(z);
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
    sw.compute_plane(0);
  }

  if (p.advance) {
    // every workgroup has read n before its own increment
    __syncthreads();
    if (tid == 0) advance_counter(p.counter, n);
  }
}

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
    const Real v = u[(static_cast<int64_t>(z0 + z) * p.ny + y0 + y) * p.nx + x0 + x];
    for (int j = 0; j < nf; ++j)
      for (int sl = 0; sl < p.nslots; ++sl) {
        const int64_t off = ring_index_q(p, sl, pid, face[j], q[j]);
        R[off] = v;
        if (SR) SR[off] = v;
      }
  }
}

__global__ void set_counter_kernel(int64_t* counter, int64_t n) {
  if (threadIdx.x == 0) {
    counter[0] = n;
    counter[1] = 0;
  }
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

template <typename Real, int DIM, int S, int SP>
size_t lds_bytes_t(const StepParams& p) {
  constexpr int SD = strip_depth<S, SP>();
  const int nsl = DIM == 3 ? 2 * SD + 2 : 1;
  const size_t plane = static_cast<size_t>(DIM >= 2 ? p.by + 2 * SD : 1) * (p.bx + 2 * SD);
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

// Workgroups per PE of the generic sweep. A 3-D PE's planes are split into
// z-chunks (each reloads the SD planes around it) within one round of
// resident workgroups (256 CUs, each holding as many as its LDS and thread
// slots allow, at most four). Only where no chunk overwrites planes another
// one reads: the new level goes to the other solution buffer, or the stage
// writes the RK2 predictor / reads it (Heun). 1-D and 2-D PEs are a single
// plane.
constexpr int kNumCUs = 256;   // compute units of an MI355X

int sweep_chunks(const StepParams& p, size_t lds, int threads, int sd) {
  if (p.ndim != 3) return 1;
  if (p.ubuf[0] == p.ubuf[1] && p.integrator != AT_RK2) return 1;
  int per_cu = static_cast<int>((160 * 1024) / (lds > 0 ? lds : 1));
  const int by_threads = 2048 / threads;
  if (per_cu > by_threads) per_cu = by_threads;
  if (per_cu > 4) per_cu = 4;
  if (per_cu < 1) per_cu = 1;
  const int64_t slots = static_cast<int64_t>(kNumCUs) * per_cu;
  if (p.npe >= kNumCUs) {
    // every CU already has a PE: chunks only add co-resident workgroups,
    // as many as fill one resident round, of at least 8 planes each
    const int want = static_cast<int>(slots / p.npe);
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
  for (int nch = 1; nch <= p.bz; ++nch) {
    const int64_t wgs = static_cast<int64_t>(p.npe) * nch;
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

template <typename Real, int DIM, int S, int SP>
hipError_t launch_t(const StepParams& p, hipStream_t st) {
  const size_t lds = lds_bytes_t<Real, DIM, S, SP>(p);
  const int threads = sweep_threads(p);
  hipLaunchKernelGGL((at_step_kernel<Real, DIM, S, SP>), dim3(p.npe * sweep_chunks(p, lds, threads, strip_depth<S, SP>())), dim3(threads),
                     lds, st, p);
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

template <typename Real, int DIM>
size_t lds_s(const StepParams& p, int s) {
  if (p.scheme == AT_SCHEME_SPACE_212) return lds_bytes_t<Real, DIM, 1, 1>(p);
  if (p.scheme == AT_SCHEME_SPACE_222) return lds_bytes_t<Real, DIM, 1, 2>(p);
  if (p.scheme == AT_SCHEME_NONUNIFORM_212) return lds_bytes_t<Real, DIM, 1, 3>(p);
  switch (s) {
    case 1: return lds_bytes_t<Real, DIM, 1, 0>(p);
    case 2: return lds_bytes_t<Real, DIM, 2, 0>(p);
    case 3: return lds_bytes_t<Real, DIM, 3, 0>(p);
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
  const int64_t field_bytes = static_cast<int64_t>(p.nx) * p.ny * p.nz * (f64 ? 8 : 4);
  if (fast3d_applies(p, f64) && field_bytes < (int64_t(1) << 32)) return launch_step_fast3d(p, f64, s, st);
  return f64 ? dispatch_dim<double>(p, s, st, false) : dispatch_dim<float>(p, s, st, false);
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
