// Discrete adjoint of the AT time step (advection-diffusion or viscous
// Burgers; Euler, AB2 or Heun RK2).
//
// One stage of the forward step computes, at every point i from a stage field
// c (u for Euler/AB2 and the first RK2 stage, the predictor u* for the second),
//   F_i = alpha sum_{a,o} c2_o (v_{a,o} - c_i) - [c . grad] ,
// where v_{a,o} = c_{i+o} for a tap inside the PE of i (Sec. 2 eq.
// general_deriv) and, for a tap across face f, the AT combination
// sum_m c_m(k) c^{n-k-m}_{i+o} of that field's history with the face's delay k
// (Sec. 3.4 Example 3 eq. cd4-at); the advection term is sum c_a c1_o (v - c_i)
// (advection-diffusion) or c_i sum c1_o (v - c_i) (Burgers; Sec. 5 eq.
// general). Linearised, dF_i = sum K_{i,a,o} dv_{a,o} + D_i dc_i with
//   K_{i,a,o} = alpha c2_o - c_a c1_o  or  alpha c2_o - c_i c1_o,
//   D_i = -sum K_{i,a,o}  (- G_i = -sum c1_o (v - c_i) for Burgers).
// Given mu = dJ/dF (one field), the stage adjoint is
//   out_j = (base terms) + D_j mu_j + sum_{o: j-o in the PE of j} K_{j-o,a,o} mu_{j-o} + A^n_j,
// where A^l gathers, at the edge strips that neighbours read, K_{i,a,o} c_m(k)
// mu_i of every later step with n - k - m = l: an adjoint ring of the forward
// ring's shape, filled in gather form (one thread per strip value: the strip
// kernel in 3-D, the stage kernel's own strip phase in 1-D / 2-D) and drained
// when the sweep reaches level l. The alpha-gradient adds
// <mu, dF/dalpha> = <mu, AT Laplacian of c>.
//
// Euler/AB2 (Sec. 4.1 eqs. time_disc, time_ab2): one stage per step, mu =
// dt (beta0 lambda^{n+1} + beta1 lambda^{n+2}), out = lambda^n with base
// lambda^{n+1}. Heun: stage 2 with mu = dt/2 lambda^{n+1} gives sigma = dJ/du*
// (base lambda^{n+1}/2, predictor ring), then stage 1 with mu = dt sigma gives
// lambda^n (base lambda^{n+1}/2 + sigma, solution ring).

#include "adjoint.hpp"

#include <algorithm>
#include <type_traits>

namespace atfd {
namespace {

constexpr int kAdjThreads = 256;

struct Pt {
  int x, y, z;      // global coordinates
  int pe;           // PE id
  int l[3];         // coordinates inside the PE
};

// (fields below 2^31 points: the host checks)
__device__ inline Pt point_of(const StepParams& p, int64_t g64) {
  Pt r;
  const uint32_t g = static_cast<uint32_t>(g64);
  const uint32_t row = g / static_cast<uint32_t>(p.nx);
  r.x = static_cast<int>(g - row * static_cast<uint32_t>(p.nx));
  r.z = static_cast<int>(row / static_cast<uint32_t>(p.ny));
  r.y = static_cast<int>(row - static_cast<uint32_t>(r.z) * static_cast<uint32_t>(p.ny));
  const int qx = r.x / p.bx, qy = r.y / p.by, qz = r.z / p.bz;
  r.l[0] = r.x - qx * p.bx;
  r.l[1] = r.y - qy * p.by;
  r.l[2] = r.z - qz * p.bz;
  r.pe = qx + p.px * (qy + p.py * qz);
  return r;
}

__device__ inline int64_t gindex(const StepParams& p, int x, int y, int z) {
  return (static_cast<int64_t>(z) * p.ny + y) * p.nx + x;
}

__device__ inline int edge_of(const StepParams& p, int a) { return a == 0 ? p.bx : a == 1 ? p.by : p.bz; }

// Component a of a 3-vector, and a write of it, by selects: a run-time index
// into a local array would put the array in scratch memory.
__device__ inline int sel3(int a, int v0, int v1, int v2) { return a == 0 ? v0 : a == 1 ? v1 : v2; }
__device__ inline void set3(int* l, int a, int v) {
  l[0] = a == 0 ? v : l[0];
  l[1] = a == 1 ? v : l[1];
  l[2] = a == 2 ? v : l[2];
}

// Element of the strip of face F = 2a + side of a PE for the point with PE
// coordinates l (which must lie in that strip): x faces [z][y][d], y faces
// [z][d][x], z faces [d][y][x], with depth d counted from the PE's low side.
__device__ inline int64_t strip_elem(const StepParams& p, int F, const int* l, int S) {
  const int a = F >> 1;
  const int b = edge_of(p, a);
  const int la = sel3(a, l[0], l[1], l[2]);
  const int d = (F & 1) ? la - (b - S) : la;
  if (a == 0) return (static_cast<int64_t>(l[2]) * p.by + l[1]) * S + d;
  if (a == 1) return (static_cast<int64_t>(l[2]) * S + d) * p.bx + l[0];
  return (static_cast<int64_t>(d) * p.by + l[1]) * p.bx + l[0];
}

// Ring index of the strip value of face F at PE coordinates l (in that strip):
// x faces plane z, [y][d]; y faces plane z, [d][x]; z faces plane d, [y][x].
__device__ inline int64_t ring_at_pt(const StepParams& p, int slot, int pe, int F, const int* l, int S) {
  const int a = F >> 1;
  const int b = edge_of(p, a);
  const int la = sel3(a, l[0], l[1], l[2]);
  const int d = (F & 1) ? la - (b - S) : la;
  if (a == 0) return ring_index(p, slot, pe, F, l[2], static_cast<int64_t>(l[1]) * S + d);
  if (a == 1) return ring_index(p, slot, pe, F, l[2], static_cast<int64_t>(d) * p.bx + l[0]);
  return ring_index(p, slot, pe, F, d, static_cast<int64_t>(l[1]) * p.bx + l[0]);
}

// Strip value t of the per-PE numbering used by the strip kernel
// and the halo buffer: PE pe, face F (its strip starts at pfo[F] inside the
// PE's pe_block values), depth d from the strip's low side and the other PE
// coordinates in l (l[F >> 1] = 0). 32-bit: the host keeps npe * pe_block
// below 2^31.
struct StripPt {
  int pe, F, d;
  int l[3];
};

template <int S>
__device__ inline StripPt strip_point(const AdjParams& q, int t) {
  const StepParams& p = q.sp;
  const int blk = static_cast<int>(p.pe_block);
  StripPt s;
  s.pe = t / blk;
  const int r = t - s.pe * blk;
  int F = 0, off = 0;
#pragma unroll
  for (int f = 1; f < 6; ++f) {
    const bool past = f < 2 * p.ndim && r >= static_cast<int>(q.pfo[f]);
    F += past ? 1 : 0;
    off = past ? static_cast<int>(q.pfo[f]) : off;
  }
  s.F = F;
  const int e = r - off;
  const int a = F >> 1;
  s.l[0] = s.l[1] = s.l[2] = 0;
  if (a == 0) {
    s.d = e % S;
    s.l[1] = (e / S) % p.by;
    s.l[2] = e / (p.by * S);
  } else if (a == 1) {
    s.l[0] = e % p.bx;
    s.d = (e / p.bx) % S;
    s.l[2] = e / (p.bx * S);
  } else {
    s.l[0] = e % p.bx;
    s.l[1] = (e / p.bx) % p.by;
    s.d = e / (p.bx * p.by);
  }
  return s;
}

__device__ inline int nbr_pe(const StepParams& p, int pid, int f) {
  int q[3] = {pid % p.px, (pid / p.px) % p.py, pid / (p.px * p.py)};
  const int a = f >> 1;
  const int ext = sel3(a, p.px, p.py, p.pz);
  set3(q, a, (sel3(a, q[0], q[1], q[2]) + ((f & 1) ? 1 : ext - 1)) % ext);
  return q[0] + p.px * (q[1] + p.py * q[2]);
}

// Delay of face f of PE pid at step n; the synchronous scheme is k = 0 with
// a single level.
__device__ inline int adj_delay(const StepParams& p, int pid, int f, int64_t n) {
  int k = 0;
  if (p.mode == AT_DELAY_RNG)
    k = raw_delay(p.key, n, static_cast<uint32_t>(pid * 2 * p.ndim + f), p.thr, p.L);
  else if (p.mode == AT_DELAY_HOST)
    k = p.host_delays[(n * p.npe + pid) * (2 * p.ndim) + f];
  else
    return 0;
  return clamp_startup(k, n, p.T);
}

__device__ inline int adj_levels(const StepParams& p) { return p.mode == AT_SYNC ? 1 : p.T; }

// mu = dJ/dF of this stage at point g: m0 y0 + m1 y1, formed where it is
// used. Without a second field (m1 = 0) y1 falls back to y0, so both loads
// are unconditional and the m1 term is an exact zero for finite y0.
template <typename Real>
__device__ inline double mu_at(const AdjParams& q, int64_t g) {
  const Real* y0 = static_cast<const Real*>(q.y0);
  const Real* y1 = static_cast<const Real*>(q.m1 != 0.0 ? q.y1 : q.y0);
  return q.m0 * static_cast<double>(y0[g]) + q.m1 * static_cast<double>(y1[g]);
}

template <typename Real>
__device__ inline double centre_at(const AdjParams& q, int64_t g) {
  return static_cast<double>(static_cast<const Real*>(q.levels)[(q.n - q.seg_start) * q.npts + g]);
}

// Tap K_{i,a,o} at a consumer point with stage value ci.
__device__ inline double tap_k(const AdjParams& q, int a, int o, double ci) {
  const StepParams& p = q.sp;
  if (q.burgers) return p.alpha * p.c2[a][o + p.s] - ci * p.c1[a][o + p.s];
  return p.kad[a][o + p.s];
}

// Scatter of step n (gather form): every strip value e of face F of PE q
// collects the transposed taps of the consumer PE across F, weighted by the
// consumer's level weights, into the adjoint ring slots of levels n-k-m.
template <typename Real, int S>
__device__ inline void scatter_elem(const AdjParams& q, const StripPt& sp, const double (*wt)[kMaxT],
                                    Real* drain = nullptr) {
  const StepParams& p = q.sp;
  Real* aring = static_cast<Real*>(q.aring);
  const int pe = sp.pe, F = sp.F, d = sp.d, a = F >> 1;
  const int* l = sp.l;
  const int b = edge_of(p, a);
  // the consumer across F reads this strip through its opposite face
  const int cons = nbr_pe(p, pe, F);
  const int cf = F ^ 1;
  // coordinate of the strip value in the consumer's frame
  const int jp = (F & 1) ? d - S : b + d;
  const int cq[3] = {cons % p.px, (cons / p.px) % p.py, cons / (p.px * p.py)};
  const int org[3] = {cq[0] * p.bx, cq[1] * p.by, cq[2] * p.bz};
  // taps from consumer points outside the consumer PE are dropped by a
  // select after unconditional loads from a clamped (in-PE) point, so that
  // every load of the element is in flight together
  double g = 0.0;
#pragma unroll
  for (int o = -S; o <= S; ++o) {
    if (o == 0) continue;
    const int ia = jp - o;
    const bool valid = ia >= 0 && ia < b;
    int c[3] = {org[0] + l[0], org[1] + l[1], org[2] + l[2]};
    set3(c, a, sel3(a, org[0], org[1], org[2]) + min(max(ia, 0), b - 1));
    const int64_t gi = gindex(p, c[0], c[1], c[2]);
    const double ci = q.burgers ? centre_at<Real>(q, gi) : 0.0;   // Burgers taps only
    const double t = tap_k(q, a, o, ci) * mu_at<Real>(q, gi);
    g += valid ? t : 0.0;
  }
  const int k = adj_delay(p, cons, cf, q.n);
  const double* w = wt[k];
  const int T = adj_levels(p);
  int lsF[3] = {l[0], l[1], l[2]};   // the strip value's PE coordinates
  set3(lsF, a, (F & 1) ? b - S + d : d);
  Real* dst[kMaxT];
  double old[kMaxT];
#pragma unroll
  for (int m = 0; m < kMaxT; ++m) {
    if (m >= T) break;
    // level n - k - m (before t = 0 only where w[m] = 0: any slot is read)
    const int slot = slot_back(static_cast<int>(q.n % q.anslots), k + m, q.anslots);
    dst[m] = aring + ring_at_pt(p, slot, pe, F, lsF, S);
    old[m] = static_cast<double>(*dst[m]);
  }
  // the level-n entry, read with the others (before the taps' sum is used)
  Real* en = nullptr;
  Real en_old = Real(0);
  if (drain) {
    en = aring + ring_at_pt(p, static_cast<int>(q.n % q.anslots), pe, F, lsF, S);
    en_old = *en;
  }
  if (drain) {
    // the caller drains level n here: its entry (this step's contribution
    // added when k = 0, as below) goes to *drain and the ring entry is
    // cleared; only older levels stay in the ring
    *drain = k == 0 ? static_cast<Real>(old[0] + w[0] * g) : en_old;
    *en = Real(0);
#pragma unroll
    for (int m = 0; m < kMaxT; ++m) {
      if (m >= T) break;
      if (k + m > 0 && w[m] != 0.0) *dst[m] = static_cast<Real>(old[m] + w[m] * g);
    }
    return;
  }
#pragma unroll
  for (int m = 0; m < kMaxT; ++m) {
    if (m >= T) break;
    if (w[m] != 0.0) *dst[m] = static_cast<Real>(old[m] + w[m] * g);
  }
}

// Value of level l (ring slot `slot`) at global point (x, y, z), which lies in
// PE `src` at PE coordinates ls: from the stored levels of the segment, or,
// for a level before the segment, from the ring as it was at the segment's
// start (the point is then an edge value of that ring, read through producer
// face pf).
template <typename Real>
__device__ inline double level_value(const AdjParams& q, int64_t l, int slot, int x, int y, int z, int src,
                                     int pf, const int* ls) {
  const StepParams& p = q.sp;
  // both candidates are loaded (from in-range addresses) and one is selected
  const bool stored = l >= q.seg_start;
  const Real* U = static_cast<const Real*>(q.levels) + (stored ? l - q.seg_start : 0) * q.npts;
  const double a = static_cast<double>(U[gindex(p, x, y, z)]);
  const Real* R0 = static_cast<const Real*>(q.ring0);
  const double b = static_cast<double>(R0[ring_at_pt(p, slot, src, pf, ls, p.s)]);
  return stored ? a : b;
}

// The forward halo values of step n, for the alpha-derivative: for every
// consumer PE, face f and element e of the producer strip it reads, the AT
// combination of the stored levels (the synchronous scheme: level n).
// hbuf[pe * pe_block + (per-PE offset of face f) + e].
template <typename Real, int S>
__device__ inline Real halo_value(const AdjParams& q, const StripPt& sp, const double (*wt)[kMaxT]) {
  const StepParams& p = q.sp;
  const int T = adj_levels(p);
  const int pe = sp.pe, f = sp.F, d = sp.d, a = f >> 1, pf = f ^ 1;
  int ls[3] = {sp.l[0], sp.l[1], sp.l[2]};
  const int b = edge_of(p, a);
  set3(ls, a, (pf & 1) ? b - S + d : d);
  const int src = nbr_pe(p, pe, f);
  const int sq[3] = {src % p.px, (src / p.px) % p.py, src / (p.px * p.py)};
  const int gx = sq[0] * p.bx + ls[0], gy = sq[1] * p.by + ls[1], gz = sq[2] * p.bz + ls[2];
  const int k = adj_delay(p, pe, f, q.n);
  const double* w = wt[k];
  if (p.mode == AT_SYNC)   // level n, always stored
    return static_cast<const Real*>(q.levels)[(q.n - q.seg_start) * q.npts + gindex(p, gx, gy, gz)];
  // all kMaxT levels are loaded unconditionally (a level m >= T repeats
  // level T - 1 and is dropped below), so the loads overlap
  const int rn = static_cast<int>(q.n % p.nslots);
  double lv[kMaxT];
#pragma unroll
  for (int m = 0; m < kMaxT; ++m)
    lv[m] = level_value<Real>(q, q.n - k - min(m, T - 1), slot_back(rn, k + min(m, T - 1), p.nslots), gx, gy,
                              gz, src, pf, ls);
  double v = 0.0;
#pragma unroll
  for (int m = 0; m < kMaxT; ++m)
    if (m < T && w[m] != 0.0) v += w[m] * lv[m];
  return static_cast<Real>(v);
}

template <typename Real, int S>
__device__ inline void halo_elem(const AdjParams& q, int t, const StripPt& sp, const double (*wt)[kMaxT]) {
  static_cast<Real*>(q.hbuf)[t] = halo_value<Real, S>(q, sp, wt);
}

// One thread per strip value t: its forward halo value (consumer view) and its
// adjoint-ring scatter (producer view) share the decode of t.
template <typename Real, int S>
__global__ __launch_bounds__(kAdjThreads) void adj_strip_kernel(AdjParams q) {
  // the level weights c_m(k) of every delay k < L (the delays are clamped
  // below L), once per workgroup
  __shared__ double s_wt[kMaxL][kMaxT];
  if (threadIdx.x < kMaxL * kMaxT) s_wt[threadIdx.x / kMaxT][threadIdx.x % kMaxT] = q.wt[threadIdx.x / kMaxT][threadIdx.x % kMaxT];
  __syncthreads();
  const int total = q.sp.npe * static_cast<int>(q.sp.pe_block);
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < total; t += gridDim.x * blockDim.x) {
    const StripPt sp = strip_point<S>(q, t);
    halo_elem<Real, S>(q, t, sp, s_wt);
    scatter_elem<Real, S>(q, sp, s_wt);
  }
}

// The stage adjoint out = b0 x0 + b1 x1 + D mu + transposed taps + the adjoint
// ring slot of level n (drained and cleared here), plus this stage's part of
// dJ/dalpha. Branch-free per point: every lane issues the same loads, a tap
// that leaves the PE selects the address of its halo value (or of a value it
// then multiplies by zero), so PE-edge points cost what interior points cost.
template <typename Real, int DIM, int S>
__global__ __launch_bounds__(kAdjThreads) void adj_lambda_kernel(AdjParams q) {
  const StepParams& p = q.sp;
  Real* __restrict__ out = static_cast<Real*>(q.out);
  const Real* __restrict__ x0 = static_cast<const Real*>(q.x0);
  // with b1 = 0, x1 falls back to x0 (an exact zero term for finite x0)
  const Real* __restrict__ x1 = static_cast<const Real*>(q.b1 != 0.0 ? q.x1 : q.x0);
  const Real* __restrict__ C = static_cast<const Real*>(q.levels) + (q.n - q.seg_start) * q.npts;
  const Real* __restrict__ hb = static_cast<const Real*>(q.hbuf);
  Real* __restrict__ aring = static_cast<Real*>(q.aring);
  const int slot_n = static_cast<int>(q.n % q.anslots);
  const int64_t st[3] = {1, p.nx, static_cast<int64_t>(p.nx) * p.ny};
  double da = 0.0;
  for (int64_t g = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; g < q.npts;
       g += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const Pt j = point_of(p, g);
    const double mu = mu_at<Real>(q, g);
    const double cj = static_cast<double>(C[g]);
    const double v1 = static_cast<double>(x1[g]);
    double acc = q.b0 * static_cast<double>(x0[g]) + q.b1 * v1;
    double lap = 0.0, grad = 0.0, sumk = 0.0;
    const Real* hpe = hb + static_cast<int64_t>(j.pe) * p.pe_block;
    // adjoint-ring entries of the strips j belongs to: every load of the
    // point is issued before the entries are cleared at the end
    Real* rsrc[2 * DIM];
    bool rin[2 * DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      const int b = edge_of(p, a);
#pragma unroll
      for (int o = -S; o <= S; ++o) {
        if (o == 0) continue;
        sumk += tap_k(q, a, o, cj);
        // transposed interior tap: from i = j - o when i lies in the PE
        const int ia = j.l[a] - o;
        const bool tin = ia >= 0 && ia < b;
        const int64_t gi = tin ? g - o * st[a] : g;
        const double mi = mu_at<Real>(q, gi);
        // the stage value at i enters the Burgers taps only (uniform branch)
        const double ci = q.burgers ? static_cast<double>(C[gi]) : 0.0;
        acc += tin ? tap_k(q, a, o, ci) * mi : 0.0;
        // forward stencil of the stage field at j: inside the PE from the
        // field, across a face from the stage's combined halo values
        const int ta = j.l[a] + o;
        const bool fin = ta >= 0 && ta < b;
        const int side = ta < 0 ? 0 : 1;
        int ls[3] = {j.l[0], j.l[1], j.l[2]};
        ls[a] = fin ? (side ? b - S : 0) : (side ? ta - b : ta + b);
        const int f = 2 * a + side;
        const int64_t pfo = side ? q.pfo[2 * a + 1] : q.pfo[2 * a];   // uniform values, no indexed load
        const Real* pv = fin ? C + (g + o * st[a]) : hpe + pfo + strip_elem(p, f ^ 1, ls, S);
        const double v = static_cast<double>(*pv) - cj;
        lap += p.c2[a][o + S] * v;
        grad += p.c1[a][o + S] * v;
      }
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        const bool in = side ? j.l[a] >= b - S : j.l[a] < S;
        int ls[3] = {j.l[0], j.l[1], j.l[2]};
        if (!in) ls[a] = side ? b - S : 0;
        Real* src = aring + ring_at_pt(p, slot_n, j.pe, 2 * a + side, ls, S);
        const double r = static_cast<double>(*src);
        acc += in ? r : 0.0;
        rsrc[2 * a + side] = src;
        rin[2 * a + side] = in;
      }
    }
#pragma unroll
    for (int f = 0; f < 2 * DIM; ++f)
      if (rin[f]) *rsrc[f] = Real(0);
    // D_j mu_j with D_j = -sum K (- G_j for Burgers)
    acc += (-sumk - (q.burgers ? grad : 0.0)) * mu;
    out[g] = static_cast<Real>(acc);
    da += mu * lap;
  }
  // fixed-order block reduction of the alpha-gradient part
  for (int off = 32; off > 0; off >>= 1) da += __shfl_down(da, off, 64);
  __shared__ double part[kAdjThreads / 64];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x / 64] = da;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kAdjThreads / 64; ++w) s += part[w];
    q.partial[blockIdx.x] += s;
  }
}

// PE-tiled form of adj_lambda_kernel (same formula, same per-point order of
// the sums): one workgroup per PE, every global value loaded once.
//  - 1-D / 2-D: the PE's plane in LDS: the stage values c with the frame of
//    forward halo values the stencil reads across the PE's faces, and the two
//    mu fields y0, y1 with a zero frame (taps of consumer points outside the
//    PE reach this point through the adjoint ring instead). The workgroup
//    first does its PE's strip work (the halo values straight into the frame,
//    the gather-form scatter into its own adjoint-ring entries, the level-n
//    drains into LDS), so no strip kernel runs before it.
//  - 3-D: each thread owns one (x, y) column of the PE and streams it in z
//    with register queues of 2S+1 planes of c, y0 and y1 (the z halo values
//    of c from hbuf, zeros for y0 and y1 beyond the PE), the x/y neighbours
//    from a double-buffered LDS plane laid out like the 2-D one. The loads of
//    the plane S+1 ahead are in flight while a plane is computed.
// The alpha-gradient part of the workgroup goes to partial[PE].
constexpr int kAdjPeThreads = 1024;

template <typename Real, int DIM, int S>
__global__ __launch_bounds__(kAdjPeThreads) void adj_lambda_pe_kernel(AdjParams q) {
  const StepParams& p = q.sp;
  extern __shared__ __align__(16) unsigned char adj_smem[];
  const int pe = blockIdx.x;
  const int qx = pe % p.px, qy = (pe / p.px) % p.py, qz = pe / (p.px * p.py);
  const int bx = p.bx, by = DIM >= 2 ? p.by : 1, bz = DIM == 3 ? p.bz : 1;
  const int x0 = qx * p.bx, y0 = qy * p.by, z0 = qz * p.bz;
  const int W = bx + 2 * S, H = DIM >= 2 ? by + 2 * S : 1;   // LDS plane: rows of W, x = 0 at column S
  const int plane = W * H;
  const int nbuf = DIM == 3 ? 2 : 1;
  Real* Cl = reinterpret_cast<Real*>(adj_smem);            // [nbuf][plane]
  Real* Y0l = Cl + nbuf * plane;
  Real* Y1l = Y0l + nbuf * plane;
  Real* __restrict__ out = static_cast<Real*>(q.out);
  const Real* __restrict__ X0 = static_cast<const Real*>(q.x0);
  const Real* __restrict__ X1 = static_cast<const Real*>(q.b1 != 0.0 ? q.x1 : q.x0);
  const Real* __restrict__ Yg0 = static_cast<const Real*>(q.y0);
  const Real* __restrict__ Yg1 = static_cast<const Real*>(q.m1 != 0.0 ? q.y1 : q.y0);
  const Real* __restrict__ C = static_cast<const Real*>(q.levels) + (q.n - q.seg_start) * q.npts;
  // (not restrict: in 1-D / 2-D this kernel writes both through the strip
  // work's own pointers first)
  const Real* hpe = static_cast<const Real*>(q.hbuf) + static_cast<int64_t>(pe) * p.pe_block;
  Real* aring = static_cast<Real*>(q.aring);
  const int slot_n = static_cast<int>(q.n % q.anslots);
  const int tid = threadIdx.x, nt = blockDim.x;
  const double m0 = q.m0, m1 = q.m1;
  // taps in LDS (read with uniform addresses where a point needs them)
  __shared__ double s_c1[3][2 * S + 1], s_c2a[3][2 * S + 1], s_kad[3][2 * S + 1], s_c2[3][2 * S + 1];
  if (tid < 3 * (2 * S + 1)) {
    const int a = tid / (2 * S + 1), o = tid % (2 * S + 1);
    s_c1[a][o] = p.c1[a][o];
    s_c2[a][o] = p.c2[a][o];
    s_c2a[a][o] = p.alpha * p.c2[a][o];
    s_kad[a][o] = p.kad[a][o];
  }
  const bool burg = q.burgers != 0;
  // tap K_{i,a,o} at a point with stage value ci (as tap_k)
  auto tapk = [&](int a, int o, double ci) -> double {
    return burg ? s_c2a[a][o + S] - ci * s_c1[a][o + S] : s_kad[a][o + S];
  };
  // forward halo value across face f (a = f >> 1) for the PE coordinates l
  // whose axis-a coordinate ta lies outside the PE
  auto halo_c = [&](int f, int* l, int ta) -> Real {
    const int a = f >> 1, b = a == 0 ? bx : a == 1 ? by : bz;
    set3(l, a, (f & 1) ? ta - b : ta + b);
    const int64_t pfo = f == 0 ? q.pfo[0] : f == 1 ? q.pfo[1] : f == 2 ? q.pfo[2] : f == 3 ? q.pfo[3]
                      : f == 4 ? q.pfo[4] : q.pfo[5];
    return hpe[pfo + strip_elem(p, f ^ 1, l, S)];
  };
  // zero frames of y0, y1; the x/y halo frame of c is written per plane
  for (int i = tid; i < nbuf * plane; i += nt) {
    Y0l[i] = Real(0);
    Y1l[i] = Real(0);
  }
  // 1-D / 2-D: the level weights c_m(k) of every k < L for the strip work
  __shared__ double s_wt[kMaxL][kMaxT];
  if (DIM <= 2 && tid < kMaxL * kMaxT) s_wt[tid / kMaxT][tid % kMaxT] = q.wt[tid / kMaxT][tid % kMaxT];
  __syncthreads();   // the zeros land before any own value is written over them
  // the per-point adjoint (x, y, z PE coordinates; global index g); cget(a, o)
  // / yget(a, o) give c and (y0, y1) at offset o along axis a
  double da = 0.0;
  // dr: the adjoint-ring entries of the strips the point lies in, one per
  // axis (dr[a], where din[a]), loaded (and cleared) by the caller; nullptr:
  // loaded and cleared here
  auto point = [&](int x, int y, int z, int64_t g, double cj, double y0j, double y1j, double x0j, double x1j,
                   auto cget, auto yget, const Real* dr, const bool* din) {
    const double mu = m0 * y0j + m1 * y1j;
    double acc = q.b0 * x0j + q.b1 * x1j;
    double lap = 0.0, grad = 0.0, sumk = 0.0;
    const int l[3] = {x, y, z};
    // the taps of axis a: from the kernel arguments where a is a compile-time
    // constant (scalar registers), else from LDS (uniform addresses)
    auto axis = [&](int a, auto args) {
      constexpr bool kArgs = decltype(args)::value;
      const int b = a == 0 ? bx : a == 1 ? by : bz;
      auto c1t = [&](int o) -> double { return kArgs ? p.c1[a][o + S] : s_c1[a][o + S]; };
      auto c2t = [&](int o) -> double { return kArgs ? p.c2[a][o + S] : s_c2[a][o + S]; };
      auto tk = [&](int o, double ci) -> double {
        if (!kArgs) return tapk(a, o, ci);
        return burg ? p.alpha * p.c2[a][o + S] - ci * p.c1[a][o + S] : p.kad[a][o + S];
      };
#pragma unroll
      for (int o = -S; o <= S; ++o) {
        if (o == 0) continue;
        sumk += tk(o, cj);
        // transposed interior tap from i = j - o (zero mu outside the PE)
        double yi0, yi1;
        yget(a, -o, yi0, yi1);
        const double mi = m0 * yi0 + m1 * yi1;
        const double ci = burg ? cget(a, -o) : 0.0;
        const int ia = l[a] - o;
        acc += (ia >= 0 && ia < b) ? tk(o, ci) * mi : 0.0;
        // forward stencil of the stage field at j
        const double v = cget(a, o) - cj;
        lap += c2t(o) * v;
        grad += c1t(o) * v;
      }
    };
    if constexpr (DIM <= 2) {
#pragma unroll
      for (int a = 0; a < DIM; ++a) axis(a, std::true_type{});
    } else {
      // one axis at a time (not unrolled over axes: bounds the values in flight)
#pragma unroll 1
      for (int a = 0; a < DIM; ++a) axis(a, std::false_type{});
    }
    // drain the adjoint-ring entries of the strips j lies in
    if (dr) {
#pragma unroll
      for (int a = 0; a < DIM; ++a)
        if (din[a]) acc += static_cast<double>(dr[a]);
    } else {
#pragma unroll
      for (int a = 0; a < DIM; ++a) {
        const int b = a == 0 ? bx : a == 1 ? by : bz;
#pragma unroll
        for (int side = 0; side < 2; ++side) {
          if (side ? l[a] >= b - S : l[a] < S) {
            Real* src = aring + ring_at_pt(p, slot_n, pe, 2 * a + side, l, S);
            acc += static_cast<double>(*src);
            *src = Real(0);
          }
        }
      }
    }
    acc += (-sumk - (burg ? grad : 0.0)) * mu;
    out[g] = static_cast<Real>(acc);
    da += mu * lap;
  };

  if constexpr (DIM <= 2) {
    // A thread's first kPre points: their base terms are loaded with the plane
    constexpr int kPre = sizeof(Real) == 4 ? 4 : 3;
    Real pre_x0[kPre], pre_x1[kPre];
#pragma unroll
    for (int k = 0; k < kPre; ++k) {
      const int i = tid + k * nt;
      pre_x0[k] = pre_x1[k] = Real(0);
      if (i < bx * by) {
        const int y = i / bx, x = i - y * bx;
        const int64_t g = gindex(p, x0 + x, y0 + y, 0);
        pre_x0[k] = X0[g];
        pre_x1[k] = X1[g];
      }
    }
    // the plane's own values: a thread's first kPre points are loaded into
    // registers here and stored to LDS after the strip work, so that those
    // loads and the strip work's are in flight together
    Real pc[kPre], p0[kPre], p1[kPre];
#pragma unroll
    for (int k = 0; k < kPre; ++k) {
      const int i = tid + k * nt;
      pc[k] = p0[k] = p1[k] = Real(0);
      if (i < bx * by) {
        const int y = i / bx, x = i - y * bx;
        const int64_t g = gindex(p, x0 + x, y0 + y, 0);
        pc[k] = C[g];
        p0[k] = Yg0[g];
        p1[k] = Yg1[g];
      }
    }
    for (int i = tid + kPre * nt; i < bx * by; i += nt) {
      const int y = i / bx, x = i - y * bx;
      const int64_t g = gindex(p, x0 + x, y0 + y, 0);
      const int at = (DIM >= 2 ? y + S : 0) * W + x + S;
      Cl[at] = C[g];
      Y0l[at] = Yg0[g];
      Y1l[at] = Yg1[g];
    }
    // This PE's strip values (the strip kernel's work, which only this
    // workgroup touches), behind the plane's loads. Items 0..blk-1: the
    // forward halo value that this PE reads across its face f (consumer
    // view), straight into the frame of the LDS plane. Items blk..2 blk-1:
    // in gather form, the transposed taps of the neighbour that reads this
    // PE's strip value into its older adjoint-ring levels, and the drained
    // level-n entry (this step's contribution included) into Dl, clearing
    // the ring entry. The two halves run in different waves side by side.
    Real* Dl = Y1l + nbuf * plane;                        // [pe_block]
    {
      const int blk = static_cast<int>(p.pe_block);
      for (int r = tid; r < 2 * blk; r += nt) {
        const bool scat = r >= blk;
        const int rr = scat ? r - blk : r;
        const StripPt sp = strip_point<S>(q, pe * blk + rr);
        if (scat) {
          scatter_elem<Real, S>(q, sp, s_wt, Dl + rr);
        } else {
          // frame position of the value: depth d of the producer strip is
          // column d - S (low face) or b + d (high face) along its axis
          const int a = sp.F >> 1, b = a == 0 ? bx : by;
          const int ta = (sp.F & 1) ? b + sp.d : sp.d - S;
          const int at = a == 0 ? (DIM >= 2 ? sp.l[1] + S : 0) * W + ta + S : (ta + S) * W + sp.l[0] + S;
          Cl[at] = halo_value<Real, S>(q, sp, s_wt);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < kPre; ++k) {
      const int i = tid + k * nt;
      if (i < bx * by) {
        const int y = i / bx, x = i - y * bx;
        const int at = (DIM >= 2 ? y + S : 0) * W + x + S;
        Cl[at] = pc[k];
        Y0l[at] = p0[k];
        Y1l[at] = p1[k];
      }
    }
    __syncthreads();
    // the drained level-n entries of a point's strips (x, y), from Dl
    auto drains = [&](int x, int y, Real* dr, bool* din) {
      const int l[3] = {x, y, 0};
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        din[a] = false;
        dr[a] = Real(0);
        if (a < DIM) {
          const int b = a == 0 ? bx : by, la = a == 0 ? x : y;
          const bool lo = la < S, hi = la >= b - S;
          if (lo || hi) {
            const int F = 2 * a + (hi ? 1 : 0);
            const int64_t pfo = F == 0 ? q.pfo[0] : F == 1 ? q.pfo[1] : F == 2 ? q.pfo[2] : q.pfo[3];
            din[a] = true;
            dr[a] = Dl[pfo + strip_elem(p, F, l, S)];
          }
        }
      }
    };
    auto plane_point = [&](int i, Real vx0, Real vx1) {
      const int y = i / bx, x = i - y * bx;
      const int at = (DIM >= 2 ? y + S : 0) * W + x + S;
      auto cget = [&](int a, int o) -> double { return static_cast<double>(Cl[at + (a == 0 ? o : o * W)]); };
      auto yget = [&](int a, int o, double& v0, double& v1) {
        const int k = at + (a == 0 ? o : o * W);
        v0 = static_cast<double>(Y0l[k]);
        v1 = static_cast<double>(Y1l[k]);
      };
      const int64_t g = gindex(p, x0 + x, y0 + y, 0);
      Real dr[2];
      bool din[2];
      drains(x, y, dr, din);
      point(x, y, 0, g, static_cast<double>(Cl[at]), static_cast<double>(Y0l[at]), static_cast<double>(Y1l[at]),
            static_cast<double>(vx0), static_cast<double>(vx1), cget, yget, dr, din);
    };
#pragma unroll
    for (int k = 0; k < kPre; ++k) {
      const int i = tid + k * nt;
      if (i < bx * by) plane_point(i, pre_x0[k], pre_x1[k]);
    }
    for (int i = tid + kPre * nt; i < bx * by; i += nt) {
      const int y = i / bx, x = i - y * bx;
      const int64_t g = gindex(p, x0 + x, y0 + y, 0);
      plane_point(i, X0[g], X1[g]);
    }
  } else {
    // one column per thread (the host launches bx * by threads)
    const int x = tid % bx, y = tid / bx;
    const int at = (y + S) * W + x + S;
    const int64_t col = gindex(p, x0 + x, y0 + y, z0);
    const int64_t zs = static_cast<int64_t>(p.nx) * p.ny;
    // values of plane zz (from -S to bz + S - 1): own planes from memory,
    // beyond the PE's z faces c from the halo buffer and y0 = y1 = 0
    auto fetch = [&](int zz, Real& cv, Real& a0, Real& a1) {
      if (zz >= 0 && zz < bz) {
        const int64_t g = col + zz * zs;
        cv = C[g];
        a0 = Yg0[g];
        a1 = Yg1[g];
      } else {
        int l[3] = {x, y, 0};
        cv = halo_c(zz < 0 ? 4 : 5, l, zz);
        a0 = a1 = Real(0);
      }
    };
    Real cq[2 * S + 1], yq0[2 * S + 1], yq1[2 * S + 1];
#pragma unroll
    for (int i = 0; i < 2 * S; ++i) fetch(i - S, cq[i], yq0[i], yq1[i]);
    Real pc, p0, p1;   // plane S ahead, prefetched
    fetch(S, pc, p0, p1);
    // x and y frame of c: thread h < nf owns one frame element of every plane
    // (its LDS position, and its halo-buffer address of plane 0 plus a
    // per-plane stride: x strips [z][y][d], y strips [z][d][x]); the value of
    // the next plane is loaded while a plane is computed
    const int nf = 2 * S * (by + bx);
    const bool has_f = tid < nf;
    int f_at = 0;
    int64_t f_addr = 0, f_stride = 0;
    if (has_f) {
      int l[3] = {0, 0, 0};
      int f, ta;
      if (tid < 2 * S * by) {
        const int side = tid >= S * by ? 1 : 0, r = side ? tid - S * by : tid, yy = r / S, d = r - yy * S;
        ta = side ? bx + d : d - S;
        l[1] = yy;
        f = side;
        f_at = (yy + S) * W + ta + S;
        f_stride = static_cast<int64_t>(by) * S;
      } else {
        const int hy = tid - 2 * S * by, side = hy >= S * bx ? 1 : 0, r = side ? hy - S * bx : hy;
        const int d = r / bx, xx = r - d * bx;
        ta = side ? by + d : d - S;
        l[0] = xx;
        f = 2 + side;
        f_at = (ta + S) * W + xx + S;
        f_stride = static_cast<int64_t>(S) * bx;
      }
      const int a = f >> 1, b = a == 0 ? bx : by;
      set3(l, a, (f & 1) ? ta - b : ta + b);
      const int64_t pfo = f == 0 ? q.pfo[0] : f == 1 ? q.pfo[1] : f == 2 ? q.pfo[2] : q.pfo[3];
      f_addr = pfo + strip_elem(p, f ^ 1, l, S);
    }
    Real fv = has_f ? hpe[f_addr] : Real(0);
    // base terms of the point, one plane ahead
    Real xv0 = X0[col], xv1 = X1[col];
    for (int z = 0; z < bz; ++z) {
      const Real xc0 = xv0, xc1 = xv1;
      if (z + 1 < bz) {
        xv0 = X0[col + (z + 1) * zs];
        xv1 = X1[col + (z + 1) * zs];
      }
      cq[2 * S] = pc;
      yq0[2 * S] = p0;
      yq1[2 * S] = p1;
      if (z + S + 1 < bz + S) fetch(z + S + 1, pc, p0, p1);
      Real* Cp = Cl + (z & 1) * plane;
      Real* P0 = Y0l + (z & 1) * plane;
      Real* P1 = Y1l + (z & 1) * plane;
      Cp[at] = cq[S];
      P0[at] = yq0[S];
      P1[at] = yq1[S];
      if (has_f) {
        Cp[f_at] = fv;
        if (z + 1 < bz) fv = hpe[f_addr + (z + 1) * f_stride];
      }
      __syncthreads();
      auto cget = [&](int a, int o) -> double {
        return static_cast<double>(a == 2 ? cq[S + o] : Cp[at + (a == 0 ? o : o * W)]);
      };
      auto yget = [&](int a, int o, double& v0, double& v1) {
        if (a == 2) {
          v0 = static_cast<double>(yq0[S + o]);
          v1 = static_cast<double>(yq1[S + o]);
        } else {
          const int k = at + (a == 0 ? o : o * W);
          v0 = static_cast<double>(P0[k]);
          v1 = static_cast<double>(P1[k]);
        }
      };
      point(x, y, z, col + z * zs, static_cast<double>(cq[S]), static_cast<double>(yq0[S]),
            static_cast<double>(yq1[S]), static_cast<double>(xc0), static_cast<double>(xc1), cget, yget,
            static_cast<const Real*>(nullptr), static_cast<const bool*>(nullptr));
#pragma unroll
      for (int i = 0; i < 2 * S; ++i) {
        cq[i] = cq[i + 1];
        yq0[i] = yq0[i + 1];
        yq1[i] = yq1[i + 1];
      }
    }
  }
  // fixed-order block reduction of the alpha-gradient part
  for (int off = 32; off > 0; off >>= 1) da += __shfl_down(da, off, 64);
  __shared__ double part[kAdjPeThreads / 64];
  if ((tid & 63) == 0) part[tid / 64] = da;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int w = 0; w < nt / 64; ++w) s += part[w];
    q.partial[pe] += s;
  }
}

template <typename Real>
size_t adj_pe_lds(const StepParams& p) {
  const int S = p.s;
  const size_t W = p.bx + 2 * S, H = p.ndim >= 2 ? p.by + 2 * S : 1;
  // 1-D / 2-D: plus the drained adjoint-ring entries of the PE's strips
  return (p.ndim == 3 ? 2 : 1) * 3 * W * H * sizeof(Real) +
         (p.ndim <= 2 ? static_cast<size_t>(p.pe_block) * sizeof(Real) : 0);
}

template <typename Real>
hipError_t launch_lambda_pe(const AdjParams& q, hipStream_t st) {
  const StepParams& p = q.sp;
  const size_t lds = adj_pe_lds<Real>(p);
  const int pts = p.bx * (p.ndim >= 2 ? p.by : 1);
  const int threads = p.ndim == 3 ? (pts + 63) / 64 * 64 : std::min(kAdjPeThreads, (pts + 63) / 64 * 64);
  // 3-D: every frame element of a plane has its own thread
  if (p.ndim == 3 && 2 * p.s * (p.bx + p.by) > threads) return hipErrorInvalidValue;
  const int key = p.ndim * 10 + p.s;
  switch (key) {
#define ATFD_ADJ_PE_CASE(D, S)                                                                          \
  case D * 10 + S:                                                                                      \
    hipLaunchKernelGGL((adj_lambda_pe_kernel<Real, D, S>), dim3(p.npe), dim3(threads), lds, st, q);      \
    break;
    ATFD_ADJ_PE_CASE(1, 1) ATFD_ADJ_PE_CASE(1, 2) ATFD_ADJ_PE_CASE(1, 3)
    ATFD_ADJ_PE_CASE(2, 1) ATFD_ADJ_PE_CASE(2, 2) ATFD_ADJ_PE_CASE(2, 3)
    ATFD_ADJ_PE_CASE(3, 1) ATFD_ADJ_PE_CASE(3, 2) ATFD_ADJ_PE_CASE(3, 3)
#undef ATFD_ADJ_PE_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_strip(const AdjParams& q, int blocks, hipStream_t st) {
  switch (q.sp.s) {
    case 1: hipLaunchKernelGGL((adj_strip_kernel<Real, 1>), dim3(blocks), dim3(kAdjThreads), 0, st, q); break;
    case 2: hipLaunchKernelGGL((adj_strip_kernel<Real, 2>), dim3(blocks), dim3(kAdjThreads), 0, st, q); break;
    case 3: hipLaunchKernelGGL((adj_strip_kernel<Real, 3>), dim3(blocks), dim3(kAdjThreads), 0, st, q); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_lambda(const AdjParams& q, int blocks, hipStream_t st) {
  const int key = q.sp.ndim * 10 + q.sp.s;
  switch (key) {
#define ATFD_ADJ_CASE(D, S)                                                                         \
  case D * 10 + S:                                                                                   \
    hipLaunchKernelGGL((adj_lambda_kernel<Real, D, S>), dim3(blocks), dim3(kAdjThreads), 0, st, q); \
    break;
    ATFD_ADJ_CASE(1, 1) ATFD_ADJ_CASE(1, 2) ATFD_ADJ_CASE(1, 3)
    ATFD_ADJ_CASE(2, 1) ATFD_ADJ_CASE(2, 2) ATFD_ADJ_CASE(2, 3)
    ATFD_ADJ_CASE(3, 1) ATFD_ADJ_CASE(3, 2) ATFD_ADJ_CASE(3, 3)
#undef ATFD_ADJ_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// One wave: lane l adds partials l, l + 64, ... in order, then a fixed
// butterfly combines the lanes.
__global__ __launch_bounds__(64) void adj_sum_kernel(const double* partial, int count, double* out) {
  double s = 0.0;
  for (int i = threadIdx.x; i < count; i += 64) s += partial[i];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  if (threadIdx.x == 0) out[0] = s;
}

}  // namespace

int adj_blocks(int64_t npts) {
  const int64_t b = (npts + kAdjThreads - 1) / kAdjThreads;
  return static_cast<int>(b < kAdjBlocks ? b : kAdjBlocks);
}

bool adj_pe_applies(const StepParams& p, bool f64) {
  const size_t lds = f64 ? adj_pe_lds<double>(p) : adj_pe_lds<float>(p);
  if (lds > 64 * 1024) return false;
  // 3-D: one thread per column, whole waves; the FP64 register queues of
  // s >= 2 would spill
  if (p.ndim == 3 && f64 && p.s >= 2) return false;
  return p.ndim <= 2 || (p.bx * p.by <= kAdjPeThreads && (p.bx * p.by) % 64 == 0 &&
                         2 * p.s * (p.bx + p.by) <= p.bx * p.by);
}

hipError_t launch_adj_step(const AdjParams& q, bool f64, hipStream_t st) {
  const int64_t strips = static_cast<int64_t>(q.sp.npe) * q.sp.pe_block;
  const int64_t sb = (strips + kAdjThreads - 1) / kAdjThreads;
  const int sblocks = static_cast<int>(sb < kAdjBlocks ? (sb > 0 ? sb : 1) : kAdjBlocks);
  const int lblocks = adj_blocks(q.npts);
  const bool pe = adj_pe_applies(q.sp, f64);
  // the 1-D / 2-D PE-tiled stage kernel does its PE's strip work itself
  const bool strip_kernel = !(pe && q.sp.ndim <= 2);
  if (f64) {
    if (strip_kernel) {
      hipError_t e = launch_strip<double>(q, sblocks, st);
      if (e != hipSuccess) return e;
    }
    hipError_t e = pe ? launch_lambda_pe<double>(q, st) : launch_lambda<double>(q, lblocks, st);
    if (e != hipSuccess) return e;
  } else {
    if (strip_kernel) {
      hipError_t e = launch_strip<float>(q, sblocks, st);
      if (e != hipSuccess) return e;
    }
    hipError_t e = pe ? launch_lambda_pe<float>(q, st) : launch_lambda<float>(q, lblocks, st);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

int adj_partials(const StepParams& p) { return p.npe > kAdjBlocks ? p.npe : kAdjBlocks; }

hipError_t launch_adj_sum(const double* partial, int count, double* out, hipStream_t st) {
  hipLaunchKernelGGL(adj_sum_kernel, dim3(1), dim3(64), 0, st, partial, count, out);
  return hipGetLastError();
}

}  // namespace atfd
