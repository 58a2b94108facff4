// Error norms of a field against the decaying advected Fourier series (Sec. 5.1
// eq. ana_sol) or against a double reference field, split over the boundary
// set I_B (points within s of a PE face) and the interior set I_I (Sec. 4
// space averages). Accumulation in double: per-thread sums, wave64 butterfly
// shuffles, one partial per workgroup, then a one-wave pass that combines the
// partials in a fixed order, so the result does not depend on scheduling.

#include "atfd_internal.hpp"

#include <mutex>

// Device scratch of the allocation-free norm evaluation (at_norms_noalloc):
// the per-workgroup partials (kNormStaticBlocks x 8 doubles) and the
// 16-double result. One copy per GPU, held until the process ends; calls that
// overlap on one GPU share it and race.
static __device__ __align__(256) double scratch[atfd::kNormStaticBlocks * 8 + 16];

namespace atfd {
namespace {

// partial layout: sum|e| over I_B, sum e^2 over I_B, sum|e| over I_I,
// sum e^2 over I_I, max|e|, non-finite count, (2 spare)
constexpr int kNP = 8;

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ inline double wave_max(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Exact solution sum_m A_m e^{-alpha |kappa_m|^2 t} sin(kappa_m . (x - c t) + phi_m).
// When the per-axis tables fit in LDS, mode m at (x, y, z) is the imaginary
// part of X_m[x] Y_m[y] Z_m[z] with X_m[x] = exp(i kappa_x h_x x), Y likewise
// and Z_m[z] = A_m e^{-alpha |kappa_m|^2 t} exp(i (kappa_z h_z z + phi_m -
// t kappa_m . c)): two complex products per mode and point instead of a sine.
// The boundary-set test is tabulated per axis as well.
constexpr size_t kNormTableBytes = 64 * 1024;

size_t norm_table_bytes(const NormParams& p) {
  const size_t rows = static_cast<size_t>(p.nx) + p.ny + p.nz;
  return static_cast<size_t>(p.nmodes) * rows * sizeof(double2) + ((rows + 15) & ~size_t{15});
}

__device__ inline bool in_boundary_layer(int c, int b, int s) {
  const int l = c % b;
  return l < s || l >= b - s;
}

// Per-point accumulation of the six partial sums.
struct NormAcc {
  double sab = 0, sqb = 0, sai = 0, sqi = 0, mx = 0, bad = 0;
  __device__ void add(double e, bool inb) {
    if (!isfinite(e)) { bad += 1.0; return; }
    const double ae = fabs(e);
    if (inb) { sab += ae; sqb += e * e; } else { sai += ae; sqi += e * e; }
    mx = fmax(mx, ae);
  }
};

template <typename Real, int MaxM, bool Table>
__global__ __launch_bounds__(256) void norms_partial_kernel(NormParams p) {
  extern __shared__ double2 tab[];   // X[m][x], Y[m][y], Z[m][z], then per-axis boundary flags
  const Real* u = static_cast<const Real*>(p.u);
  const double t = static_cast<double>(p.counter[0]) * p.dt;
  const double hx = p.length / p.nx, hy = p.length / p.ny, hz = p.length / p.nz;
  auto shift = [&](int m) {
    return p.phase[m] - t * (p.kap[m][0] * p.vel[0] + p.kap[m][1] * p.vel[1] + p.kap[m][2] * p.vel[2]);
  };
  auto decay = [&](int m) {
    const double k2 = double(p.kap[m][0]) * p.kap[m][0] + double(p.kap[m][1]) * p.kap[m][1] +
                      double(p.kap[m][2]) * p.kap[m][2];
    return p.amp[m] * exp(-p.alpha * k2 * t);
  };
  // offset of point (x, y, z) in the field (ref is always [z][y][x])
  auto at = [&](int x, int y, int z) -> size_t {
    if (p.pe_major) return static_cast<size_t>(pe_major_offset(x, y, z, p.bz, p.px, p.py));
    return (static_cast<size_t>(z) * p.ny + y) * p.nx + x;
  };
  NormAcc acc;
  if constexpr (Table) {
    const int nm = p.nmodes, nx = p.nx, ny = p.ny, nz = p.nz;
    double2* X = tab;
    double2* Y = X + nm * nx;
    double2* Z = Y + nm * ny;
    unsigned char* flag = reinterpret_cast<unsigned char*>(Z + nm * nz);   // [nx + ny + nz]
    const int ntab = nm * (nx + ny + nz);
    for (int i = threadIdx.x; i < ntab; i += blockDim.x) {
      double arg, scale = 1.0;
      if (i < nm * nx) {
        arg = p.kap[i / nx][0] * hx * (i % nx);
      } else if (i < nm * (nx + ny)) {
        const int j = i - nm * nx;
        arg = p.kap[j / ny][1] * hy * (j % ny);
      } else {
        const int j = i - nm * (nx + ny), m = j / nz;
        arg = p.kap[m][2] * hz * (j % nz) + shift(m);
        scale = decay(m);
      }
      double sv, cv;
      sincos(arg, &sv, &cv);
      tab[i] = make_double2(scale * cv, scale * sv);
    }
    for (int i = threadIdx.x; i < nx + ny + nz; i += blockDim.x) {
      bool f;
      if (i < nx) f = in_boundary_layer(i, p.bx, p.s);
      else if (i < nx + ny) f = p.ndim >= 2 && in_boundary_layer(i - nx, p.by, p.s);
      else f = p.ndim == 3 && in_boundary_layer(i - nx - ny, p.bz, p.s);
      flag[i] = f ? 1 : 0;
    }
    __syncthreads();
    // A wave takes a unit of four consecutive x rows times a segment of up to
    // 256 points: it issues the unit's 16 loads per lane first, then forms
    // each row's factor Y_m[y] Z_m[z] once, so a point costs one table read
    // and two multiply-adds per mode. 32-bit indexing: the host takes this
    // path only below 2^31 points.
    constexpr int kSeg = 256, kRows = 4, kPer = kSeg / 64;
    const unsigned nrows = static_cast<unsigned>(ny) * nz;
    const int nseg = (nx + kSeg - 1) / kSeg;
    const unsigned units = (nrows + kRows - 1) / kRows * nseg;
    const int lane = threadIdx.x & 63;
    const unsigned nwaves = gridDim.x * (blockDim.x >> 6);
    for (unsigned w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); w < units; w += nwaves) {
      const unsigned rg = w / nseg;
      const int x0 = static_cast<int>(w - rg * nseg) * kSeg + lane;
      // unconditional loads from clamped (in-range) addresses, so that all 16
      // are in flight together; out-of-range lanes are skipped below
      Real v[kRows][kPer];
#pragma unroll
      for (int g = 0; g < kRows; ++g) {
        const unsigned row = min(rg * kRows + g, nrows - 1);
        const unsigned rz = row / ny;
        const int ry = static_cast<int>(row - rz * ny);
#pragma unroll
        for (int k = 0; k < kPer; ++k) v[g][k] = u[at(min(x0 + 64 * k, nx - 1), ry, static_cast<int>(rz))];
      }
#pragma unroll
      for (int g = 0; g < kRows; ++g) {
        const unsigned row = rg * kRows + g;
        if (row >= nrows) break;
        const unsigned zz = row / ny;
        const int y = static_cast<int>(row - zz * ny), z = static_cast<int>(zz);
        const bool row_inb = (flag[nx + y] | flag[nx + ny + z]) != 0;
        double2 yz[MaxM];
#pragma unroll
        for (int m = 0; m < MaxM; ++m) {
          if (m < nm) {
            const double2 b = Y[m * ny + y], c = Z[m * nz + z];
            yz[m] = make_double2(b.x * c.x - b.y * c.y, b.x * c.y + b.y * c.x);
          }
        }
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
          const int x = x0 + 64 * k;
          if (x < nx) {
            double ref = 0.0;
#pragma unroll
            for (int m = 0; m < MaxM; ++m) {
              if (m < nm) {
                const double2 a = X[m * nx + x];
                ref += a.x * yz[m].y + a.y * yz[m].x;
              }
            }
            acc.add(static_cast<double>(v[g][k]) - ref, row_inb || flag[x] != 0);
          }
        }
      }
    }
  } else {
    const int64_t total = static_cast<int64_t>(p.nx) * p.ny * p.nz;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < total;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
      const int x = static_cast<int>(i % p.nx);
      const int y = static_cast<int>((i / p.nx) % p.ny);
      const int z = static_cast<int>(i / (static_cast<int64_t>(p.nx) * p.ny));
      double ref = 0.0;
      if (p.nmodes > 0) {
        for (int m = 0; m < p.nmodes; ++m)
          ref += decay(m) * sin(p.kap[m][0] * hx * x + p.kap[m][1] * hy * y + p.kap[m][2] * hz * z + shift(m));
      } else {
        ref = p.ref[i];
      }
      bool inb = in_boundary_layer(x, p.bx, p.s);
      if (p.ndim >= 2) inb |= in_boundary_layer(y, p.by, p.s);
      if (p.ndim == 3) inb |= in_boundary_layer(z, p.bz, p.s);
      acc.add(static_cast<double>(u[p.pe_major ? at(x, y, z) : i]) - ref, inb);
    }
  }
  __shared__ double red[4][kNP];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double v[kNP] = {wave_sum(acc.sab), wave_sum(acc.sqb), wave_sum(acc.sai), wave_sum(acc.sqi),
                   wave_max(acc.mx), wave_sum(acc.bad), 0.0, 0.0};
  if (lane == 0)
    for (int j = 0; j < kNP; ++j) red[wv][j] = v[j];
  __syncthreads();
  if (threadIdx.x == 0) {
    double out[kNP];
    for (int j = 0; j < kNP; ++j) out[j] = red[0][j];
    for (int w = 1; w < static_cast<int>(blockDim.x >> 6); ++w)
      for (int j = 0; j < kNP; ++j) out[j] = j == 4 ? fmax(out[j], red[w][j]) : out[j] + red[w][j];
    for (int j = 0; j < kNP; ++j) p.partial[blockIdx.x * kNP + j] = out[j];
  }
}

// result: [0] mean|e| all, [1] rms all, [2] max, [3] mean|e| B, [4] rms B,
// [5] mean|e| I, [6] rms I, [7] |I_B|, [8] |I_I| ; [9] non-finite count.
// One wave: lane l adds the partials of blocks l, l + 64, ... in order, then a
// fixed butterfly combines the lanes (the same order on every run).
__global__ __launch_bounds__(64) void norms_final_kernel(const double* partial, int nblocks, double nb,
                                                         double ni, double* result) {
  double acc[kNP] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nblocks; b += 64)
    for (int j = 0; j < kNP; ++j)
      acc[j] = j == 4 ? fmax(acc[j], partial[b * kNP + j]) : acc[j] + partial[b * kNP + j];
  for (int j = 0; j < kNP; ++j) acc[j] = j == 4 ? wave_max(acc[j]) : wave_sum(acc[j]);
  if (threadIdx.x != 0) return;
  const double nt = nb + ni;
  result[0] = (acc[0] + acc[2]) / nt;
  result[1] = sqrt((acc[1] + acc[3]) / nt);
  result[2] = acc[4];
  result[3] = nb > 0 ? acc[0] / nb : 0.0;
  result[4] = nb > 0 ? sqrt(acc[1] / nb) : 0.0;
  result[5] = ni > 0 ? acc[2] / ni : 0.0;
  result[6] = ni > 0 ? sqrt(acc[3] / ni) : 0.0;
  result[7] = nb;
  result[8] = ni;
  result[9] = acc[5];
}

}  // namespace

hipError_t norms_static_scratch(int device, double** ptr) {
  // the array's device address, looked up once per device with that device
  // current (the name itself is a host-side stand-in, not a device address)
  static std::once_flag once[kMaxDevices];
  static double* addr[kMaxDevices];
  static hipError_t err[kMaxDevices];
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::call_once(once[device], [device]() {
    void* a = nullptr;
    err[device] = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
    addr[device] = static_cast<double*>(a);
  });
  if (err[device] != hipSuccess) return err[device];
  *ptr = addr[device];
  return hipSuccess;
}

hipError_t launch_norms(const NormParams& p, bool f64, int nblocks, double* result,
                        hipStream_t st) {
  const size_t tb = norm_table_bytes(p);
  const int64_t npts = static_cast<int64_t>(p.nx) * p.ny * p.nz;
  const int use_table = p.nmodes > 0 && tb <= kNormTableBytes && npts < (int64_t{1} << 31) ? 1 : 0;
  const size_t lds = use_table ? tb : 0;
  const bool few = p.nmodes <= 4;
  if (!use_table && f64)
    hipLaunchKernelGGL((norms_partial_kernel<double, 1, false>), dim3(nblocks), dim3(256), 0, st, p);
  else if (!use_table)
    hipLaunchKernelGGL((norms_partial_kernel<float, 1, false>), dim3(nblocks), dim3(256), 0, st, p);
  else if (f64 && few)
    hipLaunchKernelGGL((norms_partial_kernel<double, 4, true>), dim3(nblocks), dim3(256), lds, st, p);
  else if (f64)
    hipLaunchKernelGGL((norms_partial_kernel<double, kMaxModes, true>), dim3(nblocks), dim3(256), lds, st, p);
  else if (few)
    hipLaunchKernelGGL((norms_partial_kernel<float, 4, true>), dim3(nblocks), dim3(256), lds, st, p);
  else
    hipLaunchKernelGGL((norms_partial_kernel<float, kMaxModes, true>), dim3(nblocks), dim3(256), lds, st, p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // counts of I_B and I_I follow from the geometry
  auto layer = [](int n, int b, int s, bool used) -> double {
    if (!used) return 0.0;
    return static_cast<double>(n / b) * 2.0 * s;   // boundary points per axis line
  };
  const double nx = p.nx, ny = p.ny, nz = p.nz;
  // interior count = product over axes of (points not in a boundary layer)
  const double ix = nx - layer(p.nx, p.bx, p.s, true);
  const double iy = ny - layer(p.ny, p.by, p.s, p.ndim >= 2);
  const double iz = nz - layer(p.nz, p.bz, p.s, p.ndim == 3);
  const double ni = ix * iy * iz;
  const double nb = nx * ny * nz - ni;
  hipLaunchKernelGGL(norms_final_kernel, dim3(1), dim3(64), 0, st, p.partial, nblocks, nb, ni,
                     result);
  return hipGetLastError();
}

}  // namespace atfd
