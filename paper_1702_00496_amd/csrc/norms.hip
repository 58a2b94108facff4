// Error norms of a field against the decaying advected Fourier series (Sec. 5.1
// eq. ana_sol) or against a double reference field, split over the boundary
// set I_B (points within s of a PE face) and the interior set I_I (Sec. 4
// space averages). Accumulation in double: per-thread sums, wave64 butterfly
// shuffles, one partial per workgroup, then a single-workgroup pass that adds
// the partials in index order, so the result does not depend on scheduling.

#include "atfd_internal.hpp"

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

template <typename Real>
__global__ __launch_bounds__(256) void norms_partial_kernel(NormParams p) {
  const int64_t total = static_cast<int64_t>(p.nx) * p.ny * p.nz;
  const Real* u = static_cast<const Real*>(p.u);
  const double t = static_cast<double>(p.counter[0]) * p.dt;
  double amp_t[kMaxModes], shift[kMaxModes], kx[kMaxModes], ky[kMaxModes], kz[kMaxModes];
  const double hx = p.length / p.nx, hy = p.length / p.ny, hz = p.length / p.nz;
  for (int m = 0; m < p.nmodes; ++m) {
    const double k2 = double(p.kap[m][0]) * p.kap[m][0] + double(p.kap[m][1]) * p.kap[m][1] +
                      double(p.kap[m][2]) * p.kap[m][2];
    amp_t[m] = p.amp[m] * exp(-p.alpha * k2 * t);
    shift[m] = p.phase[m] - t * (p.kap[m][0] * p.vel[0] + p.kap[m][1] * p.vel[1] +
                                 p.kap[m][2] * p.vel[2]);
    kx[m] = p.kap[m][0] * hx;
    ky[m] = p.kap[m][1] * hy;
    kz[m] = p.kap[m][2] * hz;
  }
  double sab = 0, sqb = 0, sai = 0, sqi = 0, mx = 0, bad = 0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < total;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int x = static_cast<int>(i % p.nx);
    const int y = static_cast<int>((i / p.nx) % p.ny);
    const int z = static_cast<int>(i / (static_cast<int64_t>(p.nx) * p.ny));
    double ref;
    if (p.nmodes > 0) {
      ref = 0.0;
      for (int m = 0; m < p.nmodes; ++m)
        ref += amp_t[m] * sin(kx[m] * x + ky[m] * y + kz[m] * z + shift[m]);
    } else {
      ref = p.ref[i];
    }
    const double e = static_cast<double>(u[i]) - ref;
    if (!isfinite(e)) { bad += 1.0; continue; }
    bool inb = false;
    const int lx = x % p.bx, ly = y % p.by, lz = z % p.bz;
    inb |= lx < p.s || lx >= p.bx - p.s;
    if (p.ndim >= 2) inb |= ly < p.s || ly >= p.by - p.s;
    if (p.ndim == 3) inb |= lz < p.s || lz >= p.bz - p.s;
    const double ae = fabs(e);
    if (inb) { sab += ae; sqb += e * e; } else { sai += ae; sqi += e * e; }
    mx = fmax(mx, ae);
  }
  __shared__ double red[4][kNP];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double v[kNP] = {wave_sum(sab), wave_sum(sqb), wave_sum(sai), wave_sum(sqi), wave_max(mx),
                   wave_sum(bad), 0.0, 0.0};
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
// [5] mean|e| I, [6] rms I, [7] |I_B|, [8] |I_I| ; [9] non-finite count
__global__ void norms_final_kernel(const double* partial, int nblocks, double nb, double ni,
                                   double* result) {
  if (threadIdx.x != 0) return;
  double acc[kNP] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int b = 0; b < nblocks; ++b)
    for (int j = 0; j < kNP; ++j)
      acc[j] = j == 4 ? fmax(acc[j], partial[b * kNP + j]) : acc[j] + partial[b * kNP + j];
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

hipError_t launch_norms(const NormParams& p, bool f64, int nblocks, double* result,
                        hipStream_t st) {
  if (f64)
    hipLaunchKernelGGL(norms_partial_kernel<double>, dim3(nblocks), dim3(256), 0, st, p);
  else
    hipLaunchKernelGGL(norms_partial_kernel<float>, dim3(nblocks), dim3(256), 0, st, p);
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
