// HIP kernels of the solver's observables and state updates beyond the step: the Gaussian-noise
// annealing update, the moments behind the phase-separation parameter, the population inside a
// disc, and the circulation (phase winding) of each component along a circle (Sec. 6).
// All sums are fp64 in a fixed order (deterministic).
#include "fft_device.hpp"
#include "sgpe_internal.hpp"

namespace sgpe {

// The kernels below take either state type: float4 (complex64) or double4 (complex128).
__device__ __forceinline__ float4 fma4(float a, float4 z, float4 w) {
  return make_float4(fmaf(a, z.x, w.x), fmaf(a, z.y, w.y), fmaf(a, z.z, w.z), fmaf(a, z.w, w.w));
}
__device__ __forceinline__ double4 fma4(double a, double4 z, double4 w) {
  return make_double4(fma(a, z.x, w.x), fma(a, z.y, w.y), fma(a, z.z, w.z), fma(a, z.w, w.w));
}

// psi <- psi + amp xi at every point, both components.
template <class Q, class T>
__global__ void __launch_bounds__(256) add_noise_kernel(Q* __restrict__ psi, const Q* __restrict__ xi, T amp,
                                                        long long n) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x) psi[i] = fma4(amp, xi[i], psi[i]);
}

// Per block: sum n_u n_d, sum n_u^2, sum n_d^2 (densities formed in fp64).
template <class Q>
__global__ void __launch_bounds__(256) moments_kernel(const Q* __restrict__ psi, long long n,
                                                      double* __restrict__ partials) {
  __shared__ double red[64];
  double sud = 0.0, suu = 0.0, sdd = 0.0;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x) {
    const Q w = psi[i];
    const double ur = w.x, ui = w.y, dr = w.z, di = w.w;
    const double nu = ur * ur + ui * ui, nd = dr * dr + di * di;
    sud += nu * nd;
    suu += nu * nu;
    sdd += nd * nd;
  }
  sud = block_sum(sud, red);
  suu = block_sum(suu, red);
  sdd = block_sum(sdd, red);
  if (threadIdx.x == 0) {
    partials[kMomentParts * blockIdx.x] = sud;
    partials[kMomentParts * blockIdx.x + 1] = suu;
    partials[kMomentParts * blockIdx.x + 2] = sdd;
  }
}

// Per block: sum of n_u + n_d over the grid points (x0 + j dx, y0 + i dy) with x^2 + y^2 <= r2.
template <class Q>
__global__ void __launch_bounds__(256) disk_population_kernel(const Q* __restrict__ psi, int nx, long long n,
                                                              double x0, double dx, double y0, double dy,
                                                              double r2, double* __restrict__ partials) {
  __shared__ double red[64];
  double acc = 0.0;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x) {
    const long long row = i / nx;
    const int j = static_cast<int>(i - row * nx);
    const double x = x0 + dx * j, y = y0 + dy * static_cast<double>(row);
    if (x * x + y * y <= r2) {
      const Q w = psi[i];
      const double ur = w.x, ui = w.y, dr = w.z, di = w.w;
      acc += ur * ur + ui * ui + dr * dr + di * di;
    }
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// Grid index nearest to sample k of the circle: theta_k = 2 pi k / m, (R cos, R sin) rounded to
// the nearest grid point, periodic in the box.
__device__ __forceinline__ long long circle_point(int k, int m, double radius, int nx, int ny, double xmax,
                                                  double ymax) {
  const double th = 2.0 * M_PI * static_cast<double>(k) / static_cast<double>(m);
  double sn, cs;
  sincos(th, &sn, &cs);
  const double dx = 2.0 * xmax / nx, dy = 2.0 * ymax / ny;
  long long j = llrint((radius * cs + xmax) / dx);
  long long i = llrint((radius * sn + ymax) / dy);
  j = ((j % nx) + nx) % nx;
  i = ((i % ny) + ny) % ny;
  return i * nx + j;
}

// Phase increment arg(b conj(a)) in (-pi, pi], fp64.
__device__ __forceinline__ double phase_step(double ar, double ai, double br, double bi) {
  return atan2(bi * ar - br * ai, br * ar + bi * ai);
}

template <class Q>
__global__ void __launch_bounds__(256) winding_kernel(const Q* __restrict__ psi, int nx, int ny, double xmax,
                                                      double ymax, double radius, int m, double* __restrict__ out) {
  __shared__ double red[64];
  double su = 0.0, sd = 0.0;
  for (int k = threadIdx.x; k < m; k += 256) {
    const Q a = psi[circle_point(k, m, radius, nx, ny, xmax, ymax)];
    const Q b = psi[circle_point(k + 1 == m ? 0 : k + 1, m, radius, nx, ny, xmax, ymax)];
    su += phase_step(a.x, a.y, b.x, b.y);
    sd += phase_step(a.z, a.w, b.z, b.w);
  }
  su = block_sum(su, red);
  sd = block_sum(sd, red);
  if (threadIdx.x == 0) {
    out[0] = su / (2.0 * M_PI);
    out[1] = sd / (2.0 * M_PI);
  }
}

template <class Q, class T>
static hipError_t add_noise_t(Q* psi, const Q* xi, T amp, long long npts, hipStream_t s) {
  hipLaunchKernelGGL((add_noise_kernel<Q, T>), dim3(norm_blocks()), dim3(256), 0, s, psi, xi, amp, npts);
  return hipGetLastError();
}
hipError_t launch_add_noise(float4* psi, const float4* xi, float amp, long long npts, hipStream_t s) {
  return add_noise_t(psi, xi, amp, npts, s);
}
hipError_t launch_add_noise(double4* psi, const double4* xi, double amp, long long npts, hipStream_t s) {
  return add_noise_t(psi, xi, amp, npts, s);
}

template <class Q>
static hipError_t moments_t(const Q* psi, long long npts, double* partials, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(moments_kernel<Q>, dim3(nblocks), dim3(256), 0, s, psi, npts, partials);
  return hipGetLastError();
}
hipError_t launch_moments(const float4* psi, long long npts, double* partials, int nblocks, hipStream_t s) {
  return moments_t(psi, npts, partials, nblocks, s);
}
hipError_t launch_moments(const double4* psi, long long npts, double* partials, int nblocks, hipStream_t s) {
  return moments_t(psi, npts, partials, nblocks, s);
}

template <class Q>
static hipError_t disk_t(const Q* psi, int nx, int ny, double x0, double dx, double y0, double dy, double r2,
                         double* partials, int nblocks, hipStream_t s) {
  const long long n = static_cast<long long>(nx) * ny;
  hipLaunchKernelGGL(disk_population_kernel<Q>, dim3(nblocks), dim3(256), 0, s, psi, nx, n, x0, dx, y0, dy, r2,
                     partials);
  return hipGetLastError();
}
hipError_t launch_disk_population(const float4* psi, int nx, int ny, double x0, double dx, double y0, double dy,
                                  double r2, double* partials, int nblocks, hipStream_t s) {
  return disk_t(psi, nx, ny, x0, dx, y0, dy, r2, partials, nblocks, s);
}
hipError_t launch_disk_population(const double4* psi, int nx, int ny, double x0, double dx, double y0, double dy,
                                  double r2, double* partials, int nblocks, hipStream_t s) {
  return disk_t(psi, nx, ny, x0, dx, y0, dy, r2, partials, nblocks, s);
}

template <class Q>
static hipError_t winding_t(const Q* psi, int nx, int ny, double xmax, double ymax, double radius, int m,
                            double* out, hipStream_t s) {
  hipLaunchKernelGGL(winding_kernel<Q>, dim3(1), dim3(256), 0, s, psi, nx, ny, xmax, ymax, radius, m, out);
  return hipGetLastError();
}
hipError_t launch_winding(const float4* psi, int nx, int ny, double xmax, double ymax, double radius, int m,
                          double* out, hipStream_t s) {
  return winding_t(psi, nx, ny, xmax, ymax, radius, m, out, s);
}
hipError_t launch_winding(const double4* psi, int nx, int ny, double xmax, double ymax, double radius, int m,
                          double* out, hipStream_t s) {
  return winding_t(psi, nx, ny, xmax, ymax, radius, m, out, s);
}

}  // namespace sgpe
