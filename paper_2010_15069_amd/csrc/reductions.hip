// HIP kernels of the split-step solver for gfx950: energy and norm reductions, and the
// workgroup geometry shared by all passes.
#include "fft_device.hpp"
#include "sgpe_internal.hpp"

namespace sgpe {

// -------------------------------------------------------------------------------------------
// Geometry
// -------------------------------------------------------------------------------------------
// Step kernels: lane pairs (two components) x T = n/points lanes per line; a slot of the LDS
// exchange holds both components (16 bytes).
size_t row_lds_bytes(int nx, int rows) { return size_t(rows) * size_t(nx + nx / 16) * 16; }

// column pass: the transforms' exchange slots, then the k_y operator row (one float2 per k_y)
size_t col_lds_bytes(int ny, int cols) { return size_t(cols) * size_t(ny + ny / 16) * 16 + size_t(ny) * 8; }

// complex128 column pass: double2 slots, and the k_y row (one double2 per k_y) where the kernel
// stages it in LDS (16 points per lane, below 4096 points)
size_t col_lds_bytes_c128(int ny, int cols, int points) {
  return size_t(cols) * size_t(ny + ny / 16) * 32 + (points != 16 || ny >= 4096 ? 0 : size_t(ny) * 16);
}

int row_rows_per_block(int nx, int ny, int points, size_t max_lds) {
  int rows = 128 * points / nx;  // 256 threads
  if (rows < 1) rows = 1;
  if (rows > ny) rows = ny;
  while (rows > 1 && row_lds_bytes(nx, rows) > max_lds) rows >>= 1;
  return rows;
}

bool col_cols_supported(int nx, int ny, int cols, int iters, int points, size_t max_lds) {
  if (cols > nx || nx % (cols * iters) != 0) return false;
  if (!schedule_supported(ny, cols, iters, points)) return false;
  return col_lds_bytes(ny, cols) <= max_lds;
}

int col_default_cols(int nx, int ny, int points, size_t max_lds) {
  int c = 128 * points / ny;  // 256 threads
  if (c < 1) c = 1;
  // prefer 64-byte row segments (4 columns) for 16 points per lane, 32-byte ones (2 columns) for
  // the small-grid schedules (measured), while threads and LDS allow it
  int want = points == 16 ? 4 : 2;
  while (want > c && !col_cols_supported(nx, ny, want, 1, points, max_lds)) want >>= 1;
  if (want > c) c = want;
  while (c > 1 && !col_cols_supported(nx, ny, c, 1, points, max_lds)) c >>= 1;
  return c;
}

// Energy kernels (fp64, radix-2 in LDS): one row per row-kernel workgroup (2 nx double2 of LDS);
// up to 4 columns per column-kernel workgroup (2 ny double2 each) as LDS allows.
bool energy_fits(int nx, int ny, size_t max_lds) { return size_t(2) * nx * 16 <= max_lds && size_t(2) * ny * 16 <= max_lds; }

int energy_cols_per_block(int nx, int ny, size_t max_lds) {
  int c = 4;
  while (c > 1 && (size_t(2) * c * ny * 16 > max_lds || nx % c != 0)) c >>= 1;
  return c;
}

int norm_blocks() { return 256; }

// -------------------------------------------------------------------------------------------
// Energy, in fp64 throughout (it is evaluated on demand, not per step).  The k-space quadratic
// form sum_k psi^(k)^+ H_K(k) psi^(k) of the energy splits, by Parseval's theorem along one axis at
// a time, into 1-D pieces of the state as it is, so no 2-D transform is formed:
//   * the k_x terms (k_x^2 / 2 on both components, k_l k_x sigma_z): for every row, the x-DFT
//     u~(k_x) of the row, sum over k_x; over the whole grid the sum of |u^|^2 f(k_x) is ny times the
//     sum over rows of |u~|^2 f(k_x);
//   * the k_y term (k_y^2 / 2): the same with the y-DFT of every column, times nx;
//   * the uniform Raman term Omega Re(u^* d^) of H_K: N times its real-space sum, so it joins the
//     spatial Raman term Omega(r) Re(u* d) of the real-space energy.
// Row kernel: the real-space terms, the norm and the row's k_x terms (one row per workgroup); column
// kernel: the k_y terms of up to 4 columns per workgroup.  The DFTs are in-place radix-2 transforms
// in LDS: input stored at bit-reversed positions, log2 N butterfly stages, roots exp(-2 pi i j / N)
// from fp64 host tables.  Exact to fp64 rounding, so the energy of a complex64 state carries no
// transform error of its own.  The partials are scaled so that the host's combination reads
// E = (w / N ek + w er) / norm + w ei norm0 / norm^2 (w = dx dy, N = nx ny), as for a 2-D sum.
// -------------------------------------------------------------------------------------------
__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// `count` independent length-N transforms stored one after another in `buf` (each already in
// bit-reversed order); all threads of the workgroup take part.
__device__ __forceinline__ void lds_fft64(double2* buf, int n, int log2n, int count, const double2* __restrict__ w) {
  const int half_total = count * (n >> 1);
  for (int s = 1; s <= log2n; ++s) {
    const int half = 1 << (s - 1);
    const int tw_step = n >> s;  // root index stride: exp(-2 pi i k / 2^s) = w[k n / 2^s]
    __syncthreads();
    for (int b = threadIdx.x; b < half_total; b += blockDim.x) {
      const int tr = b / (n >> 1);
      const int q = b - tr * (n >> 1);
      const int k = q & (half - 1);
      const int i0 = tr * n + ((q >> (s - 1)) << s) + k;
      const double2 a0 = buf[i0];
      const double2 a1 = zmul(buf[i0 + half], w[k * tw_step]);
      buf[i0] = make_double2(a0.x + a1.x, a0.y + a1.y);
      buf[i0 + half] = make_double2(a0.x - a1.x, a0.y - a1.y);
    }
  }
  __syncthreads();
}

__device__ __forceinline__ int bitrev(int j, int log2n) { return static_cast<int>(__brev(static_cast<unsigned>(j)) >> (32 - log2n)); }

// Point i of the state as four doubles {re_up, im_up, re_dn, im_dn}.
__device__ __forceinline__ double4 state_point(const EnergyArgs& a, size_t i) {
  if (a.psi64) return a.psi64[i];
  const float4 v = a.psi[i];
  return make_double4(v.x, v.y, v.z, v.w);
}

__global__ void __launch_bounds__(256) energy_row_kernel(EnergyArgs a) {
  extern __shared__ double2 elds[];
  __shared__ double red[64];
  const int n = a.nx, log2n = __builtin_ctz(a.nx);
  const int row = blockIdx.x;
  const double y = a.ymin + a.dy * row;
  const double om_row = a.om_y ? a.om_y[row] : 0.0;
  double er = 0.0, ei = 0.0, nr = 0.0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const double4 v = state_point(a, size_t(row) * n + j);
    const double ur = v.x, ui = v.y, dr = v.z, di = v.w;
    const double x = a.xmin + a.dx * j;
    const double V = a.wx2h * x * x + a.wy2h * y * y;
    const double nu = ur * ur + ui * ui, nd = dr * dr + di * di;
    // spatial Raman coupling Omega(r) and the uniform one Omega (its k-space sum, by Parseval)
    const double om = (a.om_x ? a.om_x[j] + om_row : 0.0) + a.omega;
    er += V * (nu + nd) + 0.5 * a.delta * (nu - nd) + om * (ur * dr + ui * di);
    ei += 0.5 * a.g_uu * nu * nu + 0.5 * a.g_dd * nd * nd + a.g_ud * nu * nd;
    nr += nu + nd;
    const int r = bitrev(j, log2n);
    elds[r] = make_double2(ur, ui);
    elds[n + r] = make_double2(dr, di);
  }
  lds_fft64(elds, n, log2n, 2, a.twx);
  double ex = 0.0;   // this row's k_x terms
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const double kx = (j < n / 2 ? j : j - n) * a.dkx;
    const double2 u = elds[j], d = elds[n + j];
    const double pu = u.x * u.x + u.y * u.y, pd = d.x * d.x + d.y * d.y;
    ex += 0.5 * kx * kx * (pu + pd) + a.k_l * kx * (pu - pd);
  }
  const double se = block_sum(er, red);
  const double sx = block_sum(ex, red);
  const double si = block_sum(ei, red);
  const double sn = block_sum(nr, red);
  if (threadIdx.x == 0) {
    // w / N * (ny * sx) = w * sx / nx: the k_x terms join the real-space linear ones
    a.row_partials[kEnergyRowParts * blockIdx.x] = se + sx / double(n);
    a.row_partials[kEnergyRowParts * blockIdx.x + 1] = si;
    a.row_partials[kEnergyRowParts * blockIdx.x + 2] = sn;
  }
}

__global__ void __launch_bounds__(256) energy_col_kernel(EnergyArgs a) {
  extern __shared__ double2 elds[];
  __shared__ double red[64];
  const int n = a.ny, log2n = __builtin_ctz(a.ny);
  const int C = a.cols;
  const int x0 = blockIdx.x * C;
  // columns x0 .. x0 + C - 1: transform 2c (up) and 2c + 1 (down) of column c
  for (int i = threadIdx.x; i < C * n; i += blockDim.x) {
    const int c = i % C, iy = i / C;
    const double4 v = state_point(a, size_t(iy) * a.nx + x0 + c);
    const int r = bitrev(iy, log2n);
    elds[(2 * c) * n + r] = make_double2(v.x, v.y);
    elds[(2 * c + 1) * n + r] = make_double2(v.z, v.w);
  }
  lds_fft64(elds, n, log2n, 2 * C, a.twy);
  double acc = 0.0;
  for (int i = threadIdx.x; i < C * n; i += blockDim.x) {
    const int c = i / n, iy = i - c * n;
    const double ky = (iy < n / 2 ? iy : iy - n) * a.dky;
    const double2 u = elds[(2 * c) * n + iy], d = elds[(2 * c + 1) * n + iy];
    acc += 0.5 * ky * ky * (u.x * u.x + u.y * u.y + d.x * d.x + d.y * d.y);
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) a.col_partials[blockIdx.x] = double(a.nx) * s;   // nx times the columns' sum
}

// -------------------------------------------------------------------------------------------
// Norm: sum |psi|^2 with a fixed grid (deterministic), fp64.
// -------------------------------------------------------------------------------------------
template <class Q>
__global__ void __launch_bounds__(256) norm_kernel(const Q* __restrict__ psi, long long n,
                                                   double* __restrict__ partials) {
  __shared__ double red[64];
  double acc = 0.0;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x) {
    const Q w = psi[i];
    const double ur = w.x, ui = w.y, dr = w.z, di = w.w;
    acc += ur * ur + ui * ui + dr * dr + di * di;
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// One wave combines the energy kernels' partials on the device: each kind summed in a fixed order
// (lane-strided, then a fixed butterfly), then the energy per particle of the state rescaled to
// norm0, E = (w / N ek + w er) / norm + w ei norm0 / norm^2 with norm = w nr.
__global__ void __launch_bounds__(64) energy_finish_kernel(const double* __restrict__ row_parts, int nrows,
                                                           const double* __restrict__ col_parts, int ncols, double w,
                                                           double inv_npts, double norm0, double* __restrict__ out) {
  const int lane = threadIdx.x;
  double er = 0.0, ei = 0.0, nr = 0.0, ek = 0.0;
  for (int b = lane; b < nrows; b += 64) {
    er += row_parts[kEnergyRowParts * b];
    ei += row_parts[kEnergyRowParts * b + 1];
    nr += row_parts[kEnergyRowParts * b + 2];
  }
  for (int b = lane; b < ncols; b += 64) ek += col_parts[b];
  er = wave_sum(er);
  ei = wave_sum(ei);
  nr = wave_sum(nr);
  ek = wave_sum(ek);
  if (lane == 0) {
    const double nrm = w * nr;
    out[0] = (w * inv_npts * ek + w * er) / nrm + w * ei * norm0 / (nrm * nrm);
  }
}

hipError_t launch_energy_finish(const EnergyArgs& a, double norm0, double* out, hipStream_t s) {
  const double w = a.dx * a.dy;
  const double inv_npts = 1.0 / (double(a.nx) * double(a.ny));
  hipLaunchKernelGGL(energy_finish_kernel, dim3(1), dim3(64), 0, s, a.row_partials, a.ny, a.col_partials,
                     a.nx / a.cols, w, inv_npts, norm0, out);
  return hipGetLastError();
}

hipError_t launch_energy(const EnergyArgs& a, hipStream_t s) {
  const size_t row_lds = size_t(2) * a.nx * sizeof(double2);
  const size_t col_lds = size_t(2) * a.cols * a.ny * sizeof(double2);
  hipLaunchKernelGGL(energy_row_kernel, dim3(a.ny), dim3(256), row_lds, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(energy_col_kernel, dim3(a.nx / a.cols), dim3(256), col_lds, s, a);
  return hipGetLastError();
}

hipError_t launch_norm(const float4* psi, long long npts, double* partials, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(norm_kernel<float4>, dim3(nblocks), dim3(256), 0, s, psi, npts, partials);
  return hipGetLastError();
}

hipError_t launch_norm(const double4* psi, long long npts, double* partials, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(norm_kernel<double4>, dim3(nblocks), dim3(256), 0, s, psi, npts, partials);
  return hipGetLastError();
}

}  // namespace sgpe
