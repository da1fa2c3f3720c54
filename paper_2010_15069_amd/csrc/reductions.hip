// HIP kernels of the split-step solver for gfx950: energy and norm reductions, and the
// workgroup geometry shared by all passes.
#include <algorithm>

#include "col_body.hpp"
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

// Energy kernels (fp64, register-resident transforms, 16 points per lane up to the line length):
// T = N / 16 lanes per component of a line, two components per lane pair.  Row kernel: 128 / T rows
// per workgroup (at least one; 512 threads at 4096 points).  Column kernel: 128 / T columns per
// workgroup (at least one), fewer where the grid has fewer.  Both interleave their transforms in
// LDS slot by slot, N + N/16 double2 slots each.
int energy_points(int n) { return n >= 16 ? 16 : n; }

size_t energy_lds_bytes(int n, int lines) { return size_t(2) * lines * size_t(n + n / 16) * 16; }

int energy_rows_per_block(int nx, int ny) {
  const int t = nx / energy_points(nx);
  return std::max(1, std::min(ny, 128 / t));
}

int energy_cols_per_block(int nx, int ny, size_t max_lds) {
  const int t = ny / energy_points(ny);
  int c = std::max(1, std::min(nx, 128 / t));
  while (c > 1 && energy_lds_bytes(ny, c) > max_lds) c >>= 1;
  return c;
}

bool energy_fits(int nx, int ny, size_t max_lds) {
  return energy_lds_bytes(nx, energy_rows_per_block(nx, ny)) <= max_lds &&
         energy_lds_bytes(ny, energy_cols_per_block(nx, ny, max_lds)) <= max_lds;
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
// Row kernel: the real-space terms, the norm and the rows' k_x terms; column kernel: the columns'
// k_y terms.  The DFTs are the step kernels' register-resident forward transform (fwd_pass: radix-16
// stages exchanged through LDS, natural order in and out) instantiated in fp64 with the roots
// rounded once to fp64, on the state widened to fp64 as it is loaded, so the energy of a complex64
// state carries no transform error of its own.  Each lane holds one component of one line.  The
// partials are scaled so that the
// host's combination reads E = (w / N ek + w er) / norm + w ei norm0 / norm^2 (w = dx dy,
// N = nx ny), as for a 2-D sum.
// -------------------------------------------------------------------------------------------
extern __shared__ __align__(16) unsigned char energy_lds[];

// The lane's component of state point i (Q: float4 for a complex64 state, double4 for complex128),
// widened to fp64.
template <class Q>
__device__ __forceinline__ double2 energy_load(const EnergyArgs& a, size_t i, int comp) {
  if constexpr (sizeof(Q) == sizeof(double4)) {
    return reinterpret_cast<const double2*>(a.psi64)[2 * i + comp];
  } else {
    const float2 v = reinterpret_cast<const float2*>(a.psi)[2 * i + comp];
    return make_double2(v.x, v.y);
  }
}

__device__ __forceinline__ int energy_freq(int j, int n) { return j < n / 2 ? j : j - n; }

// Point i of the state as four doubles {re_up, im_up, re_dn, im_dn}.
template <class Q>
__device__ __forceinline__ double4 energy_point(const EnergyArgs& a, size_t i) {
  if constexpr (sizeof(Q) == sizeof(double4)) {
    return a.psi64[i];
  } else {
    const float4 v = a.psi[i];
    return make_double4(v.x, v.y, v.z, v.w);
  }
}

template <int N, class Q>
__global__ void __launch_bounds__(512) energy_row_kernel(EnergyArgs a) {
  constexpr int P = N >= 16 ? 16 : N;
  constexpr int T = N / P;
  __shared__ double red[64];
  const int tid = threadIdx.x, comp = tid & 1, pair = tid >> 1;
  const int t = pair & (T - 1), r = pair / T;
  const int row = blockIdx.x * a.rows + r;
  const size_t row0 = size_t(row) * N;
  // The real-space terms and the norm, point by point with both components in one load (a loop of
  // few registers of its own; the transform's loads below then find the row in the L2).
  const double y = a.ymin + a.dy * row;
  const double om_row = a.om_y ? a.om_y[row] : 0.0;
  double er = 0.0, ei = 0.0, nr = 0.0;
#pragma unroll 2
  for (int j = tid & (2 * T - 1); j < N; j += 2 * T) {
    const double4 q = energy_point<Q>(a, row0 + j);
    const double x = a.xmin + a.dx * j;
    const double V = a.wx2h * x * x + a.wy2h * y * y;
    const double nu = q.x * q.x + q.y * q.y, nd = q.z * q.z + q.w * q.w;
    // spatial Raman coupling Omega(r) and the uniform one Omega (its k-space sum, by Parseval)
    const double om = (a.om_x ? a.om_x[j] + om_row : 0.0) + a.omega;
    er += V * (nu + nd) + 0.5 * a.delta * (nu - nd) + om * (q.x * q.z + q.y * q.w);
    ei += 0.5 * a.g_uu * nu * nu + 0.5 * a.g_dd * nd * nd + a.g_ud * nu * nd;
    nr += nu + nd;
  }
  // keep the transform's loads (and their registers) after the loop above
  asm volatile("" ::: "memory");
  double2 v[P];
#pragma unroll
  for (int m = 0; m < P; ++m) v[m] = energy_load<Q>(a, row0 + t + T * m, comp);
  TwPlain<N, P, double> tr;
  load_twiddles<N>(tr, t, a.twx);
  const LdsView<double2> lds{reinterpret_cast<double2*>(energy_lds) + 2 * r + comp, 1 + __builtin_ctz(a.rows)};
  fwd_pass<N>(v, lds, t, tr);
  const double kl = comp == 0 ? a.k_l : -a.k_l;
  double ex = 0.0;   // the rows' k_x terms
#pragma unroll
  for (int m = 0; m < P; ++m) {
    const double kx = energy_freq(t + T * m, N) * a.dkx;
    ex += (0.5 * kx * kx + kl * kx) * (v[m].x * v[m].x + v[m].y * v[m].y);
  }
  const double se = block_sum(er, red);
  const double sx = block_sum(ex, red);
  const double si = block_sum(ei, red);
  const double sn = block_sum(nr, red);
  if (tid == 0) {
    // w / N * (ny * sx) = w * sx / nx: the k_x terms join the real-space linear ones
    a.row_partials[kEnergyRowParts * blockIdx.x] = se + sx / double(N);
    a.row_partials[kEnergyRowParts * blockIdx.x + 1] = si;
    a.row_partials[kEnergyRowParts * blockIdx.x + 2] = sn;
  }
}

template <int N, class Q>
__global__ void __launch_bounds__(512) energy_col_kernel(EnergyArgs a) {
  constexpr int P = N >= 16 ? 16 : N;
  constexpr int T = N / P;
  __shared__ double red[64];
  const int C = a.cols;
  const int tid = threadIdx.x, comp = tid & 1, pair = tid >> 1;
  const int cc = pair & (C - 1), t = pair / C;
  const int x = col_group(blockIdx.x, gridDim.x) * C + cc;
  double2 v[P];
#pragma unroll
  for (int m = 0; m < P; ++m) v[m] = energy_load<Q>(a, size_t(t + T * m) * a.nx + x, comp);
  TwPlain<N, P, double> tr;
  load_twiddles<N>(tr, t, a.twy);
  const LdsView<double2> lds{reinterpret_cast<double2*>(energy_lds) + 2 * cc + comp, 1 + __builtin_ctz(C)};
  fwd_pass<N>(v, lds, t, tr);
  double acc = 0.0;
#pragma unroll
  for (int m = 0; m < P; ++m) {
    const double ky = energy_freq(t + T * m, N) * a.dky;
    acc += 0.5 * ky * ky * (v[m].x * v[m].x + v[m].y * v[m].y);
  }
  const double s = block_sum(acc, red);
  if (tid == 0) a.col_partials[blockIdx.x] = double(a.nx) * s;   // nx times the columns' sum
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
  hipLaunchKernelGGL(energy_finish_kernel, dim3(1), dim3(64), 0, s, a.row_partials, a.ny / a.rows, a.col_partials,
                     a.nx / a.cols, w, inv_npts, norm0, out);
  return hipGetLastError();
}

template <int N>
hipError_t launch_energy_row(const EnergyArgs& a, hipStream_t s) {
  constexpr int T = N / (N >= 16 ? 16 : N);
  const dim3 grid(a.ny / a.rows), block(2 * T * a.rows);
  const size_t lds = energy_lds_bytes(N, a.rows);
  if (a.psi64) hipLaunchKernelGGL((energy_row_kernel<N, double4>), grid, block, lds, s, a);
  else hipLaunchKernelGGL((energy_row_kernel<N, float4>), grid, block, lds, s, a);
  return hipGetLastError();
}

template <int N>
hipError_t launch_energy_col(const EnergyArgs& a, hipStream_t s) {
  constexpr int T = N / (N >= 16 ? 16 : N);
  const dim3 grid(a.nx / a.cols), block(2 * T * a.cols);
  const size_t lds = energy_lds_bytes(N, a.cols);
  if (a.psi64) hipLaunchKernelGGL((energy_col_kernel<N, double4>), grid, block, lds, s, a);
  else hipLaunchKernelGGL((energy_col_kernel<N, float4>), grid, block, lds, s, a);
  return hipGetLastError();
}

hipError_t launch_energy(const EnergyArgs& a, hipStream_t s) {
  hipError_t e = hipErrorInvalidValue;
  switch (a.nx) {
    case 16: e = launch_energy_row<16>(a, s); break;
    case 32: e = launch_energy_row<32>(a, s); break;
    case 64: e = launch_energy_row<64>(a, s); break;
    case 128: e = launch_energy_row<128>(a, s); break;
    case 256: e = launch_energy_row<256>(a, s); break;
    case 512: e = launch_energy_row<512>(a, s); break;
    case 1024: e = launch_energy_row<1024>(a, s); break;
    case 2048: e = launch_energy_row<2048>(a, s); break;
    case 4096: e = launch_energy_row<4096>(a, s); break;
    default: break;
  }
  if (e != hipSuccess) return e;
  switch (a.ny) {
    case 16: return launch_energy_col<16>(a, s);
    case 32: return launch_energy_col<32>(a, s);
    case 64: return launch_energy_col<64>(a, s);
    case 128: return launch_energy_col<128>(a, s);
    case 256: return launch_energy_col<256>(a, s);
    case 512: return launch_energy_col<512>(a, s);
    case 1024: return launch_energy_col<1024>(a, s);
    case 2048: return launch_energy_col<2048>(a, s);
    case 4096: return launch_energy_col<4096>(a, s);
    default: return hipErrorInvalidValue;
  }
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
