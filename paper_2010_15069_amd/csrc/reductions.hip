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

// Energy kernels (fp64, register-resident transforms): 8 points per lane below 1024 points, 16
// from there; T = N / points lanes per component of a line, two components per lane pair.  Lines per
// workgroup: up to 128 / T (a workgroup of at most 256 threads, 512 at 4096 points), but no more
// than keeps ~256 workgroups on the grid (small grids are latency-bound: more workgroups, each
// shorter).  Both kernels interleave their transforms in LDS slot by slot, N + N/16 double2 slots
// each.
__host__ __device__ constexpr int energy_points(int n) { return n >= 1024 ? 16 : 8; }

size_t energy_lds_bytes(int n, int lines) { return size_t(2) * lines * size_t(n + n / 16) * 16; }

static int energy_lines_per_block(int n, int count) {
  const int t = n / energy_points(n);
  return std::max(1, std::min(128 / t, count / 256));
}

int energy_rows_per_block(int nx, int ny) { return energy_lines_per_block(nx, ny); }

int energy_cols_per_block(int nx, int ny, size_t max_lds) {
  int c = energy_lines_per_block(ny, nx);
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
// k_y terms.  The DFTs are the step kernels' register-resident forward transform (fwd_pass: radix-P
// stages exchanged through LDS, natural order in and out) instantiated in fp64 with the roots
// rounded once to fp64, on the state widened to fp64 as it is loaded, so the energy of a complex64
// state carries no transform error of its own.  Each lane holds one component of one line.  The
// partials are scaled so that their combination reads E = (w / N ek + w er) / norm
// + w ei norm0 / norm^2 (w = dx dy, N = nx ny), as for a 2-D sum.
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

// Rows block*rows .. block*rows + rows - 1 of the state a describes.
template <int N, class Q>
__device__ __forceinline__ void energy_row_body(const EnergyArgs& a, int block) {
  constexpr int P = energy_points(N);
  constexpr int T = N / P;
  __shared__ double red[64];
  const int tid = threadIdx.x, comp = tid & 1, pair = tid >> 1;
  const int t = pair & (T - 1), r = pair / T;
  const int row = block * a.rows + r;
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
    a.row_partials[kEnergyRowParts * block] = se + sx / double(N);
    a.row_partials[kEnergyRowParts * block + 1] = si;
    a.row_partials[kEnergyRowParts * block + 2] = sn;
  }
}

template <int N, class Q>
__global__ void __launch_bounds__(512) energy_row_kernel(EnergyArgs a) {
  energy_row_body<N, Q>(a, blockIdx.x);
}

// Batched: grid y = the members of a batch class, each with its own arguments.
template <int N, class Q>
__global__ void __launch_bounds__(512) energy_row_kernel_batch(const EnergyArgs* __restrict__ tab) {
  const EnergyArgs a = tab[blockIdx.y];
  energy_row_body<N, Q>(a, blockIdx.x);
}

// Columns of column block `block` (of a.nx / a.cols; the blocks spread over the XCDs as the column
// pass spreads its tiles).
template <int N, class Q>
__device__ __forceinline__ void energy_col_body(const EnergyArgs& a, int block) {
  constexpr int P = energy_points(N);
  constexpr int T = N / P;
  __shared__ double red[64];
  const int C = a.cols;
  const int tid = threadIdx.x, comp = tid & 1, pair = tid >> 1;
  const int cc = pair & (C - 1), t = pair / C;
  const int x = col_group(block, a.nx / C) * C + cc;
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
  if (tid == 0) a.col_partials[block] = double(a.nx) * s;   // nx times the columns' sum
}

template <int N, class Q>
__global__ void __launch_bounds__(512) energy_col_kernel(EnergyArgs a) {
  energy_col_body<N, Q>(a, blockIdx.x);
}

template <int N, class Q>
__global__ void __launch_bounds__(512) energy_col_kernel_batch(const EnergyArgs* __restrict__ tab) {
  const EnergyArgs a = tab[blockIdx.y];
  energy_col_body<N, Q>(a, blockIdx.x);
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

// One workgroup combines the energy kernels' partials on the device: each kind summed in a fixed
// order (thread-strided, then block_sum's fixed tree), then the energy per particle of the state
// rescaled to norm0, E = (w / N ek + w er) / norm + w ei norm0 / norm^2 with norm = w nr.
__device__ __forceinline__ void energy_finish_body(const EnergyArgs& a, double* out) {
  __shared__ double red[64];
  const int nrows = a.ny / a.rows, ncols = a.nx / a.cols;
  double er = 0.0, ei = 0.0, nr = 0.0, ek = 0.0;
#pragma unroll 4
  for (int b = threadIdx.x; b < nrows; b += blockDim.x) {
    er += a.row_partials[kEnergyRowParts * b];
    ei += a.row_partials[kEnergyRowParts * b + 1];
    nr += a.row_partials[kEnergyRowParts * b + 2];
  }
#pragma unroll 4
  for (int b = threadIdx.x; b < ncols; b += blockDim.x) ek += a.col_partials[b];
  er = block_sum(er, red);
  ei = block_sum(ei, red);
  nr = block_sum(nr, red);
  ek = block_sum(ek, red);
  if (threadIdx.x == 0) {
    const double w = a.dx * a.dy;
    const double nrm = w * nr;
    out[0] = (w / (double(a.nx) * double(a.ny)) * ek + w * er) / nrm + w * ei * a.norm0 / (nrm * nrm);
  }
}

__global__ void __launch_bounds__(256) energy_finish_kernel(EnergyArgs a, double* __restrict__ out) {
  energy_finish_body(a, out);
}

__global__ void __launch_bounds__(256) energy_finish_kernel_batch(const EnergyArgs* __restrict__ tab) {
  const EnergyArgs a = tab[blockIdx.x];
  energy_finish_body(a, a.result);
}

hipError_t launch_energy_finish(const EnergyArgs& a, double* out, hipStream_t s) {
  hipLaunchKernelGGL(energy_finish_kernel, dim3(1), dim3(256), 0, s, a, out);
  return hipGetLastError();
}

template <int N>
hipError_t launch_energy_row(const EnergyArgs& a, hipStream_t s) {
  constexpr int T = N / energy_points(N);
  const dim3 grid(a.ny / a.rows), block(2 * T * a.rows);
  const size_t lds = energy_lds_bytes(N, a.rows);
  if (a.psi64) hipLaunchKernelGGL((energy_row_kernel<N, double4>), grid, block, lds, s, a);
  else hipLaunchKernelGGL((energy_row_kernel<N, float4>), grid, block, lds, s, a);
  return hipGetLastError();
}

template <int N>
hipError_t launch_energy_col(const EnergyArgs& a, hipStream_t s) {
  constexpr int T = N / energy_points(N);
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

template <int N>
hipError_t launch_energy_row_batch(const EnergyArgs* tab, int count, int ny, int rows, hipStream_t s) {
  constexpr int T = N / energy_points(N);
  hipLaunchKernelGGL((energy_row_kernel_batch<N, float4>), dim3(ny / rows, count), dim3(2 * T * rows),
                     energy_lds_bytes(N, rows), s, tab);
  return hipGetLastError();
}

template <int N>
hipError_t launch_energy_col_batch(const EnergyArgs* tab, int count, int nx, int cols, hipStream_t s) {
  constexpr int T = N / energy_points(N);
  hipLaunchKernelGGL((energy_col_kernel_batch<N, float4>), dim3(nx / cols, count), dim3(2 * T * cols),
                     energy_lds_bytes(N, cols), s, tab);
  return hipGetLastError();
}

hipError_t launch_energy_batch(const EnergyArgs* tab, int count, int nx, int ny, int rows, int cols, hipStream_t s) {
  hipError_t e = hipErrorInvalidValue;
  switch (nx) {
    case 16: e = launch_energy_row_batch<16>(tab, count, ny, rows, s); break;
    case 32: e = launch_energy_row_batch<32>(tab, count, ny, rows, s); break;
    case 64: e = launch_energy_row_batch<64>(tab, count, ny, rows, s); break;
    case 128: e = launch_energy_row_batch<128>(tab, count, ny, rows, s); break;
    case 256: e = launch_energy_row_batch<256>(tab, count, ny, rows, s); break;
    case 512: e = launch_energy_row_batch<512>(tab, count, ny, rows, s); break;
    case 1024: e = launch_energy_row_batch<1024>(tab, count, ny, rows, s); break;
    case 2048: e = launch_energy_row_batch<2048>(tab, count, ny, rows, s); break;
    case 4096: e = launch_energy_row_batch<4096>(tab, count, ny, rows, s); break;
    default: break;
  }
  if (e != hipSuccess) return e;
  switch (ny) {
    case 16: e = launch_energy_col_batch<16>(tab, count, nx, cols, s); break;
    case 32: e = launch_energy_col_batch<32>(tab, count, nx, cols, s); break;
    case 64: e = launch_energy_col_batch<64>(tab, count, nx, cols, s); break;
    case 128: e = launch_energy_col_batch<128>(tab, count, nx, cols, s); break;
    case 256: e = launch_energy_col_batch<256>(tab, count, nx, cols, s); break;
    case 512: e = launch_energy_col_batch<512>(tab, count, nx, cols, s); break;
    case 1024: e = launch_energy_col_batch<1024>(tab, count, nx, cols, s); break;
    case 2048: e = launch_energy_col_batch<2048>(tab, count, nx, cols, s); break;
    case 4096: e = launch_energy_col_batch<4096>(tab, count, nx, cols, s); break;
    default: e = hipErrorInvalidValue; break;
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(energy_finish_kernel_batch, dim3(count), dim3(256), 0, s, tab);
  return hipGetLastError();
}

// Count of non-finite values per workgroup (as doubles, in the norm's partial buffer): the check of a
// state handed over in device memory.
template <class Q>
__global__ void __launch_bounds__(256) nonfinite_kernel(const Q* __restrict__ psi, long long n,
                                                        double* __restrict__ partials) {
  __shared__ double red[64];
  double bad = 0.0;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x) {
    const Q w = psi[i];
    bad += (isfinite(w.x) && isfinite(w.y) && isfinite(w.z) && isfinite(w.w)) ? 0.0 : 1.0;
  }
  const double s = block_sum(bad, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

hipError_t launch_nonfinite(const float4* psi, long long npts, double* partials, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(nonfinite_kernel<float4>, dim3(nblocks), dim3(256), 0, s, psi, npts, partials);
  return hipGetLastError();
}

hipError_t launch_nonfinite(const double4* psi, long long npts, double* partials, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(nonfinite_kernel<double4>, dim3(nblocks), dim3(256), 0, s, psi, npts, partials);
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
