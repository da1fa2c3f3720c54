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

// Energy kernels: one lane holds both components of its 16 positions.
int energy_rows_per_block(int nx, int ny, size_t max_lds) {
  const int t = nx / 16;
  int rows = 256 / t;
  if (rows < 1) rows = 1;
  if (rows > ny) rows = ny;
  while (rows > 1 && size_t(rows) * size_t(nx + nx / 16) * 16 > max_lds) rows >>= 1;
  return rows;
}

int energy_cols_per_block(int nx, int ny, size_t max_lds) {
  const int t = ny / 16;
  int c = 256 / t;
  if (c < 1) c = 1;
  if (c > nx) c = nx;
  while (c > 1 && size_t(c) * size_t(ny + ny / 16) * 16 > max_lds) c >>= 1;
  return c;
}

int norm_blocks() { return 256; }

// -------------------------------------------------------------------------------------------
// Energy: real-space terms and norm (row kernel, then x-FFT into scratch), k-space quadratic
// form (column kernel, y-FFT, no write).  Products and sums in fp64.
// -------------------------------------------------------------------------------------------
template <int N>
__global__ void __launch_bounds__(256) energy_row_kernel(EnergyArgs a) {
  extern __shared__ float4 lds_raw[];
  __shared__ double red[64];
  constexpr int T = N / 16;
  constexpr int SLOTS = N + N / 16;
  const int tid = threadIdx.x;
  const int rloc = tid / T;
  const int t = tid - rloc * T;
  const int row = blockIdx.x * a.rows_per_block + rloc;
  const LdsView<float4> lds{lds_raw + rloc * SLOTS, 0};
  const float4* __restrict__ p = a.psi + size_t(row) * N;
  float4 v[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) v[m] = p[t + T * m];
  TwRegs<N> tr;
  load_twiddles<N>(tr, t, a.twx);
  const double y = a.ymin + a.dy * row;
  const double om_row = a.om_y ? a.om_y[row] : 0.0;
  double er = 0.0, nr = 0.0;
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int j = t + T * m;
    const double x = a.xmin + a.dx * j;
    const double V = a.wx2h * x * x + a.wy2h * y * y;
    const double ur = v[m].x, ui = v[m].y, dr = v[m].z, di = v[m].w;
    const double nu = ur * ur + ui * ui, nd = dr * dr + di * di;
    const double om = a.om_x ? a.om_x[j] + om_row : 0.0;
    er += V * (nu + nd) + 0.5 * a.delta * (nu - nd) + om * (ur * dr + ui * di) +
          0.5 * a.g_uu * nu * nu + 0.5 * a.g_dd * nd * nd + a.g_ud * nu * nd;
    nr += nu + nd;
  }
  const double se = block_sum(er, red);
  const double sn = block_sum(nr, red);
  if (tid == 0) {
    a.row_partials[2 * blockIdx.x] = se;
    a.row_partials[2 * blockIdx.x + 1] = sn;
  }
  fft_pass<N, -1>(v, lds, t, tr);
  float4* __restrict__ q = a.scratch + size_t(row) * N;
#pragma unroll
  for (int m = 0; m < 16; ++m) q[t + T * m] = v[m];
}

template <int N>
__global__ void __launch_bounds__(256) energy_col_kernel(EnergyArgs a) {
  extern __shared__ float4 lds_raw[];
  __shared__ double red[64];
  constexpr int T = N / 16;
  const int C = a.cols;
  const int tid = threadIdx.x;
  const int c = tid & (C - 1);
  const int t = tid / C;
  const int x = blockIdx.x * C + c;
  const LdsView<float4> lds{lds_raw + c, __builtin_ctz(C)};
  const float4* __restrict__ p = a.scratch + x;
  const size_t rs = size_t(a.nx);
  float4 v[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) v[m] = p[size_t(t + T * m) * rs];
  TwRegs<N> tr;
  load_twiddles<N>(tr, t, a.twy);
  fft_pass<N, -1>(v, lds, t, tr);
  const double kx = (x < a.nx / 2 ? x : x - a.nx) * a.dkx;
  const double bz = a.k_l * kx;
  double acc = 0.0;
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int iy = t + T * m;
    const double ky = (iy < N / 2 ? iy : iy - N) * a.dky;
    const double ak = 0.5 * (kx * kx + ky * ky);
    const double ur = v[m].x, ui = v[m].y, dr = v[m].z, di = v[m].w;
    const double pu = ur * ur + ui * ui, pd = dr * dr + di * di;
    acc += ak * (pu + pd) + bz * (pu - pd) + a.omega * (ur * dr + ui * di);
  }
  const double s = block_sum(acc, red);
  if (tid == 0) a.col_partials[blockIdx.x] = s;
}

// -------------------------------------------------------------------------------------------
// Norm: sum |psi|^2 with a fixed grid (deterministic), fp64.
// -------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) norm_kernel(const float4* __restrict__ psi, long long n,
                                                   double* __restrict__ partials) {
  __shared__ double red[64];
  double acc = 0.0;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x) {
    const float4 w = psi[i];
    const double ur = w.x, ui = w.y, dr = w.z, di = w.w;
    acc += ur * ur + ui * ui + dr * dr + di * di;
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

template <int N>
static hipError_t energy_row_launch(const EnergyArgs& a, hipStream_t s) {
  const dim3 block(a.rows_per_block * (N / 16));
  const dim3 grid(a.ny / a.rows_per_block);
  hipLaunchKernelGGL((energy_row_kernel<N>), grid, block, size_t(a.rows_per_block) * (N + N / 16) * 16, s, a);
  return hipGetLastError();
}

template <int N>
static hipError_t energy_col_launch(const EnergyArgs& a, hipStream_t s) {
  const dim3 block(a.cols * (N / 16));
  const dim3 grid(a.nx / a.cols);
  hipLaunchKernelGGL((energy_col_kernel<N>), grid, block, size_t(a.cols) * (N + N / 16) * 16, s, a);
  return hipGetLastError();
}

#define SGPE_SIZE_SWITCH(n, fn, ...)                      \
  switch (n) {                                            \
    case 16: return fn<16>(__VA_ARGS__);                  \
    case 32: return fn<32>(__VA_ARGS__);                  \
    case 64: return fn<64>(__VA_ARGS__);                  \
    case 128: return fn<128>(__VA_ARGS__);                \
    case 256: return fn<256>(__VA_ARGS__);                \
    case 512: return fn<512>(__VA_ARGS__);                \
    case 1024: return fn<1024>(__VA_ARGS__);              \
    case 2048: return fn<2048>(__VA_ARGS__);              \
    case 4096: return fn<4096>(__VA_ARGS__);              \
    default: return hipErrorInvalidValue;                 \
  }

static hipError_t energy_row_dispatch(const EnergyArgs& a, hipStream_t s) {
  SGPE_SIZE_SWITCH(a.nx, energy_row_launch, a, s)
}
static hipError_t energy_col_dispatch(const EnergyArgs& a, hipStream_t s) {
  SGPE_SIZE_SWITCH(a.ny, energy_col_launch, a, s)
}

hipError_t launch_energy(const EnergyArgs& a, hipStream_t s) {
  hipError_t e = energy_row_dispatch(a, s);
  if (e != hipSuccess) return e;
  return energy_col_dispatch(a, s);
}

hipError_t launch_norm(const float4* psi, long long npts, double* partials, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(norm_kernel, dim3(nblocks), dim3(256), 0, s, psi, npts, partials);
  return hipGetLastError();
}

}  // namespace sgpe
