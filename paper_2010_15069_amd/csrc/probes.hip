// Measurement kernels: the memory floor of the split step's data movement.
//
// The two passes of a step partition the grid differently among workgroups -- by rows, then by
// columns -- so between passes every point moves to a workgroup (and mostly an XCD) other than the
// one that wrote it.  These kernels move exactly that data with no arithmetic: each lane loads the
// 16 values its transform would own (one spinor component of 16 points, the 8-byte half of each
// 16-byte point), then stores them to the other buffer at the same addresses.  Alternating the
// row partition and the column partition gives the floor that a pass of the real schedule cannot
// beat; the layout and tile parameters show what the access granularity costs.
//
// Layout with L interleaved rows (L = 1 is the state's [ny][nx] layout): point (x, y) at index
// ((y / L) nx + x) L + y % L, so L rows of one column form a contiguous 16 L-byte group.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fft_device.hpp"

namespace sgpe {

__device__ __forceinline__ uint32_t probe_index(uint32_t x, uint32_t y, int lnx, int ll) {
  const uint32_t lm = (1u << ll) - 1u;
  return ((((y >> ll) << lnx) + x) << ll) + (y & lm);
}

// Row partition: workgroup w owns rows [w R, w R + R); lane pair p -> (r = p mod R, t = p / R);
// its points are x = t + T m, T = nx / 16.
template <bool WT>
__global__ void __launch_bounds__(1024) probe_rows(const float2* __restrict__ src, float2* __restrict__ dst,
                                                   int lnx, int ll, int lrows) {
  const int comp = threadIdx.x & 1;
  const uint32_t p = threadIdx.x >> 1;
  const uint32_t r = p & ((1u << lrows) - 1u);
  const uint32_t t = p >> lrows;
  const uint32_t tt = (1u << lnx) >> 4;
  const uint32_t y = (blockIdx.x << lrows) + r;
  float2 v[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) v[m] = src[2 * probe_index(t + tt * m, y, lnx, ll) + comp];
#pragma unroll
  for (int m = 0; m < 16; ++m) store_state<WT>(&dst[2 * probe_index(t + tt * m, y, lnx, ll) + comp], v[m]);
}

// Column partition: workgroup w owns columns [c0, c0 + C) (tiles dealt to XCDs in contiguous runs,
// as the column pass does); lane pair p -> (r = p mod L, c = (p / L) mod C, b = p / (L C)),
// t = b L + r; its points are y = t + T m, T = ny / 16.
template <bool WT>
__global__ void __launch_bounds__(1024) probe_cols(const float2* __restrict__ src, float2* __restrict__ dst,
                                                   int lnx, int lny, int ll, int lcols) {
  const int comp = threadIdx.x & 1;
  const uint32_t p = threadIdx.x >> 1;
  const uint32_t r = p & ((1u << ll) - 1u);
  const uint32_t c = (p >> ll) & ((1u << lcols) - 1u);
  const uint32_t b = p >> (ll + lcols);
  const uint32_t t = (b << ll) + r;
  const uint32_t tt = (1u << lny) >> 4;
  const int ng = gridDim.x;
  const int w = (ng & 7) == 0 ? (blockIdx.x & 7) * (ng >> 3) + (blockIdx.x >> 3) : blockIdx.x;
  const uint32_t x = (uint32_t(w) << lcols) + c;
  float2 v[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) v[m] = src[2 * probe_index(x, t + tt * m, lnx, ll) + comp];
#pragma unroll
  for (int m = 0; m < 16; ++m) store_state<WT>(&dst[2 * probe_index(x, t + tt * m, lnx, ll) + comp], v[m]);
}

// Wave-local variants: a wave owns one whole row (or column) with both spinor components per lane
// (16-byte point loads), lane t holding the P = length / 64 positions t + 64 m; a workgroup of W
// waves owns W adjacent rows (columns).  This is the access pattern of transforms that run inside
// one wave.
template <int P, bool WT>
__device__ __forceinline__ void probe_line_wl(const float4* __restrict__ src, float4* __restrict__ dst, uint32_t fixed,
                                              bool along_x, int lnx, int ll) {
  const uint32_t t = threadIdx.x & 63u;
  float4 v[P];
#pragma unroll
  for (int m = 0; m < P; ++m) {
    const uint32_t pos = t + 64u * m;
    v[m] = src[along_x ? probe_index(pos, fixed, lnx, ll) : probe_index(fixed, pos, lnx, ll)];
  }
#pragma unroll
  for (int m = 0; m < P; ++m) {
    const uint32_t pos = t + 64u * m;
    float4* q = &dst[along_x ? probe_index(pos, fixed, lnx, ll) : probe_index(fixed, pos, lnx, ll)];
    if constexpr (WT) {
      store_through(reinterpret_cast<float2*>(q), make_float2(v[m].x, v[m].y));
      store_through(reinterpret_cast<float2*>(q) + 1, make_float2(v[m].z, v[m].w));
    } else {
      *q = v[m];
    }
  }
}

template <int P, bool WT>
__global__ void __launch_bounds__(512) probe_rows_wl(const float4* __restrict__ src, float4* __restrict__ dst,
                                                     int lnx, int ll) {
  const uint32_t y = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  probe_line_wl<P, WT>(src, dst, y, true, lnx, ll);
}

template <int P, bool WT>
__global__ void __launch_bounds__(512) probe_cols_wl(const float4* __restrict__ src, float4* __restrict__ dst,
                                                     int lnx, int ll) {
  const int ng = gridDim.x;
  const int w = (ng & 7) == 0 ? (blockIdx.x & 7) * (ng >> 3) + (blockIdx.x >> 3) : blockIdx.x;
  const uint32_t x = uint32_t(w) * (blockDim.x >> 6) + (threadIdx.x >> 6);
  probe_line_wl<P, WT>(src, dst, x, false, lnx, ll);
}

template <int P>
static hipError_t probe_wl_launch(bool rows, const float4* src, float4* dst, int nx, int ny, int layout_rows,
                                  int waves, bool wt, hipStream_t s) {
  const int lnx = __builtin_ctz(nx), ll = __builtin_ctz(layout_rows);
  const dim3 block(64 * waves), grid((rows ? ny : nx) / waves);
  if (rows) {
    if (wt) hipLaunchKernelGGL((probe_rows_wl<P, true>), grid, block, 0, s, src, dst, lnx, ll);
    else hipLaunchKernelGGL((probe_rows_wl<P, false>), grid, block, 0, s, src, dst, lnx, ll);
  } else {
    if (wt) hipLaunchKernelGGL((probe_cols_wl<P, true>), grid, block, 0, s, src, dst, lnx, ll);
    else hipLaunchKernelGGL((probe_cols_wl<P, false>), grid, block, 0, s, src, dst, lnx, ll);
  }
  return hipGetLastError();
}

static hipError_t probe_wl(bool rows, const float4* src, float4* dst, int nx, int ny, int layout_rows, int waves,
                           bool wt, hipStream_t s) {
  switch (rows ? nx : ny) {
    case 512: return probe_wl_launch<8>(rows, src, dst, nx, ny, layout_rows, waves, wt, s);
    case 1024: return probe_wl_launch<16>(rows, src, dst, nx, ny, layout_rows, waves, wt, s);
    case 2048: return probe_wl_launch<32>(rows, src, dst, nx, ny, layout_rows, waves, wt, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_probe_rows_wl(const float4* src, float4* dst, int nx, int ny, int layout_rows, int waves,
                                bool write_through, hipStream_t s) {
  return probe_wl(true, src, dst, nx, ny, layout_rows, waves, write_through, s);
}

hipError_t launch_probe_cols_wl(const float4* src, float4* dst, int nx, int ny, int layout_rows, int waves,
                                bool write_through, hipStream_t s) {
  return probe_wl(false, src, dst, nx, ny, layout_rows, waves, write_through, s);
}

hipError_t launch_probe_rows(const float4* src, float4* dst, int nx, int ny, int layout_rows, int row_tile,
                             bool write_through, hipStream_t s) {
  const int lnx = __builtin_ctz(nx), ll = __builtin_ctz(layout_rows), lr = __builtin_ctz(row_tile);
  const dim3 block(2 * row_tile * (nx / 16)), grid(ny / row_tile);
  const float2* a = reinterpret_cast<const float2*>(src);
  float2* b = reinterpret_cast<float2*>(dst);
  if (write_through) hipLaunchKernelGGL(probe_rows<true>, grid, block, 0, s, a, b, lnx, ll, lr);
  else hipLaunchKernelGGL(probe_rows<false>, grid, block, 0, s, a, b, lnx, ll, lr);
  return hipGetLastError();
}

hipError_t launch_probe_cols(const float4* src, float4* dst, int nx, int ny, int layout_rows, int col_tile,
                             bool write_through, hipStream_t s) {
  const int lnx = __builtin_ctz(nx), lny = __builtin_ctz(ny), ll = __builtin_ctz(layout_rows),
            lc = __builtin_ctz(col_tile);
  const dim3 block(2 * col_tile * (ny / 16)), grid(nx / col_tile);
  const float2* a = reinterpret_cast<const float2*>(src);
  float2* b = reinterpret_cast<float2*>(dst);
  if (write_through) hipLaunchKernelGGL(probe_cols<true>, grid, block, 0, s, a, b, lnx, lny, ll, lc);
  else hipLaunchKernelGGL(probe_cols<false>, grid, block, 0, s, a, b, lnx, lny, ll, lc);
  return hipGetLastError();
}

// Placement: thread 0 of every workgroup records the XCD it runs on (hardware register XCC_ID,
// bits 3:0) at out[blockIdx.y * gridDim.x + blockIdx.x].
__global__ void probe_xcc_kernel(unsigned* __restrict__ out) {
  if (threadIdx.x == 0) {
    const unsigned id = __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 15u;   // hwreg(XCC_ID, 0, 4)
    out[blockIdx.y * gridDim.x + blockIdx.x] = id;
  }
}

hipError_t launch_probe_xcc(unsigned* out, int gx, int gy, int threads, hipStream_t s) {
  hipLaunchKernelGGL(probe_xcc_kernel, dim3(gx, gy), dim3(threads), 0, s, out);
  return hipGetLastError();
}

}  // namespace sgpe
