// HIP kernels of the split-step solver for gfx950: the column pass.
//
// Per column: forward y-FFT, the k-space 2x2 propagator U_K(h) (kinetic + spin-momentum term of
// Eq. (H1) and the uniform Raman coupling of Eq. (H4), exponentiated per Eq. (TEOp)), inverse
// y-FFT; in imaginary time it also writes one fp64 norm partial per workgroup.  The state is read
// and written in the mixed (k_x, y) representation left by the row pass (see row_pass.hip).
//
// Thread layout: lanes 2j and 2j+1 own the up and down component of the same positions of a
// column; consecutive lane pairs own consecutive columns, so one row of a C-column tile is
// 16 C contiguous bytes.  U_K couples the components; the partner comes over a DPP lane swap.
//
// U_K = P(k_y) M'(k_x) is applied as w + [c1 + q (w + c1)] with c1 = (M' - 1) w and q = P - 1,
// the bracket formed first and added to w once: the dominant modes of a smooth state are rounded
// once per step instead of twice per factor (which gives a coherent norm drift).
#include "fft_device.hpp"
#include "sgpe_internal.hpp"

namespace sgpe {

__device__ __forceinline__ int col_tile(int b, int ntiles) {
  // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a contiguous run of tiles so
  // that tiles sharing 128-byte lines meet in the same L2.
  if ((ntiles & 7) == 0) return (b & 7) * (ntiles >> 3) + (b >> 3);
  return b;
}

template <int N, int NORM>
__global__ void __launch_bounds__(512) col_kernel(ColArgs a) {
  extern __shared__ float2 lds_raw[];
  __shared__ double red[64];
  constexpr int T = N / 16;
  const int C = a.cols;
  const int tid = threadIdx.x;
  const int comp = tid & 1;
  const int pair = tid >> 1;
  const int cc = pair & (C - 1);
  const int t = pair / C;
  const int tile = col_tile(blockIdx.x, a.nx / C);
  const int x = tile * C + cc;
  const LdsView<float2> lds{lds_raw + 2 * cc + comp, 1 + __builtin_ctz(C)};
  // element (row y) of this lane's component is at byte offset 16 (y nx + x) + 8 comp; 32-bit
  // offsets from a wave-uniform base, the row stride a wave-uniform value
  const char* __restrict__ base = reinterpret_cast<const char*>(a.psi);
  const uint32_t rstride = 16u * static_cast<uint32_t>(a.nx);
  const uint32_t off0 = static_cast<uint32_t>(t) * rstride + 16u * static_cast<uint32_t>(x) + 8u * comp;
  const uint32_t mstride = static_cast<uint32_t>(T) * rstride;

  float2 v[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) v[m] = *reinterpret_cast<const float2*>(base + off0 + mstride * m);
  TwPlain<N> tr;
  load_twiddles<N>(tr, t, a.tw);
  // this component's row of M' - 1 at k_x: {d_own, d_other}
  const float4 d = a.kx_tab[2 * x + comp];

  fwd_pass<N>(v, lds, t, tr);

  double acc = 0.0;
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const float2 w = v[m];
    const float2 o = pair_swap(w);
    const float2 q = *reinterpret_cast<const float2*>(reinterpret_cast<const char*>(a.ky_tab) + 8u * static_cast<uint32_t>(t + T * m));
    const float c1r = fmaf(-d.w, o.y, fmaf(d.z, o.x, fmaf(-d.y, w.y, d.x * w.x)));
    const float c1i = fmaf(d.w, o.x, fmaf(d.z, o.y, fmaf(d.y, w.x, d.x * w.y)));
    const float cr = fmaf(-q.y, w.y, fmaf(q.x, w.x, fmaf(-q.y, c1i, fmaf(q.x, c1r, c1r))));
    const float ci = fmaf(q.y, w.x, fmaf(q.x, w.y, fmaf(q.y, c1r, fmaf(q.x, c1i, c1i))));
    const float2 out = make_float2(w.x + cr, w.y + ci);
    if constexpr (NORM == NORM_DOT) {
      acc += static_cast<double>(fmaf(w.x, out.x, w.y * out.y));
    } else if constexpr (NORM == NORM_SQ) {
      acc += static_cast<double>(fmaf(out.x, out.x, out.y * out.y));
    }
    v[m] = out;
  }
  if constexpr (NORM != NORM_NONE) {
    const double s = block_sum(acc, red);
    if (tid == 0) a.partials[blockIdx.x] = s;
  }

  inv_pass<N>(v, lds, t, tr);

  char* __restrict__ out = reinterpret_cast<char*>(a.psi);
#pragma unroll
  for (int m = 0; m < 16; ++m) *reinterpret_cast<float2*>(out + off0 + mstride * m) = v[m];
}

// -------------------------------------------------------------------------------------------
// Launcher
// -------------------------------------------------------------------------------------------
template <int N, int NORM>
static hipError_t col_launch_t(const ColArgs& a, hipStream_t s) {
  const dim3 block(2 * a.cols * (N / 16));
  const dim3 grid(a.nx / a.cols);
  hipLaunchKernelGGL((col_kernel<N, NORM>), grid, block, col_lds_bytes(N, a.cols), s, a);
  return hipGetLastError();
}

template <int N>
static hipError_t col_launch_n(const ColArgs& a, int norm, hipStream_t s) {
  switch (norm) {
    case NORM_NONE: return col_launch_t<N, NORM_NONE>(a, s);
    case NORM_DOT: return col_launch_t<N, NORM_DOT>(a, s);
    case NORM_SQ: return col_launch_t<N, NORM_SQ>(a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_col(const ColArgs& a, int norm, hipStream_t s) {
  switch (a.ny) {
    case 16: return col_launch_n<16>(a, norm, s);
    case 32: return col_launch_n<32>(a, norm, s);
    case 64: return col_launch_n<64>(a, norm, s);
    case 128: return col_launch_n<128>(a, norm, s);
    case 256: return col_launch_n<256>(a, norm, s);
    case 512: return col_launch_n<512>(a, norm, s);
    case 1024: return col_launch_n<1024>(a, norm, s);
    case 2048: return col_launch_n<2048>(a, norm, s);
    case 4096: return col_launch_n<4096>(a, norm, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sgpe
