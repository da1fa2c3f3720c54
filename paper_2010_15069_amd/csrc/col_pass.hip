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
#include "col_body.hpp"

namespace sgpe {


// One instance: workgroup blockIdx.x of the pass.  A batch of instances of one grid shape:
// grid of (items, instances) read by batch_item (all of an instance on one XCD), the instance's
// arguments from a device table.
template <int N, int NORM, int ITERS, int P>
__global__ void __launch_bounds__(ITERS == 2 ? 256 : 512) col_kernel(ColArgs a) {
  col_body<N, NORM, ITERS, P, true>(a, blockIdx.x, gridDim.x);
}

template <int N, int NORM, int P>
__global__ void __launch_bounds__(512) col_kernel_batch(const ColArgs* __restrict__ tab) {
  const int2 w = batch_item();
  col_body<N, NORM, 1, P, false>(tab[w.x], w.y, gridDim.x);
}

// complex128: 16 (or, for columns up to kMaxNSmallP, 8) points per lane, one tile per workgroup;
// the host keeps tiles at 256 threads except where one column alone needs more
template <int N, int NORM, int P>
__global__ void __launch_bounds__(2 * N / P > 256 ? 512 : 256) col_kernel_c128(ColArgsT<double> a) {
  col_body<N, NORM, 1, P, false>(a, blockIdx.x, gridDim.x);
}

// -------------------------------------------------------------------------------------------
// Launcher
// -------------------------------------------------------------------------------------------
template <int N, int NORM>
static hipError_t col_launch_t(const ColArgs& a, const ColArgs* tab, int count, int iters, int points, hipStream_t s) {
  const dim3 block(2 * a.cols * (N / points));
  const dim3 grid(a.nx / (a.cols * iters), tab ? count : 1);
  const size_t lds = col_lds_bytes(N, a.cols);
  if (tab) {
    if (points == 16) hipLaunchKernelGGL((col_kernel_batch<N, NORM, 16>), grid, block, lds, s, tab);
    else if constexpr (N <= kMaxNSmallP) {
      if (points == 8) hipLaunchKernelGGL((col_kernel_batch<N, NORM, 8>), grid, block, lds, s, tab);
      else hipLaunchKernelGGL((col_kernel_batch<N, NORM, 4>), grid, block, lds, s, tab);
    }
  } else if (points == 16) {
    if (iters == 2) hipLaunchKernelGGL((col_kernel<N, NORM, 2, 16>), grid, block, lds, s, a);
    else hipLaunchKernelGGL((col_kernel<N, NORM, 1, 16>), grid, block, lds, s, a);
  } else if constexpr (N <= kMaxNSmallP) {
    if (points == 8 && iters == 2) hipLaunchKernelGGL((col_kernel<N, NORM, 2, 8>), grid, block, lds, s, a);
    else if (points == 8) hipLaunchKernelGGL((col_kernel<N, NORM, 1, 8>), grid, block, lds, s, a);
    else hipLaunchKernelGGL((col_kernel<N, NORM, 1, 4>), grid, block, lds, s, a);
  }
  return hipGetLastError();
}

template <int N>
static hipError_t col_launch_n(const ColArgs& a, const ColArgs* tab, int count, int norm, int iters, int points,
                               hipStream_t s) {
  switch (norm) {
    case NORM_NONE: return col_launch_t<N, NORM_NONE>(a, tab, count, iters, points, s);
    case NORM_DOT: return col_launch_t<N, NORM_DOT>(a, tab, count, iters, points, s);
    case NORM_SQ: return col_launch_t<N, NORM_SQ>(a, tab, count, iters, points, s);
    default: return hipErrorInvalidValue;
  }
}

static hipError_t col_dispatch(const ColArgs& a, const ColArgs* tab, int count, int norm, int iters, int points,
                               hipStream_t s) {
  if (!schedule_supported(a.ny, a.cols, iters, points)) return hipErrorInvalidValue;
  if (a.nx % (a.cols * iters) != 0) return hipErrorInvalidValue;
  if (tab && (iters != 1 || count < 1 || count > 65535)) return hipErrorInvalidValue;
  switch (a.ny) {
    case 16: return col_launch_n<16>(a, tab, count, norm, iters, points, s);
    case 32: return col_launch_n<32>(a, tab, count, norm, iters, points, s);
    case 64: return col_launch_n<64>(a, tab, count, norm, iters, points, s);
    case 128: return col_launch_n<128>(a, tab, count, norm, iters, points, s);
    case 256: return col_launch_n<256>(a, tab, count, norm, iters, points, s);
    case 512: return col_launch_n<512>(a, tab, count, norm, iters, points, s);
    case 1024: return col_launch_n<1024>(a, tab, count, norm, iters, points, s);
    case 2048: return col_launch_n<2048>(a, tab, count, norm, iters, points, s);
    case 4096: return col_launch_n<4096>(a, tab, count, norm, iters, points, s);
    default: return hipErrorInvalidValue;
  }
}

template <int N, int NORM>
static hipError_t col_launch_c128(const ColArgsT<double>& a, int points, hipStream_t s) {
  const dim3 block(2 * a.cols * (N / points));
  const dim3 grid(a.nx / a.cols);
  if (block.x > (2 * N / points > 256 ? 512u : 256u)) return hipErrorInvalidValue;
  const size_t lds = col_lds_bytes_c128(N, a.cols, points);   // double2 slots (and the k_y row)
  if (points == 16) {
    hipLaunchKernelGGL((col_kernel_c128<N, NORM, 16>), grid, block, lds, s, a);
  } else if constexpr (N <= kMaxNSmallP) {
    hipLaunchKernelGGL((col_kernel_c128<N, NORM, 8>), grid, block, lds, s, a);
  }
  return hipGetLastError();
}

template <int N>
static hipError_t col_launch_c128_n(const ColArgsT<double>& a, int norm_mode, int points, hipStream_t s) {
  switch (norm_mode) {
    case NORM_NONE: return col_launch_c128<N, NORM_NONE>(a, points, s);
    case NORM_DOT: return col_launch_c128<N, NORM_DOT>(a, points, s);
    case NORM_SQ: return col_launch_c128<N, NORM_SQ>(a, points, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_col(const ColArgsT<double>& a, int norm_mode, int points, hipStream_t s) {
  if ((points != 16 && points != 8) || !schedule_supported(a.ny, a.cols, 1, points) || a.cols > a.nx ||
      a.nx % a.cols != 0)
    return hipErrorInvalidValue;
  switch (a.ny) {
    case 16: return col_launch_c128_n<16>(a, norm_mode, points, s);
    case 32: return col_launch_c128_n<32>(a, norm_mode, points, s);
    case 64: return col_launch_c128_n<64>(a, norm_mode, points, s);
    case 128: return col_launch_c128_n<128>(a, norm_mode, points, s);
    case 256: return col_launch_c128_n<256>(a, norm_mode, points, s);
    case 512: return col_launch_c128_n<512>(a, norm_mode, points, s);
    case 1024: return col_launch_c128_n<1024>(a, norm_mode, points, s);
    case 2048: return col_launch_c128_n<2048>(a, norm_mode, points, s);
    case 4096: return col_launch_c128_n<4096>(a, norm_mode, points, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_col(const ColArgs& a, int norm, int iters, int points, hipStream_t s) {
  return col_dispatch(a, nullptr, 1, norm, iters, points, s);
}

hipError_t launch_col_batch(const ColArgs& shape, const ColArgs* tab, int count, int norm, int points, hipStream_t s) {
  if (!tab) return hipErrorInvalidValue;
  return col_dispatch(shape, tab, count, norm, 1, points, s);
}

}  // namespace sgpe
