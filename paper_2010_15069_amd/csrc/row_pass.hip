// HIP kernels of the split-step solver for gfx950: the row pass.
//
// One Strang step K(dt/2) R(dt) K(dt/2) (Sec. 3.2) is computed by two fused sweeps over the
// state, which lives in HBM as [ny][nx] float4 {re_up, im_up, re_dn, im_dn}:
//
//   row pass    -- per row: inverse x-FFT, scale, real-space 2x2 exponential R (trap, detuning,
//                  mean field, spatial Raman coupling; Eqs. (H2)-(H4)), forward x-FFT;
//   column pass -- per column: forward y-FFT, k-space 2x2 propagator (kinetic, spin-momentum and
//                  uniform Raman coupling; Eqs. (H1), (H4)), inverse y-FFT.
//
// Between sweeps the state is in the mixed representation (k_x, y).  Adjacent K(dt/2) halves of
// consecutive steps are merged into one K(dt) in the column pass, so a run of n steps costs
// 2n + 2 sweeps.  In imaginary time the column pass also produces the norm that the next row pass
// rescales by (Parseval), so renormalisation costs no extra sweep.
//
// Thread layout: lanes 2j and 2j+1 own the up and down component of the same 16 positions of a
// row; a global load of a lane pair is one contiguous 16-byte point, so a wave reads 512
// contiguous bytes per instruction.  The transforms of the two components are independent; the
// 2x2 real-space exponential gets the partner component over a DPP lane swap.
//
// Every operator close to the identity is applied as psi + (U - 1) psi with U - 1 held to fp32
// relative accuracy, and the small correction is formed before it is added to psi (one rounding
// of the large value), so that unit-modulus propagators do not drift coherently.
#include "row_body.hpp"

namespace sgpe {


// Row groups are sized for 256 threads (row_rows_per_block); only a 4096-point row at 16 points
// per lane needs 512.  The tighter bound gives the variants' two real-space routines the
// registers they need without spilling.
template <int N, bool IMAG, bool FULL, int P>
__global__ void __launch_bounds__(2 * N / P > 256 ? 512 : 256) row_var_kernel(RowArgs a) {
  row_var_body<N, IMAG, FULL, P>(a, blockIdx.x);
}

// One instance: workgroup blockIdx.x of the pass.  A batch of instances of one grid shape:
// grid of (items, instances) read by batch_item (all of an instance on one XCD), the instance's
// arguments from a device table.
template <int N, int MODE, bool IMAG, bool FULL, int ITERS, int P>
__global__ void __launch_bounds__(ITERS == 2 ? 256 : 512) row_kernel(RowArgs a) {
  row_body<N, MODE, IMAG, FULL, ITERS, P, true>(a, blockIdx.x);
}

// complex128: 16 (or, for rows up to kMaxNSmallP, 8) points per lane, one row group per
// workgroup; row groups are sized for 256 threads except where one row needs 512
template <int N, int MODE, bool IMAG, bool FULL, int P>
__global__ void __launch_bounds__(2 * N / P > 256 ? 512 : 256) row_kernel_c128(RowArgsT<double> a) {
  row_body<N, MODE, IMAG, FULL, 1, P, false>(a, blockIdx.x);
}

template <int N, int MODE, bool IMAG, bool FULL, int P>
__global__ void __launch_bounds__(512) row_kernel_batch(const RowArgs* __restrict__ tab) {
  const int2 w = batch_item();
  row_body<N, MODE, IMAG, FULL, 1, P, false>(tab[w.x], w.y);
}

// -------------------------------------------------------------------------------------------
// Launcher
// -------------------------------------------------------------------------------------------
template <int N, int MODE, bool IMAG, bool FULL>
static hipError_t row_launch_t(const RowArgs& a, const RowArgs* tab, int count, int iters, int points, hipStream_t s) {
  const dim3 block(2 * a.rows_per_block * (N / points));
  const dim3 grid(a.ny / (a.rows_per_block * iters), tab ? count : 1);
  const size_t lds = row_lds_bytes(N, a.rows_per_block);
  if constexpr (MODE == ROW_VAR) {
    if (tab || iters != 1) return hipErrorInvalidValue;
    if (block.x > static_cast<unsigned>(2 * N / points > 256 ? 512 : 256)) return hipErrorInvalidValue;
    if (points == 16) hipLaunchKernelGGL((row_var_kernel<N, IMAG, FULL, 16>), grid, block, lds, s, a);
    else if constexpr (N <= kMaxNSmallP) {
      if (points == 8) hipLaunchKernelGGL((row_var_kernel<N, IMAG, FULL, 8>), grid, block, lds, s, a);
      else hipLaunchKernelGGL((row_var_kernel<N, IMAG, FULL, 4>), grid, block, lds, s, a);
    }
    return hipGetLastError();
  } else if (tab) {
    if constexpr (MODE == ROW_STEP_NLN) {
      return hipErrorInvalidValue;   // batches run the default split only
    } else {
      if (points == 16) hipLaunchKernelGGL((row_kernel_batch<N, MODE, IMAG, FULL, 16>), grid, block, lds, s, tab);
      else if constexpr (N <= kMaxNSmallP) {
        if (points == 8) hipLaunchKernelGGL((row_kernel_batch<N, MODE, IMAG, FULL, 8>), grid, block, lds, s, tab);
        else hipLaunchKernelGGL((row_kernel_batch<N, MODE, IMAG, FULL, 4>), grid, block, lds, s, tab);
      }
    }
  } else if (points == 16) {
    if (iters == 2) hipLaunchKernelGGL((row_kernel<N, MODE, IMAG, FULL, 2, 16>), grid, block, lds, s, a);
    else hipLaunchKernelGGL((row_kernel<N, MODE, IMAG, FULL, 1, 16>), grid, block, lds, s, a);
  } else if constexpr (N <= kMaxNSmallP) {
    if (points == 8 && iters == 2) hipLaunchKernelGGL((row_kernel<N, MODE, IMAG, FULL, 2, 8>), grid, block, lds, s, a);
    else if (points == 8) hipLaunchKernelGGL((row_kernel<N, MODE, IMAG, FULL, 1, 8>), grid, block, lds, s, a);
    else hipLaunchKernelGGL((row_kernel<N, MODE, IMAG, FULL, 1, 4>), grid, block, lds, s, a);
  }
  return hipGetLastError();
}

template <int N>
static hipError_t row_launch_n(const RowArgs& a, const RowArgs* tab, int count, int mode, bool imag, bool full,
                               int iters, int points, hipStream_t s) {
  switch (mode) {
    case ROW_FWD: return row_launch_t<N, ROW_FWD, false, false>(a, tab, count, iters, points, s);
    case ROW_INV: return row_launch_t<N, ROW_INV, false, false>(a, tab, count, iters, points, s);
    case ROW_STEP:
      if (imag) return full ? row_launch_t<N, ROW_STEP, true, true>(a, tab, count, iters, points, s)
                            : row_launch_t<N, ROW_STEP, true, false>(a, tab, count, iters, points, s);
      return full ? row_launch_t<N, ROW_STEP, false, true>(a, tab, count, iters, points, s)
                  : row_launch_t<N, ROW_STEP, false, false>(a, tab, count, iters, points, s);
    case ROW_STEP_NLN:
      // real time with a diagonal linear part: N L N is exactly the frozen form's one phase
      if (imag) return full ? row_launch_t<N, ROW_STEP_NLN, true, true>(a, tab, count, iters, points, s)
                            : row_launch_t<N, ROW_STEP_NLN, true, false>(a, tab, count, iters, points, s);
      return full ? row_launch_t<N, ROW_STEP_NLN, false, true>(a, tab, count, iters, points, s)
                  : row_launch_t<N, ROW_STEP, false, false>(a, tab, count, iters, points, s);
    case ROW_VAR:
      if (imag) return full ? row_launch_t<N, ROW_VAR, true, true>(a, tab, count, iters, points, s)
                            : row_launch_t<N, ROW_VAR, true, false>(a, tab, count, iters, points, s);
      return full ? row_launch_t<N, ROW_VAR, false, true>(a, tab, count, iters, points, s)
                  : row_launch_t<N, ROW_VAR, false, false>(a, tab, count, iters, points, s);
    default: return hipErrorInvalidValue;
  }
}

static hipError_t row_dispatch(const RowArgs& a, const RowArgs* tab, int count, int mode, bool imag, bool full,
                               int iters, int points, hipStream_t s) {
  if (!schedule_supported(a.nx, a.rows_per_block, iters, points)) return hipErrorInvalidValue;
  if (a.ny % (a.rows_per_block * iters) != 0) return hipErrorInvalidValue;
  if (tab && (iters != 1 || count < 1 || count > 65535)) return hipErrorInvalidValue;
  switch (a.nx) {
    case 16: return row_launch_n<16>(a, tab, count, mode, imag, full, iters, points, s);
    case 32: return row_launch_n<32>(a, tab, count, mode, imag, full, iters, points, s);
    case 64: return row_launch_n<64>(a, tab, count, mode, imag, full, iters, points, s);
    case 128: return row_launch_n<128>(a, tab, count, mode, imag, full, iters, points, s);
    case 256: return row_launch_n<256>(a, tab, count, mode, imag, full, iters, points, s);
    case 512: return row_launch_n<512>(a, tab, count, mode, imag, full, iters, points, s);
    case 1024: return row_launch_n<1024>(a, tab, count, mode, imag, full, iters, points, s);
    case 2048: return row_launch_n<2048>(a, tab, count, mode, imag, full, iters, points, s);
    case 4096: return row_launch_n<4096>(a, tab, count, mode, imag, full, iters, points, s);
    default: return hipErrorInvalidValue;
  }
}

template <int N, int MODE, bool IMAG, bool FULL>
static hipError_t row_launch_c128(const RowArgsT<double>& a, int points, hipStream_t s) {
  const dim3 block(2 * a.rows_per_block * (N / points));
  const dim3 grid(a.ny / a.rows_per_block);
  if (block.x > (2 * N / points > 256 ? 512u : 256u)) return hipErrorInvalidValue;
  const size_t lds = 2 * row_lds_bytes(N, a.rows_per_block);   // double2 slots
  if (points == 16) {
    hipLaunchKernelGGL((row_kernel_c128<N, MODE, IMAG, FULL, 16>), grid, block, lds, s, a);
  } else if constexpr (N <= kMaxNSmallP) {
    hipLaunchKernelGGL((row_kernel_c128<N, MODE, IMAG, FULL, 8>), grid, block, lds, s, a);
  }
  return hipGetLastError();
}

template <int N>
static hipError_t row_launch_c128_n(const RowArgsT<double>& a, int mode, bool imag, bool full, int points,
                                    hipStream_t s) {
  switch (mode) {
    case ROW_FWD: return row_launch_c128<N, ROW_FWD, false, false>(a, points, s);
    case ROW_INV: return row_launch_c128<N, ROW_INV, false, false>(a, points, s);
    case ROW_STEP:
      if (imag) return full ? row_launch_c128<N, ROW_STEP, true, true>(a, points, s)
                            : row_launch_c128<N, ROW_STEP, true, false>(a, points, s);
      return full ? row_launch_c128<N, ROW_STEP, false, true>(a, points, s)
                  : row_launch_c128<N, ROW_STEP, false, false>(a, points, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_row(const RowArgsT<double>& a, int mode, bool imag, bool full, int points, hipStream_t s) {
  if ((points != 16 && points != 8) || !schedule_supported(a.nx, a.rows_per_block, 1, points))
    return hipErrorInvalidValue;
  if (a.ny % a.rows_per_block != 0) return hipErrorInvalidValue;
  switch (a.nx) {
    case 16: return row_launch_c128_n<16>(a, mode, imag, full, points, s);
    case 32: return row_launch_c128_n<32>(a, mode, imag, full, points, s);
    case 64: return row_launch_c128_n<64>(a, mode, imag, full, points, s);
    case 128: return row_launch_c128_n<128>(a, mode, imag, full, points, s);
    case 256: return row_launch_c128_n<256>(a, mode, imag, full, points, s);
    case 512: return row_launch_c128_n<512>(a, mode, imag, full, points, s);
    case 1024: return row_launch_c128_n<1024>(a, mode, imag, full, points, s);
    case 2048: return row_launch_c128_n<2048>(a, mode, imag, full, points, s);
    case 4096: return row_launch_c128_n<4096>(a, mode, imag, full, points, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_row(const RowArgs& a, int mode, bool imag, bool full, int iters, int points, hipStream_t s) {
  return row_dispatch(a, nullptr, 1, mode, imag, full, iters, points, s);
}

hipError_t launch_row_batch(const RowArgs& shape, const RowArgs* tab, int count, int mode, bool imag, bool full,
                            int points, hipStream_t s) {
  if (!tab) return hipErrorInvalidValue;
  return row_dispatch(shape, tab, count, mode, imag, full, 1, points, s);
}

}  // namespace sgpe
