// HIP kernels of the split-step solver for gfx950: the column pass.
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
// Every operator close to the identity is applied as psi + (U - 1) psi with U - 1 held to fp32
// relative accuracy, so that unit-modulus propagators do not pick up a coherent |U| != 1 error
// from rounding their tables.
#include "fft_device.hpp"
#include "sgpe_internal.hpp"

namespace sgpe {
// -------------------------------------------------------------------------------------------
// Column pass
// -------------------------------------------------------------------------------------------
__device__ __forceinline__ int col_tile(int b, int ntiles) {
  // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a contiguous run of tiles so
  // that tiles sharing 128-byte lines meet in the same L2.
  if ((ntiles & 7) == 0) return (b & 7) * (ntiles >> 3) + (b >> 3);
  return b;
}

template <int N, int NORM>
__global__ void __launch_bounds__(256) col_kernel(ColArgs a) {
  extern __shared__ float4 lds_raw[];
  __shared__ double red[16];
  constexpr int T = N / 16;
  const int C = a.cols;
  const int tid = threadIdx.x;
  const int c = tid & (C - 1);
  const int t = tid / C;
  const int tile = col_tile(blockIdx.x, a.nx / C);
  const int x = tile * C + c;
  const LdsView lds{lds_raw + c, C};
  float4* __restrict__ p = a.psi + x;
  const size_t rs = size_t(a.nx);

  float4 v[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) v[m] = p[size_t(t + T * m) * rs];
  TwRegs<N> tr;
  load_twiddles<N>(tr, t, a.tw);

  fft_pass<N, -1>(v, lds, t, tr);

  const float4 d0 = a.kx_tab[2 * x];      // d11, d12
  const float4 d1 = a.kx_tab[2 * x + 1];  // d21, d22
  double acc = 0.0;
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const float4 w = v[m];
    const float2 q = a.ky_tab[t + T * m];
    // U = P M' with M' = 1 + D (per k_x) and P = 1 + q (per k_y):
    //   U w = w + [c1 + q (w + c1)],  c1 = D w.
    // The bracket is small; it is accumulated on its own and added to w once, so the dominant
    // modes of a smooth state are rounded once per step (rounding w + small twice per factor
    // gives a coherent norm drift of ~1e-8 per step).
    const float c1ur = fmaf(-d0.w, w.w, fmaf(d0.z, w.z, fmaf(-d0.y, w.y, d0.x * w.x)));
    const float c1ui = fmaf(d0.w, w.z, fmaf(d0.z, w.w, fmaf(d0.y, w.x, d0.x * w.y)));
    const float c1dr = fmaf(-d1.w, w.w, fmaf(d1.z, w.z, fmaf(-d1.y, w.y, d1.x * w.x)));
    const float c1di = fmaf(d1.w, w.z, fmaf(d1.z, w.w, fmaf(d1.y, w.x, d1.x * w.y)));
    const float cur = fmaf(-q.y, w.y, fmaf(q.x, w.x, fmaf(-q.y, c1ui, fmaf(q.x, c1ur, c1ur))));
    const float cui = fmaf(q.y, w.x, fmaf(q.x, w.y, fmaf(q.y, c1ur, fmaf(q.x, c1ui, c1ui))));
    const float cdr = fmaf(-q.y, w.w, fmaf(q.x, w.z, fmaf(-q.y, c1di, fmaf(q.x, c1dr, c1dr))));
    const float cdi = fmaf(q.y, w.z, fmaf(q.x, w.w, fmaf(q.y, c1dr, fmaf(q.x, c1di, c1di))));
    const float4 o = make_float4(w.x + cur, w.y + cui, w.z + cdr, w.w + cdi);
    if constexpr (NORM == NORM_DOT) {
      acc += static_cast<double>(fmaf(w.x, o.x, fmaf(w.y, o.y, fmaf(w.z, o.z, w.w * o.w))));
    } else if constexpr (NORM == NORM_SQ) {
      acc += static_cast<double>(fmaf(o.x, o.x, fmaf(o.y, o.y, fmaf(o.z, o.z, o.w * o.w))));
    }
    v[m] = o;
  }
  if constexpr (NORM != NORM_NONE) {
    const double s = block_sum(acc, red);
    if (tid == 0) a.partials[blockIdx.x] = s;
  }

  fft_pass<N, +1>(v, lds, t, tr);

#pragma unroll
  for (int m = 0; m < 16; ++m) p[size_t(t + T * m) * rs] = v[m];
}

// Launcher
template <int N, int NORM>
static hipError_t col_launch_t(const ColArgs& a, hipStream_t s) {
  const int t = N / 16;
  const dim3 block(a.cols * t);
  const dim3 grid(a.nx / a.cols);
  const size_t lds = col_lds_bytes(N, a.cols);
  hipLaunchKernelGGL((col_kernel<N, NORM>), grid, block, lds, s, a);
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
