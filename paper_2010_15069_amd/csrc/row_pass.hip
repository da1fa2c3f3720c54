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
// Every operator close to the identity is applied as psi + (U - 1) psi with U - 1 held to fp32
// relative accuracy, so that unit-modulus propagators do not pick up a coherent |U| != 1 error
// from rounding their tables.
#include "fft_device.hpp"
#include "sgpe_internal.hpp"

namespace sgpe {
// -------------------------------------------------------------------------------------------
// Sum of the previous column pass's partials -> scale for the row pass.  Every wave computes
// the same sum in the same order, so every workgroup applies bit-identical scales.
// -------------------------------------------------------------------------------------------
__device__ __forceinline__ float row_scale(const RowArgs& a) {
  if (a.partials == nullptr) return a.scale;
  double s = 0.0;
  if (blockDim.x >= 64) {
    const int lane = threadIdx.x & 63;
    for (int i = lane; i < a.n_partials; i += 64) s += a.partials[i];
    s = wave_sum(s);
  } else {
    for (int i = 0; i < a.n_partials; ++i) s += a.partials[i];
  }
  const double norm = a.parseval_w * s;
  return static_cast<float>(sqrt(a.norm0 / norm) * a.inv_npts);
}

// -------------------------------------------------------------------------------------------
// Real-space exponential R(h) at one point (Eqs. (H2)-(H4), densities of the input).
// hv = h V(x, y); hbx = h Omega(x) / 2.
// -------------------------------------------------------------------------------------------
template <bool IMAG, bool FULL>
__device__ __forceinline__ float4 apply_r(float4 w, float hv, float hbx, const RowArgs& a) {
  const float nu = fmaf(w.x, w.x, w.y * w.y);
  const float nd = fmaf(w.z, w.z, w.w * w.w);
  if constexpr (!FULL) {
    const float phu = fmaf(a.hg_uu, nu, fmaf(a.hg_ud, nd, hv + a.hdelta2));
    const float phd = fmaf(a.hg_dd, nd, fmaf(a.hg_ud, nu, hv - a.hdelta2));
    if constexpr (!IMAG) {
      // psi * exp(-i phi) = psi + psi (cm1 - i s); the small correction is formed first and
      // added once (one rounding of the large value per step).
      const SinCosM1 su = sincos_m1(phu);
      const SinCosM1 sd = sincos_m1(phd);
      return make_float4(w.x + fmaf(w.x, su.cm1, w.y * su.s), w.y + fmaf(w.y, su.cm1, -w.x * su.s),
                         w.z + fmaf(w.z, sd.cm1, w.w * sd.s), w.w + fmaf(w.w, sd.cm1, -w.z * sd.s));
    } else {
      const float eu = expf(-phu);
      const float ed = expf(-phd);
      return make_float4(w.x * eu, w.y * eu, w.z * ed, w.w * ed);
    }
  } else {
    // H_R = A 1 + Bx sigma_x + Bz sigma_z (all times h)
    const float gu = fmaf(a.hg_uu, nu, a.hg_ud * nd);
    const float gd = fmaf(a.hg_dd, nd, a.hg_ud * nu);
    const float ha = fmaf(0.5f, gu + gd, hv);
    const float hbz = fmaf(0.5f, gu - gd, a.hdelta2);
    const float th = sqrtf(fmaf(hbx, hbx, hbz * hbz));
    if constexpr (!IMAG) {
      // M = cos(th) 1 - i sin(th)/th (hB . sigma);  psi' = E M psi, E = exp(-i hA)
      const SinCosM1 sb = sincos_m1(th);
      const float px = sb.sinc * hbx, pz = sb.sinc * hbz;
      // X = pz psi_u + px psi_d, Y = px psi_u - pz psi_d; (M - 1) psi = cm1 psi - i (X, Y)
      const float xr = fmaf(pz, w.x, px * w.z), xi = fmaf(pz, w.y, px * w.w);
      const float yr = fmaf(px, w.x, -pz * w.z), yi = fmaf(px, w.y, -pz * w.w);
      const float mur = fmaf(sb.cm1, w.x, xi), mui = fmaf(sb.cm1, w.y, -xr);
      const float mdr = fmaf(sb.cm1, w.z, yi), mdi = fmaf(sb.cm1, w.w, -yr);
      // E M psi - psi = c_M + (E - 1)(psi + c_M), E - 1 = cm1_A - i s_A; added to psi once.
      const SinCosM1 se = sincos_m1(ha);
      const float cur = fmaf(se.s, w.y, fmaf(se.cm1, w.x, fmaf(se.s, mui, fmaf(se.cm1, mur, mur))));
      const float cui = fmaf(-se.s, w.x, fmaf(se.cm1, w.y, fmaf(-se.s, mur, fmaf(se.cm1, mui, mui))));
      const float cdr = fmaf(se.s, w.w, fmaf(se.cm1, w.z, fmaf(se.s, mdi, fmaf(se.cm1, mdr, mdr))));
      const float cdi = fmaf(-se.s, w.z, fmaf(se.cm1, w.w, fmaf(-se.s, mdr, fmaf(se.cm1, mdi, mdi))));
      return make_float4(w.x + cur, w.y + cui, w.z + cdr, w.w + cdi);
    } else {
      const float ea = expf(-ha);
      float ch, shc;  // cosh(th), sinh(th)/th
      if (th < 0.25f) {
        const float t2 = th * th;
        ch = fmaf(t2, fmaf(t2, fmaf(t2, fmaf(t2, 2.48015873e-5f, 1.38888889e-3f), 4.16666667e-2f), 0.5f), 1.0f);
        shc = fmaf(t2, fmaf(t2, fmaf(t2, fmaf(t2, 2.75573192e-6f, 1.98412698e-4f), 8.33333333e-3f),
                             1.66666667e-1f), 1.0f);
      } else {
        const float ep = expf(th);
        const float em = 1.0f / ep;
        ch = 0.5f * (ep + em);
        shc = 0.5f * (ep - em) / th;
      }
      const float m11 = ea * fmaf(-shc, hbz, ch);
      const float m22 = ea * fmaf(shc, hbz, ch);
      const float m12 = -ea * shc * hbx;
      return make_float4(fmaf(m11, w.x, m12 * w.z), fmaf(m11, w.y, m12 * w.w),
                         fmaf(m12, w.x, m22 * w.z), fmaf(m12, w.y, m22 * w.w));
    }
  }
}

// -------------------------------------------------------------------------------------------
// Row pass
// -------------------------------------------------------------------------------------------
template <int N, int MODE, bool IMAG, bool FULL>
__global__ void __launch_bounds__(256) row_kernel(RowArgs a) {
  extern __shared__ float4 lds_raw[];
  constexpr int T = N / 16;
  constexpr int SLOTS = N + N / 16;
  const int tid = threadIdx.x;
  const int rloc = tid / T;
  const int t = tid - rloc * T;
  const int row = blockIdx.x * a.rows_per_block + rloc;
  const LdsView lds{lds_raw + rloc * SLOTS, 1};
  float4* __restrict__ p = a.psi + size_t(row) * N;

  float4 v[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) v[m] = p[t + T * m];
  TwRegs<N> tr;
  load_twiddles<N>(tr, t, a.tw);

  if constexpr (MODE == ROW_FWD) {
    fft_pass<N, -1>(v, lds, t, tr);
  } else {
    const float s = row_scale(a);
    fft_pass<N, +1>(v, lds, t, tr);
#pragma unroll
    for (int m = 0; m < 16; ++m) v[m] = make_float4(v[m].x * s, v[m].y * s, v[m].z * s, v[m].w * s);
    if constexpr (MODE == ROW_STEP) {
      const float y = fmaf(static_cast<float>(row), a.dy, a.y0);
      const float hvy = a.hvy * y * y;
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        const int j = t + T * m;
        const float x = fmaf(static_cast<float>(j), a.dx, a.x0);
        const float hv = fmaf(a.hvx * x, x, hvy);
        const float hbx = FULL ? a.hbx[j] : 0.0f;
        v[m] = apply_r<IMAG, FULL>(v[m], hv, hbx, a);
      }
      fft_pass<N, -1>(v, lds, t, tr);
    }
  }
#pragma unroll
  for (int m = 0; m < 16; ++m) p[t + T * m] = v[m];
}

// Launcher
template <int N, int MODE, bool IMAG, bool FULL>
static hipError_t row_launch_t(const RowArgs& a, hipStream_t s) {
  const int t = N / 16;
  const dim3 block(a.rows_per_block * t);
  const dim3 grid(a.ny / a.rows_per_block);
  const size_t lds = row_lds_bytes(N, a.rows_per_block);
  hipLaunchKernelGGL((row_kernel<N, MODE, IMAG, FULL>), grid, block, lds, s, a);
  return hipGetLastError();
}

template <int N>
static hipError_t row_launch_n(const RowArgs& a, int mode, bool imag, bool full, hipStream_t s) {
  switch (mode) {
    case ROW_FWD: return row_launch_t<N, ROW_FWD, false, false>(a, s);
    case ROW_INV: return row_launch_t<N, ROW_INV, false, false>(a, s);
    case ROW_STEP:
      if (imag) return full ? row_launch_t<N, ROW_STEP, true, true>(a, s) : row_launch_t<N, ROW_STEP, true, false>(a, s);
      return full ? row_launch_t<N, ROW_STEP, false, true>(a, s) : row_launch_t<N, ROW_STEP, false, false>(a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_row(const RowArgs& a, int mode, bool imag, bool full, hipStream_t s) {
  switch (a.nx) {
    case 16: return row_launch_n<16>(a, mode, imag, full, s);
    case 32: return row_launch_n<32>(a, mode, imag, full, s);
    case 64: return row_launch_n<64>(a, mode, imag, full, s);
    case 128: return row_launch_n<128>(a, mode, imag, full, s);
    case 256: return row_launch_n<256>(a, mode, imag, full, s);
    case 512: return row_launch_n<512>(a, mode, imag, full, s);
    case 1024: return row_launch_n<1024>(a, mode, imag, full, s);
    case 2048: return row_launch_n<2048>(a, mode, imag, full, s);
    case 4096: return row_launch_n<4096>(a, mode, imag, full, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sgpe
