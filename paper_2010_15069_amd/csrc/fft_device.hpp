// Device building blocks of the split-step solver: register-resident Stockham FFT passes over
// the two spinor components at once, compensated (hi + lo) twiddle products, and the (U - 1)
// sine/cosine helper used by the unit-modulus real-space propagators.
//
// A grid point is carried as one float4 {re_up, im_up, re_dn, im_dn}; both components share the
// FFT's index arithmetic and twiddles.
//
// FFT organisation (transform length N = 16^a * r, r in {1, 2, 4, 8}): T = N/16 threads own one
// transform, thread t holding the 16 positions t + T*m (m = 0..15).  Each Stockham stage of radix
// R performs 16/R butterflies per thread on registers {u + (16/R) r}; the outputs of every stage
// but the last go through LDS, and the last stage's outputs land back in the thread's own
// registers in natural order.  So the first stage reads and the last stage writes the positions
// t + T*m, which are contiguous across threads: global loads and stores are coalesced and no
// digit reversal pass exists.
//
// Accuracy: fp32 twiddles rounded once are off the unit circle by ~3e-8, and the same error is
// re-applied every step, so it accumulates coherently over thousands of steps.  Every
// non-trivial twiddle -- the stage twiddles from the table and the constants inside the radix-8
// and radix-16 butterflies -- is therefore applied as z*w_hi + z*w_lo with w_hi + w_lo equal to the
// exact root of unity to ~1e-15.
#pragma once

#include <hip/hip_runtime.h>

namespace sgpe {

// ---------------------------------------------------------------------------------------------
// float4 = two complex numbers
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ float4 add4(float4 a, float4 b) {
  return make_float4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w);
}
__device__ __forceinline__ float4 sub4(float4 a, float4 b) {
  return make_float4(a.x - b.x, a.y - b.y, a.z - b.z, a.w - b.w);
}
// Multiply by exp(DIR * i*pi/2) = DIR * i  (DIR = -1: forward transform sign).
template <int DIR>
__device__ __forceinline__ float4 rot90(float4 a) {
  if constexpr (DIR < 0) return make_float4(a.y, -a.x, a.w, -a.z);   // * (-i)
  else return make_float4(-a.y, a.x, -a.w, a.z);                      // * (+i)
}

// z * (c + i*DIR*s) with c = ch + cl and s = sh + sl given as hi/lo pairs.
template <int DIR>
__device__ __forceinline__ float2 cmul_comp(float re, float im, float ch, float cl, float sh, float sl) {
  const float ds_h = DIR < 0 ? -sh : sh;
  const float ds_l = DIR < 0 ? -sl : sl;
  // re = re*c - im*(DIR s), im = re*(DIR s) + im*c; the lo parts go into the innermost term.
  const float lo_r = fmaf(re, cl, -im * ds_l);
  const float lo_i = fmaf(re, ds_l, im * cl);
  const float out_r = fmaf(re, ch, fmaf(-im, ds_h, lo_r));
  const float out_i = fmaf(re, ds_h, fmaf(im, ch, lo_i));
  return make_float2(out_r, out_i);
}

template <int DIR>
__device__ __forceinline__ float4 cmul4_comp(float4 a, float ch, float cl, float sh, float sl) {
  const float2 u = cmul_comp<DIR>(a.x, a.y, ch, cl, sh, sl);
  const float2 d = cmul_comp<DIR>(a.z, a.w, ch, cl, sh, sl);
  return make_float4(u.x, u.y, d.x, d.y);
}

// Multiply by a table twiddle w = exp(-2 pi i j / N) stored as {re_hi, im_hi, re_lo, im_lo};
// the inverse transform (DIR = +1) uses conj(w).
template <int DIR>
__device__ __forceinline__ float4 twmul(float4 a, float4 w) {
  // table holds c - i s  (forward root); cmul_comp<DIR> builds c + i*DIR*s, so pass s = -im.
  return cmul4_comp<DIR>(a, w.x, w.z, -w.y, -w.w);
}

// Compensated split constants (value = hi + lo to fp64 accuracy).
// 1/sqrt(2)
#define SGPE_R2_HI 0.70710676908493042f
#define SGPE_R2_LO 1.21016175e-08f
// cos(pi/8), sin(pi/8)
#define SGPE_C8_HI 0.92387950420379639f
#define SGPE_C8_LO 2.83074897e-08f
#define SGPE_S8_HI 0.38268342614173889f
#define SGPE_S8_LO 6.22335072e-09f

// exp(DIR*i*pi/4) * z: (1 + DIR i)/sqrt(2) * z
template <int DIR>
__device__ __forceinline__ float4 rot45(float4 a) {
  float4 s;
  if constexpr (DIR < 0) {  // (1 - i)(x + iy) = (x + y) + i(y - x)
    s = make_float4(a.x + a.y, a.y - a.x, a.z + a.w, a.w - a.z);
  } else {                  // (1 + i)(x + iy) = (x - y) + i(x + y)
    s = make_float4(a.x - a.y, a.x + a.y, a.z - a.w, a.z + a.w);
  }
  return make_float4(fmaf(s.x, SGPE_R2_HI, s.x * SGPE_R2_LO), fmaf(s.y, SGPE_R2_HI, s.y * SGPE_R2_LO),
                     fmaf(s.z, SGPE_R2_HI, s.z * SGPE_R2_LO), fmaf(s.w, SGPE_R2_HI, s.w * SGPE_R2_LO));
}

// ---------------------------------------------------------------------------------------------
// Small DFTs in registers, natural order in and out: y_k = sum_r x_r exp(DIR 2 pi i r k / R).
// ---------------------------------------------------------------------------------------------
template <int DIR>
__device__ __forceinline__ void dft2(float4& a0, float4& a1) {
  const float4 t = a0;
  a0 = add4(t, a1);
  a1 = sub4(t, a1);
}

template <int DIR>
__device__ __forceinline__ void dft4(float4& a0, float4& a1, float4& a2, float4& a3) {
  const float4 t0 = add4(a0, a2), t1 = sub4(a0, a2);
  const float4 t2 = add4(a1, a3), t3 = rot90<DIR>(sub4(a1, a3));
  a0 = add4(t0, t2);
  a2 = sub4(t0, t2);
  a1 = add4(t1, t3);
  a3 = sub4(t1, t3);
}

template <int DIR>
__device__ __forceinline__ void dft8(float4 (&a)[8]) {
  float4 e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
  float4 o0 = a[1], o1 = a[3], o2 = a[5], o3 = a[7];
  dft4<DIR>(e0, e1, e2, e3);
  dft4<DIR>(o0, o1, o2, o3);
  o1 = rot45<DIR>(o1);
  o2 = rot90<DIR>(o2);
  o3 = rot90<DIR>(rot45<DIR>(o3));
  a[0] = add4(e0, o0); a[4] = sub4(e0, o0);
  a[1] = add4(e1, o1); a[5] = sub4(e1, o1);
  a[2] = add4(e2, o2); a[6] = sub4(e2, o2);
  a[3] = add4(e3, o3); a[7] = sub4(e3, o3);
}

// 16-point DFT as 4x4: x index r = r1 + 4 r2, output k = k2 + 4 k1.
template <int DIR>
__device__ __forceinline__ void dft16(float4 (&a)[16]) {
#pragma unroll
  for (int r1 = 0; r1 < 4; ++r1) dft4<DIR>(a[r1], a[r1 + 4], a[r1 + 8], a[r1 + 12]);
  // slot r1 + 4 k2 holds A[r1][k2]; multiply by W16^(r1 k2).
  // W16^1 = c8 + i DIR s8; W16^2 = rot45; W16^3 = s8 + i DIR c8; W16^4 = rot90;
  // W16^6 = rot90*rot45; W16^9 = -W16^1.
  a[5] = cmul4_comp<DIR>(a[5], SGPE_C8_HI, SGPE_C8_LO, SGPE_S8_HI, SGPE_S8_LO);    // (1,1): 1
  a[9] = rot45<DIR>(a[9]);                                                          // (1,2): 2
  a[13] = cmul4_comp<DIR>(a[13], SGPE_S8_HI, SGPE_S8_LO, SGPE_C8_HI, SGPE_C8_LO);  // (1,3): 3
  a[6] = rot45<DIR>(a[6]);                                                          // (2,1): 2
  a[10] = rot90<DIR>(a[10]);                                                        // (2,2): 4
  a[14] = rot90<DIR>(rot45<DIR>(a[14]));                                            // (2,3): 6
  a[7] = cmul4_comp<DIR>(a[7], SGPE_S8_HI, SGPE_S8_LO, SGPE_C8_HI, SGPE_C8_LO);    // (3,1): 3
  a[11] = rot90<DIR>(rot45<DIR>(a[11]));                                            // (3,2): 6
  {                                                                                 // (3,3): 9
    const float4 t = cmul4_comp<DIR>(a[15], SGPE_C8_HI, SGPE_C8_LO, SGPE_S8_HI, SGPE_S8_LO);
    a[15] = make_float4(-t.x, -t.y, -t.z, -t.w);
  }
#pragma unroll
  for (int k2 = 0; k2 < 4; ++k2) dft4<DIR>(a[4 * k2], a[4 * k2 + 1], a[4 * k2 + 2], a[4 * k2 + 3]);
  // slot k1 + 4 k2 now holds y[k2 + 4 k1]: transpose the 4x4 register tile.
  float4 t[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) t[i] = a[i];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) a[k2 + 4 * k1] = t[k1 + 4 * k2];
}

template <int R, int DIR>
__device__ __forceinline__ void dft(float4 (&a)[R]) {
  if constexpr (R == 2) {
    dft2<DIR>(a[0], a[1]);
  } else if constexpr (R == 4) {
    dft4<DIR>(a[0], a[1], a[2], a[3]);
  } else if constexpr (R == 8) {
    dft8<DIR>(a);
  } else {
    static_assert(R == 16, "radix");
    dft16<DIR>(a);
  }
}

// ---------------------------------------------------------------------------------------------
// LDS addressing: a transform's N points occupy N + N/16 float4 slots (one pad slot per 16) and
// C transforms are interleaved slot by slot (column pass: lanes of consecutive columns hit
// consecutive float4s).
// ---------------------------------------------------------------------------------------------
struct LdsView {
  float4* base;  // slot 0 of transform c
  int stride;    // C
  __device__ __forceinline__ float4& at(int pos) const { return base[(pos + (pos >> 4)) * stride]; }
};

// Stage twiddles a thread needs for a length-N transform: the first stage (L = 1) needs none;
// a later stage of radix R uses W_N^(s r N/(R L)) for its 16/R butterflies and r = 1..R-1.
template <int N, int L = 1>
constexpr int tw_count() {
  constexpr int REM = N / L;
  constexpr int R = REM >= 16 ? 16 : REM;
  constexpr int here = L > 1 ? (16 / R) * (R - 1) : 0;
  if constexpr (R == REM) return here;
  else return here + tw_count<N, L * R>();
}

// Per-thread register copy of those twiddles, loaded once per kernel (they depend only on the
// thread index) and shared by the forward and inverse transforms (the inverse conjugates).
template <int N>
struct TwRegs {
  static constexpr int COUNT = tw_count<N>() > 0 ? tw_count<N>() : 1;
  float4 w[COUNT];
};

template <int N, int L = 1, int BASE = 0>
__device__ __forceinline__ void load_twiddles(TwRegs<N>& tr, int t, const float4* __restrict__ tw) {
  constexpr int T = N / 16;
  constexpr int REM = N / L;
  constexpr int R = REM >= 16 ? 16 : REM;
  constexpr int U = 16 / R;
  constexpr int TW_STRIDE = N / (R * L);
  if constexpr (L > 1) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int s = (t + T * u) & (L - 1);
#pragma unroll
      for (int r = 1; r < R; ++r) tr.w[BASE + u * (R - 1) + (r - 1)] = tw[s * r * TW_STRIDE];
    }
  }
  if constexpr (R != REM) {
    constexpr int NEXT = BASE + (L > 1 ? U * (R - 1) : 0);
    load_twiddles<N, L * R, NEXT>(tr, t, tw);
  }
}

// One Stockham stage: radix R, L = product of the radices already applied; its twiddles start at
// tr.w[BASE].
template <int N, int R, int L, int DIR, bool LAST, int BASE>
__device__ __forceinline__ void stockham_stage(float4 (&v)[16], const LdsView& lds, int t,
                                               const TwRegs<N>& tr) {
  constexpr int T = N / 16;
  constexpr int U = 16 / R;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    float4 a[R];
#pragma unroll
    for (int r = 0; r < R; ++r) a[r] = v[u + U * r];
    const int b = t + T * u;
    const int s = b & (L - 1);
    if constexpr (L > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) a[r] = twmul<DIR>(a[r], tr.w[BASE + u * (R - 1) + (r - 1)]);
    }
    dft<R, DIR>(a);
    if constexpr (LAST) {
#pragma unroll
      for (int k = 0; k < R; ++k) v[u + U * k] = a[k];
    } else {
      const int q = b / L;
#pragma unroll
      for (int k = 0; k < R; ++k) lds.at(q * R * L + s + L * k) = a[k];
    }
  }
}

// Full length-N transform of the 16 registers (positions t + T*m) in place.  All threads of the
// workgroup call it (it contains workgroup barriers).
template <int N, int DIR, int L = 1, int BASE = 0>
__device__ __forceinline__ void fft_pass(float4 (&v)[16], const LdsView& lds, int t, const TwRegs<N>& tr) {
  constexpr int REM = N / L;
  constexpr int R = REM >= 16 ? 16 : REM;
  constexpr bool LAST = (R == REM);
  constexpr int T = N / 16;
  stockham_stage<N, R, L, DIR, LAST, BASE>(v, lds, t, tr);
  if constexpr (!LAST) {
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 16; ++m) v[m] = lds.at(t + T * m);
    __syncthreads();
    constexpr int NEXT = BASE + (L > 1 ? (16 / R) * (R - 1) : 0);
    fft_pass<N, DIR, L * R, NEXT>(v, lds, t, tr);
  }
}

// ---------------------------------------------------------------------------------------------
// (cos(phi) - 1, sin(phi)) with relative accuracy on both parts for small |phi|.
// Cody-Waite reduction by pi/2 (the first product is exact inside the FMA for |k| < 2^10),
// Taylor polynomials on |r| <= pi/4.  Also returns sin(phi)/phi (1 at phi = 0).
// ---------------------------------------------------------------------------------------------
struct SinCosM1 {
  float cm1, s, sinc;
};

__device__ __forceinline__ SinCosM1 sincos_m1_reduced(float phi) {
  const float k = rintf(phi * 0.636619772367581343f);
  float r = fmaf(-k, 1.57079637050628662f, phi);   // pi/2 hi
  r = fmaf(-k, -4.37113900018624283e-8f, r);        // pi/2 lo
  const float r2 = r * r;
  const float ps = r2 * fmaf(r2, fmaf(r2, fmaf(r2, 2.75573192e-6f, -1.98412698e-4f), 8.33333333e-3f),
                             -1.66666667e-1f);   // sin r / r - 1
  const float sr = fmaf(r, ps, r);
  const float cr_m1 = r2 * fmaf(r2, fmaf(r2, fmaf(r2, fmaf(r2, -2.75573192e-7f, 2.48015873e-5f),
                                                  -1.38888889e-3f), 4.16666667e-2f), -0.5f);
  const int q = static_cast<int>(k) & 3;
  SinCosM1 out;
  if (q == 0) {
    out.cm1 = cr_m1;
    out.s = sr;
    out.sinc = 1.0f + ps;
  } else {
    const float cr = cr_m1 + 1.0f;
    const float c = q == 1 ? -sr : (q == 2 ? -cr : sr);
    out.s = q == 1 ? cr : (q == 2 ? -sr : -cr);
    out.cm1 = c - 1.0f;
    out.sinc = out.s / phi;
  }
  return out;
}

// |phi| <= pi/4 needs no reduction; the polynomials alone are accurate there.
__device__ __forceinline__ SinCosM1 sincos_m1_small(float phi) {
  const float r2 = phi * phi;
  const float ps = r2 * fmaf(r2, fmaf(r2, fmaf(r2, 2.75573192e-6f, -1.98412698e-4f), 8.33333333e-3f),
                             -1.66666667e-1f);
  SinCosM1 out;
  out.s = fmaf(phi, ps, phi);
  out.cm1 = r2 * fmaf(r2, fmaf(r2, fmaf(r2, fmaf(r2, -2.75573192e-7f, 2.48015873e-5f),
                                             -1.38888889e-3f), 4.16666667e-2f), -0.5f);
  out.sinc = 1.0f + ps;
  return out;
}

__device__ __forceinline__ SinCosM1 sincos_m1(float phi) {
  // The branch is uniform in the common case (every phase of the wave below pi/4).
  if (fabsf(phi) <= 0.785398163f) return sincos_m1_small(phi);
  return sincos_m1_reduced(phi);
}

// ---------------------------------------------------------------------------------------------
// Deterministic reductions in fp64.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the workgroup; every thread must call it; red must hold >= blockDim.x/64 doubles.
// Result valid in every thread.
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < nw; ++w) s += red[w];
  __syncthreads();
  return s;
}

}  // namespace sgpe
