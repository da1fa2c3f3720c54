// Device building blocks of the split-step solver's step kernels: register-resident Stockham FFT
// passes, the (U - 1) sine/cosine helpers of the unit-modulus real-space propagators, lane-pair
// exchange and fp64 reductions.
//
// FFT organisation (transform length N, P points per lane, P in {4, 8, 16}): T = N/P lanes own one
// transform, lane t holding the P positions t + T*m (m = 0..P-1); in the step kernels each lane
// owns one spinor component and the neighbouring lane the other component of the same positions.
// Each Stockham stage of radix R (P, then a smaller remainder) performs P/R butterflies per lane on
// registers; the outputs of every stage but the last go through LDS, and the last stage's outputs
// land back in the lane's own registers in natural order.  So the first stage reads and the last
// stage writes the positions t + T*m, which are contiguous across lanes: global loads and stores
// are coalesced and no digit-reversal pass exists.  Roots are rounded once to fp32; the inverse
// transform is the exact inverse of the forward one (see "Step-kernel transforms" below).
#pragma once

#include <hip/hip_runtime.h>

#include "sgpe_internal.hpp"

namespace sgpe {

// ---------------------------------------------------------------------------------------------
// Complex arithmetic on float2 (one complex) and float4 (two complexes sharing the operation).
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ float2 vadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 vsub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 vneg(float2 a) { return make_float2(-a.x, -a.y); }
__device__ __forceinline__ float2 vscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float4 vadd(float4 a, float4 b) {
  return make_float4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w);
}
__device__ __forceinline__ float4 vsub(float4 a, float4 b) {
  return make_float4(a.x - b.x, a.y - b.y, a.z - b.z, a.w - b.w);
}
__device__ __forceinline__ float4 vneg(float4 a) { return make_float4(-a.x, -a.y, -a.z, -a.w); }
__device__ __forceinline__ float4 vscale(float4 a, float s) {
  return make_float4(a.x * s, a.y * s, a.z * s, a.w * s);
}
__device__ __forceinline__ double2 vadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 vsub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 vneg(double2 a) { return make_double2(-a.x, -a.y); }
__device__ __forceinline__ double2 vscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }

// The real type of a complex type (the complex types of a precision are in sgpe_internal.hpp).
template <class C> struct RealOf;
template <> struct RealOf<float2> { using T = float; };
template <> struct RealOf<double2> { using T = double; };
__device__ __forceinline__ float2 mk2(float x, float y) { return make_float2(x, y); }
__device__ __forceinline__ double2 mk2(double x, double y) { return make_double2(x, y); }
// fp32 intrinsics for float (the complex64 code is unchanged by the templating), fp64 for double
__device__ __forceinline__ float fma_(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float exp_(float x) { return expf(x); }
__device__ __forceinline__ double exp_(double x) { return exp(x); }
__device__ __forceinline__ float sqrt_(float x) { return sqrtf(x); }
__device__ __forceinline__ double sqrt_(double x) { return sqrt(x); }
__device__ __forceinline__ float fabs_(float x) { return fabsf(x); }
__device__ __forceinline__ double fabs_(double x) { return fabs(x); }

// ---------------------------------------------------------------------------------------------
// State stores of the step kernels.  Consecutive passes split the grid between workgroups by
// rows, then by columns, so almost every point a pass writes is next read on another XCD, whose
// L2 it must leave first.  A plain store parks the line dirty in the writer's L2, and the end of
// the kernel writes back every XCD's dirty lines in one burst that the next kernel then waits
// for.  A device-scope store goes through the L2 to the memory side as it is issued, so that
// traffic overlaps the rest of the pass.  Relaxed order: the scope is the only property wanted
// (every point has a single writer in a pass, and kernel boundaries order the passes).
// Measured per launch kind: write-through wins for single-instance complex64 passes (one round
// of workgroups, nothing behind the last stores); batched launches, whose later workgroups
// already overlap the write-back, and complex128 points (two 8-byte device-scope stores per
// 16-byte component) are faster with plain stores.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ void store_through(float2* p, float2 v) {
  unsigned long long b;
  __builtin_memcpy(&b, &v, sizeof b);
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <bool WT, class C>
__device__ __forceinline__ void store_state(C* p, C v) {
  if constexpr (WT && sizeof(C) == sizeof(float2)) {
    store_through(p, v);
  } else {
    *p = v;
  }
}

// ---------------------------------------------------------------------------------------------
// Batched launches (grid x = work items of one instance, grid y = instances).  The dispatcher
// deals a launch's workgroups to the eight XCDs in turn, by linear workgroup index (x fastest),
// continuing its rotation from where the previous launch left it.  Reading the grid as
// instance-major (instance, item) pairs and giving the workgroups L = k mod 8 the k-th eighth of
// that sequence keeps all of an instance's items on one XCD within a launch; when consecutive
// launches start the rotation at the same XCD (every launch of a batch has a multiple of 8
// workgroups), a pass also reads what the previous pass wrote into the same L2.  The map is a
// bijection whenever the grid holds a multiple of 8 workgroups (the identity otherwise); results do
// not depend on where a workgroup runs.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ int2 batch_item() {
  const unsigned gx = gridDim.x, total = gx * gridDim.y;
  unsigned l = blockIdx.y * gx + blockIdx.x;
  if ((total & 7u) == 0) l = (l & 7u) * (total >> 3) + (l >> 3);
  return make_int2(int(l / gx), int(l % gx));   // (instance, item)
}

// ---------------------------------------------------------------------------------------------
// LDS addressing: a transform's N positions occupy N + N/16 slots (one pad slot per 16
// positions) and `stride` transforms are interleaved slot by slot, so that lanes which own
// neighbouring transforms touch neighbouring slots.
// ---------------------------------------------------------------------------------------------
template <class V>
struct LdsView {
  V* base;     // slot 0 of this thread's transform
  int shift;   // log2 of the number of interleaved transforms (a power of two)
  __device__ __forceinline__ V& at(int pos) const { return base[(pos + (pos >> 4)) << shift]; }
};

// ---------------------------------------------------------------------------------------------
// Step-kernel transforms: a forward transform with roots rounded once to fp32, and its exact
// inverse.
//
// A forward transform with fp32-rounded roots w~ is a slightly perturbed DFT.  Followed by the
// textbook inverse (conjugate roots), the round trip is not the identity: |w~| != 1 scales every
// butterfly path and that same map is re-applied every step (a coherent drift).  Here the inverse
// instead undoes the forward stage by stage in reverse order: each small DFT by its conjugate
// structure and each rounded root by v = conj(w~) / |w~|^2.  v is held as conj(w~) plus a low part
// conj(w~) eta (eta = 1/|w~|^2 - 1, about 1e-8) that enters the fma chain of the product before
// the large terms, so every result is rounded once from the exact product.  (Scaling a rounded
// product by 1 + eta afterwards does not work: eta is below half an ulp and the rounding drops
// it, the same way every step.)  The pair is then an exact inverse in exact arithmetic, the round
// trip carries only unbiased rounding, and the rounded roots enter the split step only through
// commutators with the step's operators, O(dt eps) per step.  The forward costs 4 instructions
// per complex product instead of 8 for a compensated one; the inverse costs 8.
// ---------------------------------------------------------------------------------------------
// Butterfly constants.  fp32: the rounded 1/sqrt(2), cos(pi/8), sin(pi/8) and the low parts that
// make the inverse exact.  fp64: the rounded constants; their modulus error (~1e-16) is left in
// place -- applied every step it drifts by ~1e-10 over 10^6 steps -- so the low parts are zero.
template <class T> struct Roots;
template <> struct Roots<float> {
  static constexpr float R2 = 0.70710676908493042f;      // fp32(1/sqrt(2))
  static constexpr float R2_LO = 2.42032350e-08f;        // r2 (1/(2 r2^2) - 1) for the fp32 r2
  static constexpr float C8 = 0.92387950420379639f;      // fp32(cos(pi/8))
  static constexpr float S8 = 0.38268342614173889f;      // fp32(sin(pi/8))
  static constexpr float C8_LO = 5.27244843e-08f;        // c8 eta8, eta8 = 1/(c8^2 + s8^2) - 1
  static constexpr float S8_LO = 2.18391971e-08f;        // s8 eta8
};
template <> struct Roots<double> {
  static constexpr double R2 = 0.70710678118654752440;
  static constexpr double R2_LO = 0.0;
  static constexpr double C8 = 0.92387953251128675613;
  static constexpr double S8 = 0.38268343236508977173;
  static constexpr double C8_LO = 0.0;
  static constexpr double S8_LO = 0.0;
};

template <class C>
__device__ __forceinline__ C pf_rot90(C a) { return mk2(a.y, -a.x); }   // * (-i)
template <class C>
__device__ __forceinline__ C pi_rot90(C a) { return mk2(-a.y, a.x); }   // * (+i)
// * r2 (1 - i) and its exact inverse * (1 + i) / (2 r2)
template <class C>
__device__ __forceinline__ C pf_rot45(C a) {
  using K = Roots<typename RealOf<C>::T>;
  return mk2(K::R2 * (a.x + a.y), K::R2 * (a.y - a.x));
}
template <class C>
__device__ __forceinline__ C pi_rot45(C a) {
  using K = Roots<typename RealOf<C>::T>;
  const auto d = a.x - a.y, e = a.x + a.y;
  return mk2(fma_(d, K::R2, d * K::R2_LO), fma_(e, K::R2, e * K::R2_LO));
}
// * (c - i s) and its exact inverse * ((c + lx) + i (s + ly)), (lx, ly) = (c, s) eta
template <class C, class T = typename RealOf<C>::T>
__device__ __forceinline__ C pf_cmul(C a, T c, T s) {
  return mk2(fma_(a.x, c, a.y * s), fma_(a.y, c, -a.x * s));
}
template <class C, class T = typename RealOf<C>::T>
__device__ __forceinline__ C pi_cmul(C a, T c, T s, T lx, T ly) {
  return mk2(fma_(a.x, c, fma_(-a.y, s, fma_(a.x, lx, -a.y * ly))),
             fma_(a.y, c, fma_(a.x, s, fma_(a.y, lx, a.x * ly))));
}

// forward small DFTs (sign -1)
template <class C>
__device__ __forceinline__ void pf_dft4(C& a0, C& a1, C& a2, C& a3) {
  const C t0 = vadd(a0, a2), t1 = vsub(a0, a2);
  const C t2 = vadd(a1, a3), t3 = pf_rot90(vsub(a1, a3));
  a0 = vadd(t0, t2);
  a2 = vsub(t0, t2);
  a1 = vadd(t1, t3);
  a3 = vsub(t1, t3);
}
// its exact inverse times 4 (conjugate structure; the constants are exact)
template <class C>
__device__ __forceinline__ void pi_dft4(C& a0, C& a1, C& a2, C& a3) {
  const C t0 = vadd(a0, a2), t1 = vsub(a0, a2);
  const C t2 = vadd(a1, a3), t3 = pi_rot90(vsub(a1, a3));
  a0 = vadd(t0, t2);
  a2 = vsub(t0, t2);
  a1 = vadd(t1, t3);
  a3 = vsub(t1, t3);
}

template <class C>
__device__ __forceinline__ void pf_dft8(C (&a)[8]) {
  C e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
  C o0 = a[1], o1 = a[3], o2 = a[5], o3 = a[7];
  pf_dft4(e0, e1, e2, e3);
  pf_dft4(o0, o1, o2, o3);
  o1 = pf_rot45(o1);
  o2 = pf_rot90(o2);
  o3 = pf_rot90(pf_rot45(o3));
  a[0] = vadd(e0, o0); a[4] = vsub(e0, o0);
  a[1] = vadd(e1, o1); a[5] = vsub(e1, o1);
  a[2] = vadd(e2, o2); a[6] = vsub(e2, o2);
  a[3] = vadd(e3, o3); a[7] = vsub(e3, o3);
}
// exact inverse of pf_dft8, times 8
template <class C>
__device__ __forceinline__ void pi_dft8(C (&a)[8]) {
  C e0 = vadd(a[0], a[4]), o0 = vsub(a[0], a[4]);
  C e1 = vadd(a[1], a[5]), o1 = vsub(a[1], a[5]);
  C e2 = vadd(a[2], a[6]), o2 = vsub(a[2], a[6]);
  C e3 = vadd(a[3], a[7]), o3 = vsub(a[3], a[7]);
  o1 = pi_rot45(o1);
  o2 = pi_rot90(o2);
  o3 = pi_rot45(pi_rot90(o3));
  pi_dft4(e0, e1, e2, e3);
  pi_dft4(o0, o1, o2, o3);
  a[0] = e0; a[2] = e1; a[4] = e2; a[6] = e3;
  a[1] = o0; a[3] = o1; a[5] = o2; a[7] = o3;
}

// forward 16-point DFT (4x4; input r = r1 + 4 r2, output k = k2 + 4 k1)
template <class C>
__device__ __forceinline__ void pf_dft16(C (&a)[16]) {
  using K = Roots<typename RealOf<C>::T>;
#pragma unroll
  for (int r1 = 0; r1 < 4; ++r1) pf_dft4(a[r1], a[r1 + 4], a[r1 + 8], a[r1 + 12]);
  a[5] = pf_cmul(a[5], K::C8, K::S8);                    // W16^1
  a[9] = pf_rot45(a[9]);                                 // W16^2
  a[13] = pf_cmul(a[13], K::S8, K::C8);                  // W16^3
  a[6] = pf_rot45(a[6]);                                 // W16^2
  a[10] = pf_rot90(a[10]);                               // W16^4
  a[14] = pf_rot90(pf_rot45(a[14]));                     // W16^6
  a[7] = pf_cmul(a[7], K::S8, K::C8);                    // W16^3
  a[11] = pf_rot90(pf_rot45(a[11]));                     // W16^6
  a[15] = vneg(pf_cmul(a[15], K::C8, K::S8));            // W16^9 = -W16^1
#pragma unroll
  for (int k2 = 0; k2 < 4; ++k2) pf_dft4(a[4 * k2], a[4 * k2 + 1], a[4 * k2 + 2], a[4 * k2 + 3]);
  C t[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) t[i] = a[i];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) a[k2 + 4 * k1] = t[k1 + 4 * k2];
}
// exact inverse of pf_dft16, times 16: the same steps undone in reverse order
template <class C>
__device__ __forceinline__ void pi_dft16(C (&a)[16]) {
  using K = Roots<typename RealOf<C>::T>;
  C t[16];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) t[k1 + 4 * k2] = a[k2 + 4 * k1];
#pragma unroll
  for (int k2 = 0; k2 < 4; ++k2) pi_dft4(t[4 * k2], t[4 * k2 + 1], t[4 * k2 + 2], t[4 * k2 + 3]);
  t[5] = pi_cmul(t[5], K::C8, K::S8, K::C8_LO, K::S8_LO);
  t[9] = pi_rot45(t[9]);
  t[13] = pi_cmul(t[13], K::S8, K::C8, K::S8_LO, K::C8_LO);
  t[6] = pi_rot45(t[6]);
  t[10] = pi_rot90(t[10]);
  t[14] = pi_rot45(pi_rot90(t[14]));
  t[7] = pi_cmul(t[7], K::S8, K::C8, K::S8_LO, K::C8_LO);
  t[11] = pi_rot45(pi_rot90(t[11]));
  t[15] = vneg(pi_cmul(t[15], K::C8, K::S8, K::C8_LO, K::S8_LO));
#pragma unroll
  for (int r1 = 0; r1 < 4; ++r1) pi_dft4(t[r1], t[r1 + 4], t[r1 + 8], t[r1 + 12]);
#pragma unroll
  for (int i = 0; i < 16; ++i) a[i] = t[i];
}

template <int R, class C>
__device__ __forceinline__ void pf_dft(C (&a)[R]) {
  if constexpr (R == 2) {
    const C t = a[0];
    a[0] = vadd(t, a[1]);
    a[1] = vsub(t, a[1]);
  } else if constexpr (R == 4) {
    pf_dft4(a[0], a[1], a[2], a[3]);
  } else if constexpr (R == 8) {
    pf_dft8(a);
  } else {
    static_assert(R == 16, "radix");
    pf_dft16(a);
  }
}
template <int R, class C>
__device__ __forceinline__ void pi_dft(C (&a)[R]) {
  if constexpr (R == 2) {
    const C t = a[0];
    a[0] = vadd(t, a[1]);
    a[1] = vsub(t, a[1]);
  } else if constexpr (R == 4) {
    pi_dft4(a[0], a[1], a[2], a[3]);
  } else if constexpr (R == 8) {
    pi_dft8(a);
  } else {
    static_assert(R == 16, "radix");
    pi_dft16(a);
  }
}

// Step-kernel transforms with P points per thread (P = 4, 8 or 16; T = N / P threads per
// transform, thread t holding positions t + T m).  Stages have radix P, then the remainder.

// Stage roots a thread needs: the first stage (L = 1) needs none; a later stage of radix R uses
// W_N^(s r N/(R L)) for its P/R butterflies and r = 1..R-1.
template <int N, int P, int L = 1>
constexpr int tw_count_p() {
  constexpr int REM = N / L;
  constexpr int R = REM >= P ? P : REM;
  constexpr int here = L > 1 ? (P / R) * (R - 1) : 0;
  if constexpr (R == REM) return here;
  else return here + tw_count_p<N, P, L * R>();
}

// Radix of the last stage of a length-N transform with P points per thread (radix-P stages,
// then the remainder).
template <int N, int P, int L = 1>
constexpr int last_radix() {
  constexpr int REM = N / L;
  if constexpr (REM <= P) return REM;
  else return last_radix<N, P, L * P>();
}

// Per-thread stage roots for the step kernels: fp32 (cos, sin) of each root and eta, where
// 1 + eta = 1/|root|^2 of the rounded pair; the inverse forms its low part (cos, sin) eta with two
// products at use (its rounding, ~1e-15, lies far below the fp32 rounding it feeds).  Table
// entries are float4 {cos, sin, eta, 0} of exp(-2 pi i j / N).  Loaded once per kernel (they
// depend only on the thread index); three registers per root.
// fp64 roots carry no modulus correction (their |w~| - 1 is ~1e-16; see Roots<double>), so the fp64
// instantiation holds no eta and its inverse multiplies by conj(w~) alone: 2 registers per root
// fewer, and the 4-instruction product instead of the corrected one.
template <int N, int P = 16, class T = float>
struct TwPlain {
  static constexpr int COUNT = tw_count_p<N, P>() > 0 ? tw_count_p<N, P>() : 1;
  static constexpr bool CORRECTED = sizeof(T) == 4;
  cplx_t<T> cs[COUNT];
  T eta[CORRECTED ? COUNT : 1];
};

template <int N, int P, int L = 1, int BASE = 0, class TR>
__device__ __forceinline__ void load_twiddles(TwPlain<N, P, TR>& tr, int t, const typename Cplx<TR>::Q* __restrict__ tw) {
  using Q = typename Cplx<TR>::Q;
  constexpr int T = N / P;
  constexpr int REM = N / L;
  constexpr int R = REM >= P ? P : REM;
  constexpr int U = P / R;
  constexpr int TW_STRIDE = N / (R * L);
  if constexpr (L > 1) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      // byte offset of root s r TW_STRIDE, 32-bit from the uniform table base
      const uint32_t o = static_cast<uint32_t>((t + T * u) & (L - 1)) * (uint32_t(sizeof(Q)) * TW_STRIDE);
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const Q w = *reinterpret_cast<const Q*>(reinterpret_cast<const char*>(tw) + o * r);
        tr.cs[BASE + u * (R - 1) + (r - 1)] = mk2(w.x, w.y);
        if constexpr (TwPlain<N, P, TR>::CORRECTED) tr.eta[BASE + u * (R - 1) + (r - 1)] = w.z;
      }
    }
  }
  if constexpr (R != REM) {
    constexpr int NEXT = BASE + (L > 1 ? U * (R - 1) : 0);
    load_twiddles<N, P, L * R, NEXT>(tr, t, tw);
  }
}

// forward stage (plain roots)
template <int N, int P, int R, int L, bool LAST, int BASE, class C, class TR>
__device__ __forceinline__ void pf_stage(C (&v)[P], const LdsView<C>& lds, int t, const TwPlain<N, P, TR>& tr) {
  constexpr int T = N / P;
  constexpr int U = P / R;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    C a[R];
#pragma unroll
    for (int r = 0; r < R; ++r) a[r] = v[u + U * r];
    const int b = t + T * u;
    const int s = b & (L - 1);
    if constexpr (L > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const C w = tr.cs[BASE + u * (R - 1) + (r - 1)];
        a[r] = pf_cmul(a[r], w.x, w.y);
      }
    }
    pf_dft<R>(a);
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

// Forward length-N transform (positions t + T*m in and out), plain roots.
template <int N, int L = 1, int BASE = 0, int P, class C, class TR>
__device__ __forceinline__ void fwd_pass(C (&v)[P], const LdsView<C>& lds, int t, const TwPlain<N, P, TR>& tr) {
  constexpr int REM = N / L;
  constexpr int R = REM >= P ? P : REM;
  constexpr bool LAST = (R == REM);
  constexpr int T = N / P;
  pf_stage<N, P, R, L, LAST, BASE>(v, lds, t, tr);
  if constexpr (!LAST) {
    __syncthreads();
#pragma unroll
    for (int m = 0; m < P; ++m) v[m] = lds.at(t + T * m);
    __syncthreads();
    constexpr int NEXT = BASE + (L > 1 ? (P / R) * (R - 1) : 0);
    fwd_pass<N, L * R, NEXT>(v, lds, t, tr);
  }
}

// Inverse stage: the forward stage's outputs (from LDS, or the registers for the last stage)
// through the exact inverse butterfly and inverse roots, into registers {u + U r}.
template <int N, int P, int R, int L, bool LAST, int BASE, class C, class TR>
__device__ __forceinline__ void pi_stage(C (&v)[P], const LdsView<C>& lds, int t, const TwPlain<N, P, TR>& tr) {
  constexpr int T = N / P;
  constexpr int U = P / R;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    C a[R];
    const int b = t + T * u;
    const int s = b & (L - 1);
    if constexpr (LAST) {
#pragma unroll
      for (int k = 0; k < R; ++k) a[k] = v[u + U * k];
    } else {
      const int q = b / L;
#pragma unroll
      for (int k = 0; k < R; ++k) a[k] = lds.at(q * R * L + s + L * k);
    }
    pi_dft<R>(a);
    if constexpr (L > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const C w = tr.cs[BASE + u * (R - 1) + (r - 1)];
        if constexpr (TwPlain<N, P, TR>::CORRECTED) {
          const TR eta = tr.eta[BASE + u * (R - 1) + (r - 1)];
          a[r] = pi_cmul(a[r], w.x, w.y, w.x * eta, w.y * eta);
        } else {
          a[r] = mk2(fma_(a[r].x, w.x, -a[r].y * w.y), fma_(a[r].y, w.x, a[r].x * w.y));   // * conj(w~)
        }
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) v[u + U * r] = a[r];
  }
}

// Exact inverse of fwd_pass, times N: the stages undone in reverse order.  All threads of the
// workgroup call it; on return every LDS read is complete.
template <int N, int L = 1, int BASE = 0, int P, class C, class TR>
__device__ __forceinline__ void inv_pass(C (&v)[P], const LdsView<C>& lds, int t, const TwPlain<N, P, TR>& tr) {
  constexpr int REM = N / L;
  constexpr int R = REM >= P ? P : REM;
  constexpr bool LAST = (R == REM);
  constexpr int T = N / P;
  if constexpr (LAST) {
    pi_stage<N, P, R, L, true, BASE>(v, lds, t, tr);
  } else {
    constexpr int NEXT = BASE + (L > 1 ? (P / R) * (R - 1) : 0);
    inv_pass<N, L * R, NEXT>(v, lds, t, tr);
    // undo "read positions t + T m from LDS", then this stage
#pragma unroll
    for (int m = 0; m < P; ++m) lds.at(t + T * m) = v[m];
    __syncthreads();
    pi_stage<N, P, R, L, false, BASE>(v, lds, t, tr);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------------
// Lane pairs: lanes 2j and 2j+1 hold the two spinor components of the same positions.  The
// partner's value comes over the DPP quad permutation [1,0,3,2] (no LDS traffic, no barrier).
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ float pair_swap(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ float2 pair_swap(float2 x) { return make_float2(pair_swap(x.x), pair_swap(x.y)); }
__device__ __forceinline__ double pair_swap(double x) {
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), 0xB1, 0xF, 0xF, false);
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), 0xB1, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double2 pair_swap(double2 x) { return make_double2(pair_swap(x.x), pair_swap(x.y)); }

// ---------------------------------------------------------------------------------------------
// (cos(phi) - 1, sin(phi)) with relative accuracy on both parts for small |phi|, and
// sin(phi)/phi.  Cody-Waite reduction by pi/2 (the first product is exact inside the FMA for
// |k| < 2^10), Taylor polynomials on |r| <= pi/4.
// ---------------------------------------------------------------------------------------------
struct SinCosM1 {
  float cm1, s, sinc;
};

__host__ __device__ __forceinline__ SinCosM1 sincos_m1_reduced(float phi) {
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
    // cos and sin have period 2 pi, so the reduced values serve for every k = 0 mod 4; sin(phi)/phi
    // does not: (1 + ps) = sin(r)/r equals it only for k = 0
    out.cm1 = cr_m1;
    out.s = sr;
    out.sinc = k == 0.0f ? 1.0f + ps : sr / phi;
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
__host__ __device__ __forceinline__ SinCosM1 sincos_m1_small(float phi) {
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
  if (fabsf(phi) <= 0.785398163f) return sincos_m1_small(phi);
  return sincos_m1_reduced(phi);
}

// The same with the routine fixed at compile time: SMALL requires |phi| <= pi/4; the reduced
// routine is exact for every phi.  Kernels pick one per wave (see wave_all), so a wave runs one
// straight-line routine instead of both paths under an execution mask.
template <bool SMALL>
__device__ __forceinline__ SinCosM1 sincos_m1_t(float phi) {
  if constexpr (SMALL) return sincos_m1_small(phi);
  else return sincos_m1_reduced(phi);
}
constexpr float kSmallPhase = 0.785398163f;   // pi/4

// fp64: (cos(phi) - 1, sin(phi), sin(phi)/phi) from one fp64 library sincos of phi/2, by the
// half-angle identities cos(phi) - 1 = -2 sin^2(phi/2) (relative accuracy for small phi) and
// sin(phi) = 2 sin(phi/2) cos(phi/2); one routine for every phi, so SMALL makes no difference.
struct SinCosM1d {
  double cm1, s, sinc;
};
template <bool SMALL>
__device__ __forceinline__ SinCosM1d sincos_m1_t(double phi) {
  SinCosM1d out;
  double h, c;
  sincos(0.5 * phi, &h, &c);
  out.s = 2.0 * h * c;
  out.cm1 = -2.0 * h * h;
  out.sinc = phi != 0.0 ? out.s / phi : 1.0;
  return out;
}

// True in every lane iff p holds in every active lane of the wave (a wave-uniform value).
__device__ __forceinline__ bool wave_all(bool p) { return __builtin_amdgcn_ballot_w64(!p) == 0; }

// ---------------------------------------------------------------------------------------------
// Deterministic reductions in fp64.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the workgroup in a fixed order; every thread must call it; red must hold 64 doubles.
// Result valid in every thread.
__device__ __forceinline__ double block_sum(double v, double* red) {
  const int n = blockDim.x;
  double s = 0.0;
  if ((n & 63) == 0) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    for (int w = 0; w < (n >> 6); ++w) s += red[w];
  } else {  // a workgroup smaller than one wave (small grids)
    __syncthreads();
    red[threadIdx.x] = v;
    __syncthreads();
    for (int i = 0; i < n; ++i) s += red[i];
  }
  __syncthreads();
  return s;
}

}  // namespace sgpe
