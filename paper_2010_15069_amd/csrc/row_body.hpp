// Device bodies of the row pass (see row_pass.hip for the kernels and the pass's place in a
// step): the norm scale from the column pass's partials, the real-space exponential R(h) of
// Eqs. (H2)-(H4) (closed form with frozen densities, or N(h/2) L(h) N(h/2)), and the row body
// itself -- inverse x-FFT, scale, R, forward x-FFT -- shared by every kernel that runs rows.
#pragma once

#include "fft_device.hpp"
#include "sgpe_internal.hpp"

namespace sgpe {


// -------------------------------------------------------------------------------------------
// Sum of the previous column pass's partials -> scale for the row pass.  Every wave computes
// the same sum in the same order (lane l adds partials l, l + 64, ... in turn, then a fixed
// butterfly across the wave), so every workgroup applies bit-identical scales.  Up to 64 K
// partials are loaded at kernel start as K masked loads per lane, ahead of the data (a
// runtime-length loop of loads would make the wave wait for every outstanding load); more
// partials, or workgroups narrower than a wave, take the loop after the inverse transform.
// K = 4 (256 partials), and 16 (1024) for complex128 rows of up to 1024 points, whose 1-column
// tiles leave nx partials.
// -------------------------------------------------------------------------------------------
template <class R, int N>
constexpr int prefetch_per_lane() { return sizeof(R) == 8 && N <= 1024 ? 16 : 4; }

template <class A, int K>
__device__ __forceinline__ void prefetch_partials(const A& a, double (&pv)[K]) {
  const int lane = threadIdx.x & 63;
  // a uniform branch around unconditional loads (indices clamped into range; the surplus
  // masked out at the sum), so no lane-dependent control flow waits on a load
  if (a.partials != nullptr && a.n_partials <= 64 * K && blockDim.x >= 64) {
#pragma unroll
    for (int k = 0; k < K; ++k) pv[k] = a.partials[min(lane + 64 * k, a.n_partials - 1)];
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) pv[k] = 0.0;
  }
}

template <class A, int K>
__device__ __forceinline__ decltype(A::scale) row_scale(const A& a, const double (&pv)[K]) {
  if (a.partials == nullptr) return a.scale;
  double s = 0.0;
  if (blockDim.x >= 64) {
    if (a.n_partials <= 64 * K) {
      const int lane = threadIdx.x & 63;
#pragma unroll
      for (int k = 0; k < K; ++k) s += (lane + 64 * k < a.n_partials) ? pv[k] : 0.0;
    } else {
      const int lane = threadIdx.x & 63;
      for (int i = lane; i < a.n_partials; i += 64) s += a.partials[i];
    }
    s = wave_sum(s);
  } else {
    for (int i = 0; i < a.n_partials; ++i) s += a.partials[i];
  }
  const double norm = a.parseval_w * s;
  return static_cast<decltype(A::scale)>(sqrt(a.norm0 / norm) * a.inv_npts);
}

// A norm-derived scale that is not finite and positive means that the norm the partials gave was
// zero, infinite or NaN (a diverging or overflowing imaginary-time run).  Workgroup 0 records it in
// the context's status word; the host reports it at the next synchronising call.
template <class A, class R>
__device__ __forceinline__ void check_scale(const A& a, R s, int wg) {
  if (a.partials != nullptr && a.nonfinite != nullptr && wg == 0 && threadIdx.x == 0 &&
      !(s > R(0) && __builtin_isfinite(s)))
    __hip_atomic_store(a.nonfinite, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// -------------------------------------------------------------------------------------------
// Real-space exponential R(h) (Eqs. (H2)-(H4), densities of the input).  Each lane applies its
// component's row of the 2x2 exponential to its value w; o is the partner lane's value at the
// same point.  hv = h V(x, y); hbx = h Omega(x, y) / 2 with Omega(x, y) = Omega_x(x) + Omega_y(y).
// -------------------------------------------------------------------------------------------
template <class T>
struct RCoef {
  T hd_own;          // +- h delta / 2 for this component
  T hg_own;          // h g_{ss} of this component
  T hg_ud;           // h g_{up dn}
  T sgn;             // +1 up, -1 down
  T hg_uu, hg_dd, hdelta2;
};

// Diagonal R (no spatial Raman coupling): w exp(-ph) in imaginary time, w exp(-i ph) in real
// time, with ph = h (V + g_own n_own + g_ud n_other +- delta/2).  The real-time form is
// w + w (cm1 - i s), the small correction formed first.
template <bool IMAG, bool SMALL, class C, class T>
__device__ __forceinline__ C apply_r_diag(C w, T ph) {
  if constexpr (!IMAG) {
    const auto sc = sincos_m1_t<SMALL>(ph);
    return mk2(w.x + fma_(w.x, sc.cm1, w.y * sc.s), w.y + fma_(w.y, sc.cm1, -w.x * sc.s));
  } else {
    return vscale(w, exp_(-ph));
  }
}

// Full 2x2 R: H_R = A 1 + Bx sigma_x + Bz sigma_z (all times h).  The angles (A, |B|) of this
// point, for the wave's choice of routine.
template <class T>
struct RFull {
  T ha, hbz, th;
};
template <class T>
__device__ __forceinline__ RFull<T> r_full_angles(T n_own, T n_oth, T hv, const RCoef<T>& c, T hbx) {
  const T nu = c.sgn > T(0) ? n_own : n_oth;
  const T nd = c.sgn > T(0) ? n_oth : n_own;
  const T gu = fma_(c.hg_uu, nu, c.hg_ud * nd);
  const T gd = fma_(c.hg_dd, nd, c.hg_ud * nu);
  RFull<T> f;
  f.ha = fma_(T(0.5), gu + gd, hv);
  f.hbz = fma_(T(0.5), gu - gd, c.hdelta2);
  f.th = sqrt_(fma_(hbx, hbx, f.hbz * f.hbz));
  return f;
}
// Whether the SMALL routines are valid for this point.
template <bool IMAG, class T>
__device__ __forceinline__ bool r_full_small(const RFull<T>& f) {
  if constexpr (!IMAG) return fabs_(f.ha) <= T(kSmallPhase) && f.th <= T(kSmallPhase);
  else return f.th < T(0.25);
}

template <bool IMAG, bool SMALL, class C, class T>
__device__ __forceinline__ C apply_r_full(C w, C o, const RFull<T>& f, T hbx, T sgn) {
  if constexpr (!IMAG) {
    // M = cos(th) 1 - i sin(th)/th (hB . sigma): this component's row of (M - 1) psi is
    // cm1 w - i X with X = +-pz w + px o.
    const auto sb = sincos_m1_t<SMALL>(f.th);
    const T px = sb.sinc * hbx, pz = sgn * sb.sinc * f.hbz;
    const T xr = fma_(pz, w.x, px * o.x), xi = fma_(pz, w.y, px * o.y);
    const T mr = fma_(sb.cm1, w.x, xi), mi = fma_(sb.cm1, w.y, -xr);
    // E M psi - psi = c_M + (E - 1)(w + c_M), E - 1 = cm1_A - i s_A; added to w once.
    const auto se = sincos_m1_t<SMALL>(f.ha);
    const T cr = fma_(se.s, w.y, fma_(se.cm1, w.x, fma_(se.s, mi, fma_(se.cm1, mr, mr))));
    const T ci = fma_(-se.s, w.x, fma_(se.cm1, w.y, fma_(-se.s, mr, fma_(se.cm1, mi, mi))));
    return mk2(w.x + cr, w.y + ci);
  } else {
    const T ea = exp_(-f.ha);
    T ch, shc;  // cosh(th), sinh(th)/th
    if constexpr (sizeof(T) == 8) {
      ch = cosh(f.th);
      shc = f.th > 1e-4 ? sinh(f.th) / f.th : fma(f.th * f.th, 1.0 / 6.0, 1.0);   // next term th^4/120
    } else if constexpr (SMALL) {
      const float t2 = f.th * f.th;
      ch = fmaf(t2, fmaf(t2, fmaf(t2, fmaf(t2, 2.48015873e-5f, 1.38888889e-3f), 4.16666667e-2f), 0.5f), 1.0f);
      shc = fmaf(t2, fmaf(t2, fmaf(t2, fmaf(t2, 2.75573192e-6f, 1.98412698e-4f), 8.33333333e-3f),
                           1.66666667e-1f), 1.0f);
    } else {
      if (f.th < 0.25f) {
        const float t2 = f.th * f.th;
        ch = fmaf(t2, fmaf(t2, fmaf(t2, fmaf(t2, 2.48015873e-5f, 1.38888889e-3f), 4.16666667e-2f), 0.5f), 1.0f);
        shc = fmaf(t2, fmaf(t2, fmaf(t2, fmaf(t2, 2.75573192e-6f, 1.98412698e-4f), 8.33333333e-3f),
                             1.66666667e-1f), 1.0f);
      } else {
        const float ep = expf(f.th);
        const float em = 1.0f / ep;
        ch = 0.5f * (ep + em);
        shc = 0.5f * (ep - em) / f.th;
      }
    }
    const T m_own = ea * fma_(-sgn * shc, f.hbz, ch);
    const T m_x = -ea * shc * hbx;
    return mk2(fma_(m_own, w.x, m_x * o.x), fma_(m_own, w.y, m_x * o.y));
  }
}

// -------------------------------------------------------------------------------------------
// Row pass
// -------------------------------------------------------------------------------------------
// R on the thread's 16 points.  For each point index the wave takes one routine: the short one
// when every lane's angles allow it (the common case), else the general one -- a wave-uniform
// branch, so a wave never runs both.
// hbx_r: this lane's h Omega_x / 2 at its P positions, hb_row: h Omega_y / 2 of the row (full
// 2x2 variant only; loaded by the caller ahead of the transforms).
template <int N, bool IMAG, bool FULL, int P, class C, class R>
__device__ __forceinline__ void row_apply_r(C (&v)[P], const RowArgsT<R>& a, int row, int t, bool up,
                                            const R (&hbx_r)[P], R hb_row) {
  constexpr int T = N / P;
  RCoef<R> c;
  c.sgn = up ? R(1) : R(-1);
  c.hd_own = up ? a.hdelta2 : -a.hdelta2;
  c.hg_own = up ? a.hg_uu : a.hg_dd;
  c.hg_ud = a.hg_ud;
  c.hg_uu = a.hg_uu;
  c.hg_dd = a.hg_dd;
  c.hdelta2 = a.hdelta2;
  const R y = fma_(static_cast<R>(row), a.dy, a.y0);
  const R hvy = a.hvy * y * y;
#pragma unroll
  for (int m = 0; m < P; ++m) {
    const int j = t + T * m;
    const R x = fma_(static_cast<R>(j), a.dx, a.x0);
    const R hv = fma_(a.hvx * x, x, hvy);
    const R n_own = fma_(v[m].x, v[m].x, v[m].y * v[m].y);
    if constexpr (!FULL) {
      const R n_oth = pair_swap(n_own);
      const R ph = fma_(c.hg_own, n_own, fma_(c.hg_ud, n_oth, hv + c.hd_own));
      if (IMAG || wave_all(fabs_(ph) <= R(kSmallPhase))) v[m] = apply_r_diag<IMAG, true>(v[m], ph);
      else v[m] = apply_r_diag<IMAG, false>(v[m], ph);
    } else {
      const R hbx = hbx_r[m] + hb_row;
      const C o = pair_swap(v[m]);
      const R n_oth = fma_(o.x, o.x, o.y * o.y);
      const RFull<R> f = r_full_angles(n_own, n_oth, hv, c, hbx);
      if (wave_all(r_full_small<IMAG>(f))) v[m] = apply_r_full<IMAG, true>(v[m], o, f, hbx, c.sgn);
      else v[m] = apply_r_full<IMAG, false>(v[m], o, f, hbx, c.sgn);
    }
  }
}

// R(h) split to second order as N(h/2) L(h) N(h/2): the mean-field phase with the densities of
// its input, the exponential of the linear real-space terms (trap, detuning, spatial coupling),
// the mean-field phase again with the updated densities.  Coefficients as in row_apply_r.
template <int N, bool IMAG, bool FULL, int P, class C, class R>
__device__ __forceinline__ void row_apply_r_nln(C (&v)[P], const RowArgsT<R>& a, int row, int t, bool up,
                                                const R (&hbx_r)[P], R hb_row) {
  if constexpr (!FULL && !IMAG) {
    // Real time with a diagonal linear part: the three factors are phases, which commute and leave
    // both densities as they are, so their product is the one phase of the frozen form with the
    // input's densities -- the same exponent, evaluated once instead of three times.
    row_apply_r<N, IMAG, FULL>(v, a, row, t, up, hbx_r, hb_row);
    return;
  }
  constexpr int T = N / P;
  RCoef<R> c;
  c.sgn = up ? R(1) : R(-1);
  c.hd_own = up ? a.hdelta2 : -a.hdelta2;
  c.hg_own = up ? a.hg_uu : a.hg_dd;
  c.hg_ud = a.hg_ud;
  c.hg_uu = a.hg_uu;
  c.hg_dd = a.hg_dd;
  c.hdelta2 = a.hdelta2;
  const R y = fma_(static_cast<R>(row), a.dy, a.y0);
  const R hvy = a.hvy * y * y;
  auto half_n = [&](C w) {
    const R n_own = fma_(w.x, w.x, w.y * w.y);
    const R n_oth = pair_swap(n_own);
    const R ph = R(0.5) * fma_(c.hg_own, n_own, c.hg_ud * n_oth);
    if (IMAG || wave_all(fabs_(ph) <= R(kSmallPhase))) return apply_r_diag<IMAG, true>(w, ph);
    return apply_r_diag<IMAG, false>(w, ph);
  };
#pragma unroll
  for (int m = 0; m < P; ++m) {
    const int j = t + T * m;
    const R x = fma_(static_cast<R>(j), a.dx, a.x0);
    const R hv = fma_(a.hvx * x, x, hvy);
    C w = half_n(v[m]);
    if constexpr (!FULL) {
      const R ph = hv + c.hd_own;
      if (IMAG || wave_all(fabs_(ph) <= R(kSmallPhase))) w = apply_r_diag<IMAG, true>(w, ph);
      else w = apply_r_diag<IMAG, false>(w, ph);
    } else {
      const R hbx = hbx_r[m] + hb_row;
      const C o = pair_swap(w);
      RFull<R> f;
      f.ha = hv;
      f.hbz = c.hdelta2;
      f.th = sqrt_(fma_(hbx, hbx, f.hbz * f.hbz));
      if (wave_all(r_full_small<IMAG>(f))) w = apply_r_full<IMAG, true>(w, o, f, hbx, c.sgn);
      else w = apply_r_full<IMAG, false>(w, o, f, hbx, c.sgn);
    }
    v[m] = half_n(w);
  }
}

// A workgroup handles ITERS groups of rows_per_block rows, one after the other; the next group's
// data is loaded into registers before the current group is transformed, so its memory latency
// hides behind this group's arithmetic.  P points per lane: T = N / P lanes per transform.
// The kernels' dynamic LDS, typed per precision where it is used.
extern __shared__ __align__(16) unsigned char row_lds[];

template <int N, int MODE, bool IMAG, bool FULL, int ITERS, int P, bool WT, class R>
__device__ __forceinline__ void row_body(const RowArgsT<R>& a, int wg) {
  using C = cplx_t<R>;
  C* const lds_raw = reinterpret_cast<C*>(row_lds);
  constexpr int T = N / P;
  constexpr int SLOTS = N + N / 16;
  constexpr uint32_t PB = sizeof(point_t<R>), CB = sizeof(C);   // bytes per point / component
  const int tid = threadIdx.x;
  const int comp = tid & 1;
  const int pair = tid >> 1;
  const int rloc = pair / T;
  const int t = pair - rloc * T;
  const int row0 = wg * ITERS * a.rows_per_block + rloc;
  constexpr bool STEP = MODE == ROW_STEP || MODE == ROW_STEP_NLN;
  const LdsView<C> lds{lds_raw + rloc * 2 * SLOTS + comp, 1};
  // element `pos` of this lane's component is at byte offset PB pos from the row start; 32-bit
  // offsets from a wave-uniform base
  const char* __restrict__ base = reinterpret_cast<const char*>(a.psi);
  char* __restrict__ out = reinterpret_cast<char*>(a.psi);
  const uint32_t lane_off = static_cast<uint32_t>(t) * PB + CB * comp;
  const uint32_t group_stride = static_cast<uint32_t>(a.rows_per_block) * (PB * N);

  double pv[prefetch_per_lane<R, N>()];
  if constexpr (MODE != ROW_FWD) prefetch_partials(a, pv);
  C v[P], nxt[P];
  uint32_t off = static_cast<uint32_t>(row0) * (PB * N) + lane_off;
  // Load order: the inverse transform starts with the last forward stage, whose butterfly u
  // takes positions u + U k; issuing those loads together lets it start before the rest land.
  constexpr int RL = MODE == ROW_FWD ? P : last_radix<N, P>();
  constexpr int UL = P / RL;
#pragma unroll
  for (int i = 0; i < P; ++i) {
    const int m = i / RL + UL * (i % RL);
    v[m] = *reinterpret_cast<const C*>(base + (off + PB * T * m));
  }
  TwPlain<N, P, R> tr;
  load_twiddles<N>(tr, t, a.tw);
  // spatial Raman tables: the x part is the same for every row of the workgroup
  R hbx_r[P], hby_r[ITERS];
  if constexpr (FULL && STEP) {
#pragma unroll
    for (int m = 0; m < P; ++m) hbx_r[m] = a.hbx[t + T * m];
#pragma unroll
    for (int it = 0; it < ITERS; ++it) hby_r[it] = a.hby[row0 + it * a.rows_per_block];
  }
  R s = R(1);

#pragma unroll
  for (int it = 0; it < ITERS; ++it) {
    if (it + 1 < ITERS) {
#pragma unroll
      for (int i = 0; i < P; ++i) {
        const int m = i / RL + UL * (i % RL);
        nxt[m] = *reinterpret_cast<const C*>(base + (off + group_stride + PB * T * m));
      }
    }
    if constexpr (MODE == ROW_FWD) {
      fwd_pass<N>(v, lds, t, tr);
    } else {
      inv_pass<N>(v, lds, t, tr);
      if (it == 0) {
        s = row_scale(a, pv);
        check_scale(a, s, wg);
      }
#pragma unroll
      for (int m = 0; m < P; ++m) v[m] = vscale(v[m], s);
      if constexpr (MODE == ROW_STEP_NLN) {
        row_apply_r_nln<N, IMAG, FULL>(v, a, row0 + it * a.rows_per_block, t, comp == 0, hbx_r,
                                       FULL ? hby_r[it] : R(0));
        fwd_pass<N>(v, lds, t, tr);
      } else if constexpr (MODE == ROW_STEP) {
        row_apply_r<N, IMAG, FULL>(v, a, row0 + it * a.rows_per_block, t, comp == 0, hbx_r,
                                   FULL ? hby_r[it] : R(0));
        fwd_pass<N>(v, lds, t, tr);
      }
    }
#pragma unroll
    for (int m = 0; m < P; ++m) store_state<WT>(reinterpret_cast<C*>(out + (off + PB * T * m)), v[m]);
    if (it + 1 < ITERS) {
#pragma unroll
      for (int m = 0; m < P; ++m) v[m] = nxt[m];
      off += group_stride;
    }
  }
}

// The general row pass of the splitting variants (one row group per workgroup); see RowVarFlags.
template <int N, bool IMAG, bool FULL, int P>
__device__ __forceinline__ void row_var_body(const RowArgs& a, int wg) {
  float2* const lds_raw = reinterpret_cast<float2*>(row_lds);
  __shared__ double red[64];
  constexpr int T = N / P;
  constexpr int SLOTS = N + N / 16;
  const int tid = threadIdx.x;
  const int comp = tid & 1;
  const int pair = tid >> 1;
  const int rloc = pair / T;
  const int t = pair - rloc * T;
  const int row = wg * a.rows_per_block + rloc;
  const LdsView<float2> lds{lds_raw + rloc * 2 * SLOTS + comp, 1};
  const char* __restrict__ base = reinterpret_cast<const char*>(a.psi);
  char* __restrict__ out = reinterpret_cast<char*>(a.psi);
  const uint32_t off = static_cast<uint32_t>(row) * (16u * N) + static_cast<uint32_t>(t) * 16u + 8u * comp;
  const int flags = a.var_flags;

  double pv[prefetch_per_lane<float, N>()];
  prefetch_partials(a, pv);
  float2 v[P];
#pragma unroll
  for (int m = 0; m < P; ++m) v[m] = *reinterpret_cast<const float2*>(base + (off + 16u * T * m));
  TwPlain<N, P> tr;
  load_twiddles<N>(tr, t, a.tw);
  float hbx_r[P], hb_row = 0.0f;
  if constexpr (FULL) {
#pragma unroll
    for (int m = 0; m < P; ++m) hbx_r[m] = a.hbx[t + T * m] * a.hfrac;
    hb_row = a.hby[row] * a.hfrac;
  }
  const bool mid = (flags & VAR_MID_SCALE) != 0;
  if (flags & (VAR_INV | VAR_SCALE)) {
    if (flags & VAR_INV) inv_pass<N>(v, lds, t, tr);
    const float s = mid ? a.scale : row_scale(a, pv);
    if (!mid) check_scale(a, s, wg);
#pragma unroll
    for (int m = 0; m < P; ++m) v[m] = vscale(v[m], s);
  }
  for (int r = 0; r < a.var_r; ++r) {
    if (a.var_nln) row_apply_r_nln<N, IMAG, FULL>(v, a, row, t, comp == 0, hbx_r, hb_row);
    else row_apply_r<N, IMAG, FULL>(v, a, row, t, comp == 0, hbx_r, hb_row);
    if (mid && r == 0) {
      const float c = row_scale(a, pv);
      check_scale(a, c, wg);
#pragma unroll
      for (int m = 0; m < P; ++m) v[m] = vscale(v[m], c);
    }
  }
  if (flags & VAR_NORM_OUT) {
    double acc = 0.0;
#pragma unroll
    for (int m = 0; m < P; ++m) acc += double(v[m].x) * double(v[m].x) + double(v[m].y) * double(v[m].y);
    acc = block_sum(acc, red);
    if (tid == 0) a.partials_out[wg] = acc;
  }
  if (flags & VAR_FWD) fwd_pass<N>(v, lds, t, tr);
  if (!(flags & VAR_NO_STORE)) {
#pragma unroll
    for (int m = 0; m < P; ++m) store_state<true>(reinterpret_cast<float2*>(out + (off + 16u * T * m)), v[m]);
  }
}

}  // namespace sgpe
