// Device body of the column pass (see col_pass.hip for the kernels): forward y-FFT, the k-space
// 2x2 propagator of Eqs. (H1), (H4) (Eq. TEOp), inverse y-FFT, and the imaginary-time norm
// partials -- shared by every kernel that runs column tiles.
#pragma once

#include "fft_device.hpp"
#include "sgpe_internal.hpp"

namespace sgpe {


__device__ __forceinline__ int col_group(int b, int ngroups) {
  // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a contiguous run of tile groups
  // so that tiles sharing 128-byte lines meet in the same L2.
  if ((ngroups & 7) == 0) return (b & 7) * (ngroups >> 3) + (b >> 3);
  return b;
}

// A workgroup handles ITERS adjacent tiles of C columns, one after the other; the next tile's
// data is loaded into registers before the current tile is transformed.  P points per lane:
// T = N / P lanes per transform.
extern __shared__ __align__(16) unsigned char col_lds[];

template <int N, int NORM, int ITERS, int P, bool WT, class R>
__device__ __forceinline__ void col_body(const ColArgsT<R>& a, int wg, int ngroups) {
  using CX = cplx_t<R>;
  CX* const lds_raw = reinterpret_cast<CX*>(col_lds);
  constexpr uint32_t PB = sizeof(point_t<R>), CB = sizeof(CX);   // bytes per point / component
  __shared__ double red[64];
  constexpr int T = N / P;
  const int C = a.cols;
  const int tid = threadIdx.x;
  const int comp = tid & 1;
  const int pair = tid >> 1;
  const int cc = pair & (C - 1);
  const int t = pair / C;
  const int tile0 = col_group(wg, ngroups) * ITERS;
  const int x0 = tile0 * C + cc;
  const LdsView<CX> lds{lds_raw + 2 * cc + comp, 1 + __builtin_ctz(C)};
  // element (row y) of this lane's component is at byte offset PB (y nx + x) + CB comp; 32-bit
  // offsets from a wave-uniform base, the row stride a wave-uniform value
  const char* __restrict__ base = reinterpret_cast<const char*>(a.psi);
  char* __restrict__ out = reinterpret_cast<char*>(a.psi);
  const uint32_t rstride = PB * static_cast<uint32_t>(a.nx);
  const uint32_t mstride = static_cast<uint32_t>(T) * rstride;
  const uint32_t tile_stride = PB * static_cast<uint32_t>(C);
  uint32_t off = static_cast<uint32_t>(t) * rstride + PB * static_cast<uint32_t>(x0) + CB * comp;

  // The k_y operator values of the lane's P rows.  With 16 points per lane the row is staged in
  // LDS (loaded per point after the forward transform, its latency would sit in the middle of the
  // pass); its loads go out first, into registers (at most P/2 per thread: a workgroup has at
  // least 2N/P threads), so writing them to LDS waits for them alone and not for the data behind
  // them.  With 8 or 4 points per lane the lane's own P values are loaded into registers up front
  // instead (measured: 13.45 -> 13.07 us per step at 512^2; at 16 points per lane the extra
  // registers cost 1 us at 1024^2).
  // complex128 columns of 4096 points leave no LDS for the k_y row (the exchange slots take 139 KB):
  // there each point's value is loaded after the forward transform, from the L2-resident table.
  constexpr bool KY_GLOBAL = sizeof(R) == 8 && N >= 4096;
  constexpr bool KY_LDS = P == 16 && !KY_GLOBAL;
  constexpr int KY_MAX = KY_LDS ? P / 2 : 1;
  const int nth = blockDim.x;
  CX kyv[KY_MAX], kyr[(KY_LDS || KY_GLOBAL) ? 1 : P];
  if constexpr (KY_GLOBAL) {
  } else if constexpr (KY_LDS) {
#pragma unroll
    for (int k = 0; k < KY_MAX; ++k)
      if (k * nth < N) kyv[k] = a.ky_tab[min(tid + k * nth, N - 1)];
  } else {
#pragma unroll
    for (int m = 0; m < P; ++m) kyr[m] = a.ky_tab[t + T * m];
  }
  CX v[P], nxt[P];
#pragma unroll
  for (int m = 0; m < P; ++m) v[m] = *reinterpret_cast<const CX*>(base + (off + mstride * m));
  // this component's row of M' - 1 at k_x: {d_own, d_other}
  point_t<R> d = a.kx_tab[2 * x0 + comp], dn = d;
  TwPlain<N, P, R> tr;
  load_twiddles<N>(tr, t, a.tw);
  CX* __restrict__ kyl = lds_raw + 2 * C * (N + N / 16);
  if constexpr (KY_LDS) {
#pragma unroll
    for (int k = 0; k < KY_MAX; ++k)
      if (k * nth < N && tid + k * nth < N) kyl[tid + k * nth] = kyv[k];
  }

  double acc = 0.0;
#pragma unroll
  for (int it = 0; it < ITERS; ++it) {
    if (it + 1 < ITERS) {
#pragma unroll
      for (int m = 0; m < P; ++m)
        nxt[m] = *reinterpret_cast<const CX*>(base + (off + tile_stride + mstride * m));
      dn = a.kx_tab[2 * (x0 + (it + 1) * C) + comp];
    }
    fwd_pass<N>(v, lds, t, tr);
    if constexpr (N <= P) __syncthreads();   // a single-stage transform has no barrier of its own

#pragma unroll
    for (int m = 0; m < P; ++m) {
      const CX w = v[m];
      const CX o = pair_swap(w);
      CX q;
      if constexpr (KY_GLOBAL) q = a.ky_tab[t + T * m];
      else if constexpr (KY_LDS) q = kyl[t + T * m];
      else q = kyr[m];
      const R c1r = fma_(-d.w, o.y, fma_(d.z, o.x, fma_(-d.y, w.y, d.x * w.x)));
      const R c1i = fma_(d.w, o.x, fma_(d.z, o.y, fma_(d.y, w.x, d.x * w.y)));
      const R cr = fma_(-q.y, w.y, fma_(q.x, w.x, fma_(-q.y, c1i, fma_(q.x, c1r, c1r))));
      const R ci = fma_(q.y, w.x, fma_(q.x, w.y, fma_(q.y, c1r, fma_(q.x, c1i, c1i))));
      const CX res = mk2(w.x + cr, w.y + ci);
      if constexpr (NORM == NORM_DOT) {
        acc += static_cast<double>(fma_(w.x, res.x, w.y * res.y));
      } else if constexpr (NORM == NORM_SQ) {
        acc += static_cast<double>(fma_(res.x, res.x, res.y * res.y));
      }
      v[m] = res;
    }

    inv_pass<N>(v, lds, t, tr);

#pragma unroll
    for (int m = 0; m < P; ++m) store_state<WT>(reinterpret_cast<CX*>(out + (off + mstride * m)), v[m]);
    if (it + 1 < ITERS) {
#pragma unroll
      for (int m = 0; m < P; ++m) v[m] = nxt[m];
      d = dn;
      off += tile_stride;
    }
  }
  if constexpr (NORM != NORM_NONE) {
    const double sum = block_sum(acc, red);
    if (tid == 0) a.partials[wg] = sum;
  }
}

}  // namespace sgpe
