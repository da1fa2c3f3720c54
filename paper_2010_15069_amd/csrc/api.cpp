// Host side of the split-step solver: parameter validation, fp64 construction of the operator
// and twiddle tables, the fused step schedule, and the C ABI declared in include/sgpe.h.
#include "sgpe.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <type_traits>
#include <cstring>
#include <new>
#include <vector>

#include "host_internal.hpp"
#include "sgpe_internal.hpp"

using sgpe::ColArgs;
using sgpe::EnergyArgs;
using sgpe::RowArgs;

namespace {

constexpr int kMinN = 16;
constexpr int kMaxN = 4096;

bool is_pow2(int32_t n) { return n > 0 && (n & (n - 1)) == 0; }
bool is_finite(double v) { return std::isfinite(v); }

}  // namespace


namespace sgpe_host {

inline float4 mk4(double a, double b, double c, double d, float) { return make_float4(float(a), float(b), float(c), float(d)); }
inline double4 mk4(double a, double b, double c, double d, double) { return make_double4(a, b, c, d); }
inline float2 mk2h(double a, double b, float) { return make_float2(float(a), float(b)); }
inline double2 mk2h(double a, double b, double) { return make_double2(a, b); }

sgpe_status dev_alloc(sgpe_ctx* c, void** ptr, size_t bytes) {
  *ptr = nullptr;
  if (hipMalloc(ptr, bytes) != hipSuccess) {
    (void)hipGetLastError();
    *ptr = nullptr;
    return SGPE_ENOMEM;
  }
  c->allocations.push_back(*ptr);
  return SGPE_OK;
}

template <class T>
sgpe_status upload(sgpe_ctx* c, T** dst, const std::vector<T>& host) {
  void* p = nullptr;
  sgpe_status st = dev_alloc(c, &p, host.size() * sizeof(T));
  if (st != SGPE_OK) return st;
  if (hipMemcpy(p, host.data(), host.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    return SGPE_EDEVICE;
  }
  *dst = static_cast<T*>(p);
  return SGPE_OK;
}

// Tables of the spatial Raman coupling Omega_x(x_j) + Omega_y(y_i) (Eq. (H4) with Omega(r)): the
// step kernels' half-angles dt Omega / 2 in fp32 and the energy kernel's Omega in fp64.  NULL
// stands for a zero profile.  Allocated on first use, overwritten in place afterwards.
sgpe_status raman_tables(sgpe_ctx* c, const double* om_x, const double* om_y) {
  const sgpe_params& p = c->p;
  sgpe_status st;
  void* ptr = nullptr;
  if (c->prec == SGPE_C128 && !c->hbx64) {
    if ((st = dev_alloc(c, &ptr, size_t(p.nx) * sizeof(double))) != SGPE_OK) return st;
    c->hbx64 = static_cast<double*>(ptr);
    if ((st = dev_alloc(c, &ptr, size_t(p.ny) * sizeof(double))) != SGPE_OK) return st;
    c->hby64 = static_cast<double*>(ptr);
  }
  if (!c->hbx) {
    if ((st = dev_alloc(c, &ptr, size_t(p.nx) * sizeof(float))) != SGPE_OK) return st;
    c->hbx = static_cast<float*>(ptr);
    if ((st = dev_alloc(c, &ptr, size_t(p.ny) * sizeof(float))) != SGPE_OK) return st;
    c->hby = static_cast<float*>(ptr);
    if ((st = dev_alloc(c, &ptr, size_t(p.nx) * sizeof(double))) != SGPE_OK) return st;
    c->omx = static_cast<double*>(ptr);
    if ((st = dev_alloc(c, &ptr, size_t(p.ny) * sizeof(double))) != SGPE_OK) return st;
    c->omy = static_cast<double*>(ptr);
  }
  std::vector<double> ox(p.nx, 0.0), oy(p.ny, 0.0);
  if (om_x) ox.assign(om_x, om_x + p.nx);
  if (om_y) oy.assign(om_y, om_y + p.ny);
  std::vector<float> hx(p.nx), hy(p.ny);
  std::vector<double> hx64(p.nx), hy64(p.ny);
  for (int j = 0; j < p.nx; ++j) hx64[j] = 0.5 * p.dt * ox[j], hx[j] = float(hx64[j]);
  for (int i = 0; i < p.ny; ++i) hy64[i] = 0.5 * p.dt * oy[i], hy[i] = float(hy64[i]);
  if (c->prec == SGPE_C128 &&
      (hipStreamSynchronize(c->stream) != hipSuccess ||
       hipMemcpy(c->hbx64, hx64.data(), hx64.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
       hipMemcpy(c->hby64, hy64.data(), hy64.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)) {
    (void)hipGetLastError();
    return SGPE_EDEVICE;
  }
  // the stream's queued steps may still read the old tables
  if (hipStreamSynchronize(c->stream) != hipSuccess ||
      hipMemcpy(c->hbx, hx.data(), hx.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->hby, hy.data(), hy.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->omx, ox.data(), ox.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->omy, oy.data(), oy.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    return SGPE_EDEVICE;
  }
  return SGPE_OK;
}

// Forward roots exp(-2 pi i j / n), j < n / 2, in fp64 (energy kernels).
// Roots exp(-2 pi i j / n) rounded once to fp32 as {cos, sin, eta, 0}, where
// 1 + eta = 1 / (cos^2 + sin^2) of the rounded pair (evaluated in fp64): the step kernels'
// forward transform multiplies by the rounded root, their exact inverse by conj(root)(1 + eta),
// whose low part conj(root) eta they form from cos, sin and eta.
// fp64 (complex128 kernels): the roots rounded to fp64 with eta = 0 -- their modulus error, ~1e-16,
// needs no correction at that precision.
template <class T = float>
std::vector<sgpe::point_t<T>> twiddles_plain(int n) {
  std::vector<sgpe::point_t<T>> t(n);
  for (int j = 0; j < n; ++j) {
    const double a = 2.0 * M_PI * double(j) / double(n);
    const T c = T(std::cos(a)), s = T(std::sin(a));
    const double eta = std::is_same<T, float>::value ? 1.0 / (double(c) * double(c) + double(s) * double(s)) - 1.0 : 0.0;
    t[j] = mk4(c, s, eta, 0.0, T());
  }
  return t;
}

// FFT-ordered angular wave numbers: 2 pi fftfreq(n, d).
double kval(int j, int n, double d) {
  const int m = j < n / 2 ? j : j - n;
  return 2.0 * M_PI * double(m) / (double(n) * d);
}

// k-space 2x2 propagator factored as P(k_y) M'(k_x) with
//   M'(k_x) = e^{-h kx^2/2 (i)} [ c 1 - s (b . sigma) ],  b = (omega/2, k_l k_x),
//   P(k_y)  = e^{-h ky^2/2 (i)};
// stored as M' - 1 (four complex entries) and P - 1, to fp32 relative accuracy.
template <class T = float>
void k_tables(const sgpe_params& p, bool imag, double h, std::vector<sgpe::point_t<T>>& kx_out,
              std::vector<sgpe::cplx_t<T>>& ky_out) {
  const double dx = 2.0 * p.xmax / p.nx, dy = 2.0 * p.ymax / p.ny;
  kx_out.assign(2 * size_t(p.nx), mk4(0, 0, 0, 0, T()));
  ky_out.assign(size_t(p.ny), mk2h(0, 0, T()));
  for (int j = 0; j < p.nx; ++j) {
    const double kx = kval(j, p.nx, dx);
    const double bx = 0.5 * p.omega, bz = p.k_l * kx;
    const double bm = std::hypot(bx, bz);
    const double al = 0.5 * h * kx * kx;
    double m11r, m11i, m12r, m12i, m22r, m22i;
    if (!imag) {
      const double c = std::cos(h * bm);
      const double s = bm > 0.0 ? std::sin(h * bm) / bm : h;
      const double pr = std::cos(al), pi = -std::sin(al);
      // pref * (c - i s bz), pref * (-i s bx), pref * (c + i s bz)
      m11r = pr * c + pi * s * bz;  m11i = pi * c - pr * s * bz;
      m12r = pi * s * bx;           m12i = -pr * s * bx;
      m22r = pr * c - pi * s * bz;  m22i = pi * c + pr * s * bz;
    } else {
      const double ch = std::cosh(h * bm);
      const double sh = bm > 0.0 ? std::sinh(h * bm) / bm : h;
      const double pr = std::exp(-al);
      m11r = pr * (ch - sh * bz);  m11i = 0.0;
      m12r = -pr * sh * bx;        m12i = 0.0;
      m22r = pr * (ch + sh * bz);  m22i = 0.0;
    }
    // per component: {d_own, d_other} of its row of M' - 1 (up: d11, d12; down: d22, d21)
    kx_out[2 * size_t(j)] = mk4(m11r - 1.0, m11i, m12r, m12i, T());
    kx_out[2 * size_t(j) + 1] = mk4(m22r - 1.0, m22i, m12r, m12i, T());
  }
  for (int i = 0; i < p.ny; ++i) {
    const double ky = kval(i, p.ny, dy);
    const double be = 0.5 * h * ky * ky;
    if (!imag) {
      const double sh = std::sin(0.5 * be);
      ky_out[i] = mk2h(-2.0 * sh * sh, -std::sin(be), T());
    } else {
      ky_out[i] = mk2h(std::expm1(-be), 0.0, T());
    }
  }
}

// Default schedule (from measured sweeps on MI355X).  Points per lane: 16 where the grid alone
// fills the device; on small grids fewer points per lane (more lanes, a shorter instruction
// stream per lane) cut each pass's latency.  Row prefetching (two row groups per workgroup) pays
// only for small rows whose one-group grid is a single round of resident workgroups (two per
// compute unit): then nothing else would overlap the first loads and last stores.  Column
// prefetching needs the narrower tile and measured slower everywhere; it stays off by default.
int default_points(int n, size_t npts) {
  if (n > sgpe::kMaxNSmallP) return 16;
  if (npts >= (size_t(1) << 19)) return 16;
  return npts >= (size_t(1) << 17) ? 8 : 4;
}

void default_schedule(sgpe_ctx* c) {
  const int nx = c->p.nx, ny = c->p.ny;
  const size_t npts = size_t(nx) * size_t(ny);
  c->row_points = default_points(nx, npts);
  c->col_points = default_points(ny, npts);
  c->rows = sgpe::row_rows_per_block(nx, ny, c->row_points, c->max_lds);
  c->cols = sgpe::col_default_cols(nx, ny, c->col_points, c->max_lds);
  c->row_iters = 1;
  c->col_iters = 1;
  // Column tiles: as many workgroups as compute units, up to one per CU, where that tile is
  // supported (measured: 1 column at 128^2 and 256^2, -9 % and -4 % per step; 512^2-1024^2 already
  // have one per CU; at 2048^2 it would take 2048 threads).
  {
    const int cc = std::max(1, nx / c->n_cu);
    if ((cc & (cc - 1)) == 0 && sgpe::col_cols_supported(nx, ny, cc, 1, c->col_points, c->max_lds)) c->cols = cc;
  }
  // One row per workgroup where a row takes at least two waves (measured at 256^2-2048^2: fastest,
  // or within 1 % at 512^2; one 4-row workgroup per CU was 8 % slower per step at 1024^2 and row
  // prefetch slower everywhere).  Smaller rows keep the derived tile.
  if (nx / c->row_points >= 64 && sgpe::schedule_supported(nx, 1, 1, c->row_points) &&
      sgpe::row_lds_bytes(nx, 1) <= c->max_lds) {
    c->rows = 1;
    return;
  }
  const int groups = ny / c->rows;
  if (c->row_points == 16 && groups == 2 * c->n_cu && sgpe::schedule_supported(nx, c->rows, 2, 16))
    c->row_iters = 2;
}

int col_groups(const sgpe_ctx* c) { return c->p.nx / (c->cols * c->col_iters); }

sgpe_status apply_schedule(sgpe_ctx* c, const sgpe_schedule& s) {
  const sgpe_params& p = c->p;
  if (s.row_points != 4 && s.row_points != 8 && s.row_points != 16) return SGPE_EINVAL;
  if (s.col_tile < 1) return SGPE_EINVAL;
  if (s.row_tile < 0) return SGPE_EINVAL;
  const int rows = s.row_tile > 0 ? s.row_tile : sgpe::row_rows_per_block(p.nx, p.ny, s.row_points, c->max_lds);
  if (rows > p.ny || !sgpe::schedule_supported(p.nx, rows, s.row_iters, s.row_points) ||
      p.ny % (rows * s.row_iters) != 0 ||
      sgpe::row_lds_bytes(p.nx, rows) > c->max_lds)
    return SGPE_EINVAL;
  if (!sgpe::col_cols_supported(p.nx, p.ny, s.col_tile, s.col_iters, s.col_points, c->max_lds)) return SGPE_EINVAL;
  c->rows = rows;
  c->cols = s.col_tile;
  c->row_iters = s.row_iters;
  c->col_iters = s.col_iters;
  c->row_points = s.row_points;
  c->col_points = s.col_points;
  return SGPE_OK;
}

sgpe_schedule get_schedule(const sgpe_ctx* c) {
  sgpe_schedule s{};
  s.col_tile = c->cols;
  s.row_tile = c->rows;
  s.row_iters = c->row_iters;
  s.col_iters = c->col_iters;
  s.row_points = c->row_points;
  s.col_points = c->col_points;
  return s;
}

sgpe_status status_of(hipError_t e) {
  if (e == hipSuccess) return SGPE_OK;
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return SGPE_ENOMEM;
  return SGPE_EDEVICE;
}

template <class T>
sgpe::RowArgsT<T> row_args_t(const sgpe_ctx* c, double h_sub) {
  const sgpe_params& p = c->p;
  sgpe::RowArgsT<T> a{};
  if constexpr (std::is_same<T, double>::value) {
    a.psi = c->psi64;
    a.tw = c->twp64_x;
    a.hbx = c->hbx64;
    a.hby = c->hby64;
  } else {
    a.psi = c->psi;
    a.tw = c->twp_x;
    a.hbx = c->hbx;
    a.hby = c->hby;
  }
  a.nx = p.nx;
  a.ny = p.ny;
  a.rows_per_block = c->rows;
  a.scale = T(1);
  a.partials = nullptr;
  a.n_partials = 0;
  const double dx = 2.0 * p.xmax / p.nx, dy = 2.0 * p.ymax / p.ny;
  const double npts = double(p.nx) * double(p.ny);
  a.norm0 = p.norm0;
  a.parseval_w = dx * dy / npts;
  a.inv_npts = 1.0 / npts;
  a.x0 = T(-p.xmax);
  a.dx = T(dx);
  a.y0 = T(-p.ymax);
  a.dy = T(dy);
  const double h = h_sub > 0.0 ? h_sub : p.dt;
  a.hfrac = T(h / p.dt);
  a.hvx = T(0.5 * h * p.wx * p.wx);
  a.hvy = T(0.5 * h * p.wy * p.wy);
  a.hdelta2 = T(0.5 * h * p.delta);
  a.hg_uu = T(h * p.g_uu);
  a.hg_dd = T(h * p.g_dd);
  a.hg_ud = T(h * p.g_ud);
  a.nonfinite = c->status_dev;
  return a;
}

RowArgs row_args(const sgpe_ctx* c, double h_sub) { return row_args_t<float>(c, h_sub); }

template <class T>
sgpe::ColArgsT<T> col_args_t(const sgpe_ctx* c, bool imag, bool half) {
  sgpe::ColArgsT<T> a{};
  const int idx = 2 * (imag ? 1 : 0) + (half ? 1 : 0);
  if constexpr (std::is_same<T, double>::value) {
    a.psi = c->psi64;
    a.tw = c->twp64_y;
    a.kx_tab = c->kx64[idx];
    a.ky_tab = c->ky64[idx];
  } else {
    a.psi = c->psi;
    a.tw = c->twp_y;
    a.kx_tab = c->kx_tab[idx];
    a.ky_tab = c->ky_tab[idx];
  }
  a.nx = c->p.nx;
  a.ny = c->p.ny;
  a.cols = c->cols;
  a.partials = c->partials;
  return a;
}

ColArgs col_args(const sgpe_ctx* c, bool imag, bool half) { return col_args_t<float>(c, imag, half); }

// The fused schedule on a complex128 state: the same sequence of passes as run_steps, with the
// fp64 instantiations of the kernels (16 or 8 points per lane, no prefetch).
static sgpe_status run_steps_c128(sgpe_ctx* c, int64_t n, bool imag) {
  const double npts = double(c->p.nx) * double(c->p.ny);
  hipStream_t s = c->stream;
  sgpe::RowArgsT<double> ra = row_args_t<double>(c, 0.0);
  // a pending tail of this kind continues as in run_steps; one of the other kind completes first
  const int kind = imag ? 2 : 1;
  if (c->tail_pending != 0 && c->tail_pending != kind) {
    const sgpe_status st = flush_tail(c);
    if (st != SGPE_OK) return st;
  }
  const bool cont = c->tail_pending == kind;
  c->tail_pending = 0;
  hipError_t e;
  if (cont) {
    e = sgpe::launch_col(col_args_t<double>(c, imag, false), imag ? sgpe::NORM_DOT : sgpe::NORM_NONE, c->col_points,
                         s);
  } else {
    e = sgpe::launch_row(ra, sgpe::ROW_FWD, false, false, c->row_points, s);
    if (e == hipSuccess) e = sgpe::launch_col(col_args_t<double>(c, imag, true), sgpe::NORM_NONE, c->col_points, s);
  }
  const bool defer = c->own_psi;
  for (int64_t i = 1; i <= n && e == hipSuccess; ++i) {
    sgpe::RowArgsT<double> r = ra;
    r.scale = 1.0 / npts;
    if (imag && (i > 1 || cont)) {
      r.partials = c->partials;
      r.n_partials = col_groups(c);
    }
    e = sgpe::launch_row(r, sgpe::ROW_STEP, imag, c->full2x2, c->row_points, s);
    const bool last = (i == n);
    if (last && defer) break;   // the last K(dt/2) and the inverse x-transform wait (flush_tail)
    const int nm = imag ? (last ? sgpe::NORM_SQ : sgpe::NORM_DOT) : sgpe::NORM_NONE;
    if (e == hipSuccess) e = sgpe::launch_col(col_args_t<double>(c, imag, last), nm, c->col_points, s);
  }
  if (e == hipSuccess && defer) {
    c->tail_pending = kind;
    return SGPE_OK;
  }
  if (e == hipSuccess) {
    sgpe::RowArgsT<double> r = ra;
    r.scale = 1.0 / npts;
    if (imag) {
      r.partials = c->partials;
      r.n_partials = col_groups(c);
    }
    e = sgpe::launch_row(r, sgpe::ROW_INV, false, false, c->row_points, s);
  }
  return status_of(e);
}

// The fused schedule of n steps: K(dt/2) [R K(dt)]^(n-1) R K(dt/2), with the normalisation of
// step i applied (as a scale) at the start of the next row pass.
static sgpe_status run_steps_variant(sgpe_ctx* c, int64_t n, bool imag);

sgpe_status run_steps(sgpe_ctx* c, int64_t n, bool imag, std::vector<hipEvent_t>* ev) {
  if (n == 0) return SGPE_OK;
  const bool variant = c->split_order != SGPE_SPLIT_KRK || c->split_rs != SGPE_RSPLIT_FROZEN;
  // K-R-K with R = N L N differs from the default only inside the row pass's R: on a complex64
  // state it runs the fused schedule below with that row pass (and continues across calls)
  const bool krk_nln = c->split_order == SGPE_SPLIT_KRK && c->split_rs == SGPE_RSPLIT_NLN && c->prec != SGPE_C128;
  if (variant && !krk_nln) {
    // the variants complete every call; a tail of the default schedule completes first
    const sgpe_status st = flush_tail(c);
    if (st != SGPE_OK) return st;
  }
  if (c->prec == SGPE_C128) {
    if (ev) return SGPE_ESTATE;
    return run_steps_c128(c, n, imag);
  }
  if (variant) {
    if (ev) return SGPE_ESTATE;
    if (!krk_nln) return run_steps_variant(c, n, imag);
  }
  const int step_mode = krk_nln ? sgpe::ROW_STEP_NLN : sgpe::ROW_STEP;
  const double npts = double(c->p.nx) * double(c->p.ny);
  const float inv_n = float(1.0 / npts);  // exact: a power of two
  hipStream_t s = c->stream;
  hipError_t e;
  RowArgs ra = row_args(c);
  // A tail of the other kind (or any tail before a timed profile) completes first.  A tail of this
  // kind continues: the merged K(dt) below completes the previous call's last step and begins this
  // call's first, exactly as inside one call (in imaginary time its NORM_DOT partials give the
  // norm at that step boundary, and the first row pass rescales by it).
  const int kind = imag ? 2 : 1;
  if (c->tail_pending != 0 && (c->tail_pending != kind || ev)) {
    const sgpe_status st = flush_tail(c);
    if (st != SGPE_OK) return st;
  }
  const bool cont = c->tail_pending == kind;
  c->tail_pending = 0;
  if (cont) {
    e = sgpe::launch_col(col_args(c, imag, false), imag ? sgpe::NORM_DOT : sgpe::NORM_NONE, c->col_iters,
                         c->col_points, s);
  } else {
    e = sgpe::launch_row(ra, sgpe::ROW_FWD, false, false, c->row_iters, c->row_points, s);
    if (e == hipSuccess)
      e = sgpe::launch_col(col_args(c, imag, true), sgpe::NORM_NONE, c->col_iters, c->col_points, s);
  }
  if (e != hipSuccess) return status_of(e);
  // a context on a caller's state buffer, and a timed profile, complete every call
  const bool defer = c->own_psi && !ev;
  size_t evi = 0;
  for (int64_t i = 1; i <= n; ++i) {
    RowArgs r = ra;
    r.scale = inv_n;
    if (imag && (i > 1 || cont)) {
      r.partials = c->partials;
      r.n_partials = col_groups(c);
    }
    if (ev) (void)hipEventRecord((*ev)[evi++], s);
    e = sgpe::launch_row(r, step_mode, imag, c->full2x2, c->row_iters, c->row_points, s);
    if (e != hipSuccess) return status_of(e);
    if (ev) (void)hipEventRecord((*ev)[evi++], s);
    const bool last = (i == n);
    if (last && defer) break;   // the last K(dt/2) and the inverse x-transform wait (flush_tail)
    const int nm = imag ? (last ? sgpe::NORM_SQ : sgpe::NORM_DOT) : sgpe::NORM_NONE;
    e = sgpe::launch_col(col_args(c, imag, last), nm, c->col_iters, c->col_points, s);
    if (e != hipSuccess) return status_of(e);
    if (ev) (void)hipEventRecord((*ev)[evi++], s);
  }
  if (defer) {
    c->tail_pending = kind;
    return SGPE_OK;
  }
  RowArgs r = ra;
  r.scale = inv_n;
  if (imag) {
    r.partials = c->partials;
    r.n_partials = col_groups(c);
  }
  e = sgpe::launch_row(r, sgpe::ROW_INV, false, false, c->row_iters, c->row_points, s);
  return status_of(e);
}

// The tail a step call of the default schedule left (either precision): the last step's K(dt/2)
// (with the imaginary-time norm partials of the finished step) and the inverse x-transform (with
// its rescaling), exactly as the call would have ended.
sgpe_status flush_tail(sgpe_ctx* c) {
  if (c->tail_pending == 0) return SGPE_OK;
  const bool imag = c->tail_pending == 2;
  c->tail_pending = 0;
  const int nm = imag ? sgpe::NORM_SQ : sgpe::NORM_NONE;
  if (c->prec == SGPE_C128) {
    hipError_t e = sgpe::launch_col(col_args_t<double>(c, imag, true), nm, c->col_points, c->stream);
    if (e != hipSuccess) return status_of(e);
    sgpe::RowArgsT<double> r = row_args_t<double>(c, 0.0);
    r.scale = 1.0 / (double(c->p.nx) * double(c->p.ny));
    if (imag) {
      r.partials = c->partials;
      r.n_partials = col_groups(c);
    }
    return status_of(sgpe::launch_row(r, sgpe::ROW_INV, false, false, c->row_points, c->stream));
  }
  hipError_t e = sgpe::launch_col(col_args(c, imag, true), nm, c->col_iters, c->col_points, c->stream);
  if (e != hipSuccess) return status_of(e);
  RowArgs r = row_args(c);
  r.scale = float(1.0 / (double(c->p.nx) * double(c->p.ny)));
  if (imag) {
    r.partials = c->partials;
    r.n_partials = col_groups(c);
  }
  e = sgpe::launch_row(r, sgpe::ROW_INV, false, false, c->row_iters, c->row_points, c->stream);
  return status_of(e);
}

// The R-K-R splitting variants (sgpe_set_splitting), built from the general row pass (K-R-K with
// R as N L N is the fused schedule of run_steps with the ROW_STEP_NLN row pass):
//   R-K-R, real time:       row (R(dt/2), fwd-x); n x [col K(dt); row (inv-x, R(dt/2), R(dt/2), fwd-x)],
//                           the last row pass (inv-x, R(dt/2)) only;
//   R-K-R, imaginary time:  the norm falls between the two R halves, so each step's row work takes
//                           two passes: (inv-x, R(dt/2), norm partials) that stores nothing, then
//                           (inv-x, R(dt/2), scale, R(dt/2), fwd-x).  The second recomputes the
//                           first's R(dt/2) from the same input with the same code, so the partials
//                           belong to exactly the state it rescales, and no intermediate state is
//                           stored (one complex64 rounding fewer per step, and 48 instead of 64 bytes
//                           per point of row traffic).
static sgpe_status run_steps_variant(sgpe_ctx* c, int64_t n, bool imag) {
  if (n == 0) return SGPE_OK;
  const sgpe_params& p = c->p;
  const double npts = double(p.nx) * double(p.ny);
  const float inv_n = float(1.0 / npts);
  const int rs = c->split_rs;
  // the general row pass is built for 256-thread workgroups (512 only at 4096 points)
  const int var_rows = std::min(c->rows, sgpe::row_rows_per_block(p.nx, p.ny, c->row_points, c->max_lds));
  const int row_groups = p.ny / var_rows;
  hipStream_t s = c->stream;
  hipError_t e = hipSuccess;
  auto row = [&](double h, int flags, int nr, const double* parts, int nparts, bool real_space_parts) {
    RowArgs r = row_args(c, h);
    r.rows_per_block = var_rows;
    r.var_flags = flags;
    r.var_r = nr;
    r.var_nln = rs;
    r.scale = (flags & sgpe::VAR_INV) ? inv_n : 1.0f;   // with VAR_MID_SCALE: the inverse's 1/N only
    r.partials = parts;
    r.n_partials = nparts;
    if (real_space_parts) {
      r.parseval_w = (2.0 * p.xmax / p.nx) * (2.0 * p.ymax / p.ny);
      r.inv_npts = 1.0;
    }
    r.partials_out = c->partials;
    if (e == hipSuccess) e = sgpe::launch_row(r, sgpe::ROW_VAR, imag, c->full2x2, 1, c->row_points, s);
  };
  auto col = [&](bool half, int norm_mode) {
    if (e == hipSuccess) e = sgpe::launch_col(col_args(c, imag, half), norm_mode, c->col_iters, c->col_points, s);
  };
  // R-K-R
  const double h = 0.5 * p.dt;
  row(h, sgpe::VAR_FWD, 1, nullptr, 0, false);
  for (int64_t i = 1; i <= n; ++i) {
    col(false, sgpe::NORM_NONE);
    const bool last = (i == n);
    if (!imag) {
      row(h, last ? sgpe::VAR_INV : (sgpe::VAR_INV | sgpe::VAR_FWD), last ? 1 : 2, nullptr, 0, false);
    } else {
      row(h, sgpe::VAR_INV | sgpe::VAR_NORM_OUT | sgpe::VAR_NO_STORE, 1, nullptr, 0, false);
      row(h, sgpe::VAR_INV | sgpe::VAR_MID_SCALE | (last ? 0 : sgpe::VAR_FWD), last ? 1 : 2, c->partials, row_groups,
          true);
    }
  }
  return status_of(e);
}

EnergyArgs energy_args(const sgpe_ctx* c, double* row_partials, double* col_partials) {
  const sgpe_params& p = c->p;
  EnergyArgs a{};
  a.psi = c->psi;
  a.psi64 = c->psi64;
  a.nx = p.nx;
  a.ny = p.ny;
  a.norm0 = p.norm0;
  a.result = nullptr;
  a.rows = sgpe::energy_rows_per_block(p.nx, p.ny);
  a.cols = sgpe::energy_cols_per_block(p.nx, p.ny, c->max_lds);
  a.twx = c->twp64_x;
  a.twy = c->twp64_y;
  a.xmin = -p.xmax;
  a.dx = 2.0 * p.xmax / p.nx;
  a.ymin = -p.ymax;
  a.dy = 2.0 * p.ymax / p.ny;
  a.wx2h = 0.5 * p.wx * p.wx;
  a.wy2h = 0.5 * p.wy * p.wy;
  a.delta = p.delta;
  a.g_uu = p.g_uu;
  a.g_dd = p.g_dd;
  a.g_ud = p.g_ud;
  a.k_l = p.k_l;
  a.omega = p.omega;
  a.om_x = c->full2x2 ? c->omx : nullptr;
  a.om_y = c->full2x2 ? c->omy : nullptr;
  a.dkx = M_PI / p.xmax;
  a.dky = M_PI / p.ymax;
  a.row_partials = row_partials;
  a.col_partials = col_partials;
  return a;
}

sgpe_status check_ctx_no_flush(sgpe_ctx* c) {
  if (!c) return SGPE_EINVAL;
  if (hipSetDevice(c->device) != hipSuccess) {
    (void)hipGetLastError();
    return SGPE_EDEVICE;
  }
  return SGPE_OK;
}

sgpe_status check_ctx(sgpe_ctx* c) {
  const sgpe_status st = check_ctx_no_flush(c);
  return st != SGPE_OK ? st : flush_tail(c);
}

sgpe_status latched_status(sgpe_ctx* c) {
  if (c->status_host && __atomic_load_n(c->status_host, __ATOMIC_ACQUIRE) != 0u) c->latched = SGPE_ENONFINITE;
  return c->latched;
}

sgpe_status sync_and_latch(sgpe_ctx* c) {
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return SGPE_EDEVICE;
  }
  return latched_status(c);
}

sgpe_status fetch_partials(sgpe_ctx* c, const double* dev, size_t n, const double** host) {
  *host = nullptr;
  if (n > c->host_part_n) {
    // the old buffer may still be the destination of a queued copy
    if (hipStreamSynchronize(c->stream) != hipSuccess) {
      (void)hipGetLastError();
      return SGPE_EDEVICE;
    }
    if (c->host_part) (void)hipHostFree(c->host_part);
    c->host_part = nullptr;
    c->host_part_n = 0;
    void* ptr = nullptr;
    if (hipHostMalloc(&ptr, n * sizeof(double), hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return SGPE_ENOMEM;
    }
    c->host_part = static_cast<double*>(ptr);
    c->host_part_n = n;
  }
  if (hipMemcpyAsync(c->host_part, dev, n * sizeof(double), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    (void)hipGetLastError();
    return SGPE_EDEVICE;
  }
  *host = c->host_part;
  return SGPE_OK;
}

}  // namespace sgpe_host

using namespace sgpe_host;

extern "C" {

sgpe_status sgpe_validate_params(const sgpe_params* p) {
  if (!p) return SGPE_EINVAL;
  if (!is_pow2(p->nx) || !is_pow2(p->ny)) return SGPE_EINVAL;
  if (p->nx < kMinN || p->ny < kMinN || p->nx > kMaxN || p->ny > kMaxN) return SGPE_EINVAL;
  const double vals[] = {p->xmax, p->ymax, p->g_uu, p->g_dd, p->g_ud, p->k_l, p->omega, p->delta,
                         p->wx, p->wy, p->omega_r0, p->omega_rw, p->dt, p->norm0};
  for (double v : vals)
    if (!is_finite(v)) return SGPE_EINVAL;
  if (!(p->xmax > 0.0) || !(p->ymax > 0.0)) return SGPE_EINVAL;
  if (!(p->dt > 0.0) || !(p->norm0 > 0.0)) return SGPE_EINVAL;
  if (p->wx < 0.0 || p->wy < 0.0) return SGPE_EINVAL;
  if (p->omega_r0 != 0.0 && !(p->omega_rw > 0.0)) return SGPE_EINVAL;
  return SGPE_OK;
}

int32_t sgpe_device_count(void) {
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return -int32_t(e);
  }
  return n;
}

const char* sgpe_strerror(sgpe_status s) {
  switch (s) {
    case SGPE_OK: return "success";
    case SGPE_EINVAL: return "invalid argument";
    case SGPE_ENOMEM: return "out of device memory or grid too large";
    case SGPE_EDEVICE: return "no usable gfx950 device or HIP runtime error";
    case SGPE_ENONFINITE: return "non-finite value in the state";
    case SGPE_ESTATE: return "call not valid in the current state";
  }
  return "unknown status";
}

// Columns per column-pass tile for complex128: at most 4, 256 threads where one column allows it,
// within the LDS (double2 slots take twice the bytes); at 8 points per lane also at least as many
// workgroups as compute units where one column allows it (measured at 256^2 and 512^2: 1 and 2
// columns, 90.8k and 48.3k imaginary steps/s, against 88.5k and 44.2k for 2 and 1).
static int c128_cols(int nx, int ny, int points, int n_cu, size_t max_lds) {
  int c = 4;
  while (c > 1 && (2 * c * (ny / points) > 256 || c > nx || nx % c != 0 ||
                   !sgpe::schedule_supported(ny, c, 1, points) ||
                   sgpe::col_lds_bytes_c128(ny, c, points) > max_lds || (points == 8 && nx / c < n_cu)))
    c >>= 1;
  return c;
}

static int c128_rows(const sgpe_ctx* c, int points) {
  // one row per workgroup where a row takes at least one wave (measured: 29.1 -> 27.5 us per
  // imaginary step at 512^2, 64.3 -> 63.8 at 1024^2, unchanged at 2048^2), else the derived tile
  const sgpe_params& p = c->p;
  return p.nx / points >= 32 ? 1 : sgpe::row_rows_per_block(p.nx, p.ny, points, c->max_lds / 2);
}

// 8 points per lane where the length allows it, 16 beyond.  An fp64 lane at 16 points holds 64
// registers of points and more of roots (over 200 in all, two waves per SIMD, the column kernel
// spilling); at 8 it runs about 1.1-1.5x the steps/s (1024^2: 17.6k -> 19.3k imaginary, 16.1k ->
// 21.7k real; 512^2: 37.3k -> 48.3k; 256^2: 61.7k -> 90.8k imaginary steps/s).
static void default_schedule_c128(sgpe_ctx* c) {
  const int rp = c->p.nx <= sgpe::kMaxNSmallP ? 8 : 16;
  const int cp = c->p.ny <= sgpe::kMaxNSmallP ? 8 : 16;
  c->rows = c128_rows(c, rp);
  c->cols = c128_cols(c->p.nx, c->p.ny, cp, c->n_cu, c->max_lds);
  c->row_points = rp;
  c->col_points = cp;
  c->row_iters = c->col_iters = 1;
}

// complex128 schedules: 16 or 8 points per lane in each pass (8 for lengths up to kMaxNSmallP),
// one row group / column tile per workgroup, at most 256 threads per workgroup unless one line
// alone needs 512, double2 LDS slots within the device's LDS.
static sgpe_status apply_schedule_c128(sgpe_ctx* c, const sgpe_schedule& s) {
  const sgpe_params& p = c->p;
  auto points_ok = [](int pts, int n) { return pts == 16 || (pts == 8 && n <= sgpe::kMaxNSmallP); };
  auto bound = [](int n, int pts) { return 2 * n / pts > 256 ? 512 : 256; };
  if (!points_ok(s.row_points, p.nx) || !points_ok(s.col_points, p.ny)) return SGPE_EINVAL;
  if (s.row_iters != 1 || s.col_iters != 1 || s.row_tile < 0 || s.col_tile < 1) return SGPE_EINVAL;
  const int rows = s.row_tile > 0 ? s.row_tile : c128_rows(c, s.row_points);
  if (rows > p.ny || p.ny % rows != 0 || !sgpe::schedule_supported(p.nx, rows, 1, s.row_points) ||
      2 * rows * (p.nx / s.row_points) > bound(p.nx, s.row_points) ||
      2 * sgpe::row_lds_bytes(p.nx, rows) > c->max_lds)
    return SGPE_EINVAL;
  const int cols = s.col_tile;
  if (cols > p.nx || p.nx % cols != 0 || !sgpe::schedule_supported(p.ny, cols, 1, s.col_points) ||
      2 * cols * (p.ny / s.col_points) > bound(p.ny, s.col_points) ||
      sgpe::col_lds_bytes_c128(p.ny, cols, s.col_points) > c->max_lds)
    return SGPE_EINVAL;
  c->rows = rows;
  c->cols = cols;
  c->row_points = s.row_points;
  c->col_points = s.col_points;
  c->row_iters = c->col_iters = 1;
  return SGPE_OK;
}

sgpe_status sgpe_create(const sgpe_params* p, void* hip_stream, void* psi_dev, sgpe_ctx** out) {
  return sgpe_create_ex(p, SGPE_C64, hip_stream, psi_dev, out);
}

sgpe_status sgpe_create_ex(const sgpe_params* p, int32_t precision, void* hip_stream, void* psi_dev, sgpe_ctx** out) {
  if (!out) return SGPE_EINVAL;
  *out = nullptr;
  if (precision != SGPE_C64 && precision != SGPE_C128) return SGPE_EINVAL;
  sgpe_status st = sgpe_validate_params(p);
  if (st != SGPE_OK) return st;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    return SGPE_EDEVICE;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return SGPE_EDEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return SGPE_EDEVICE;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return SGPE_EDEVICE;
  if (psi_dev && (reinterpret_cast<uintptr_t>(psi_dev) & 15u) != 0) return SGPE_EINVAL;

  sgpe_ctx* c = new (std::nothrow) sgpe_ctx();
  if (!c) return SGPE_ENOMEM;
  c->p = *p;
  c->device = dev;
  c->stream = static_cast<hipStream_t>(hip_stream);
  // the kernels' static LDS (reduction scratch) is < 256 bytes
  c->max_lds = prop.sharedMemPerBlock > 256 ? size_t(prop.sharedMemPerBlock) - 256 : 0;
  c->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 1;
  c->prec = precision;
  default_schedule(c);
  const bool c128 = precision == SGPE_C128;
  if (c128) default_schedule_c128(c);
  c->full2x2 = (p->omega_r0 != 0.0);
  const size_t wb = c128 ? 2 : 1;   // LDS bytes per slot relative to complex64
  const size_t col_lds = c128 ? sgpe::col_lds_bytes_c128(p->ny, c->cols, c->col_points) : sgpe::col_lds_bytes(p->ny, c->cols);
  if (wb * sgpe::row_lds_bytes(p->nx, c->rows) > c->max_lds || col_lds > c->max_lds ||
      !sgpe::energy_fits(p->nx, p->ny, c->max_lds)) {
    delete c;
    return SGPE_ENOMEM;
  }

  const size_t npts = size_t(p->nx) * size_t(p->ny);
  auto fail = [&](sgpe_status s) {
    sgpe_destroy(c);
    return s;
  };
  const size_t state_bytes = npts * (c128 ? sizeof(double4) : sizeof(float4));
  void* state = psi_dev;
  if (!state) {
    if ((st = dev_alloc(c, &state, state_bytes)) != SGPE_OK) return fail(st);
    c->own_psi = true;
  }
  if (c128) c->psi64 = static_cast<double4*>(state);
  else c->psi = static_cast<float4*>(state);
  if ((st = upload(c, &c->twp64_x, twiddles_plain<double>(p->nx))) != SGPE_OK) return fail(st);
  if ((st = upload(c, &c->twp64_y, twiddles_plain<double>(p->ny))) != SGPE_OK) return fail(st);
  if (!c128) {
    if ((st = upload(c, &c->twp_x, twiddles_plain(p->nx))) != SGPE_OK) return fail(st);
    if ((st = upload(c, &c->twp_y, twiddles_plain(p->ny))) != SGPE_OK) return fail(st);
  }
  for (int imag = 0; imag < 2; ++imag) {
    for (int half = 0; half < 2; ++half) {
      const int idx = 2 * imag + half;
      const double h = half ? 0.5 * p->dt : p->dt;
      if (c128) {
        std::vector<double4> kx;
        std::vector<double2> ky;
        k_tables<double>(*p, imag != 0, h, kx, ky);
        if ((st = upload(c, &c->kx64[idx], kx)) != SGPE_OK) return fail(st);
        if ((st = upload(c, &c->ky64[idx], ky)) != SGPE_OK) return fail(st);
      } else {
        std::vector<float4> kx;
        std::vector<float2> ky;
        k_tables(*p, imag != 0, h, kx, ky);
        if ((st = upload(c, &c->kx_tab[idx], kx)) != SGPE_OK) return fail(st);
        if ((st = upload(c, &c->ky_tab[idx], ky)) != SGPE_OK) return fail(st);
      }
    }
  }
  if (c->full2x2) {
    std::vector<double> om(p->nx);
    const double dx = 2.0 * p->xmax / p->nx;
    for (int j = 0; j < p->nx; ++j) om[j] = p->omega_r0 * std::tanh((-p->xmax + dx * j) / p->omega_rw);
    if ((st = raman_tables(c, om.data(), nullptr)) != SGPE_OK) return fail(st);
  }
  void* ptr = nullptr;
  if ((st = dev_alloc(c, &ptr, kMaxPartials * sizeof(double))) != SGPE_OK) return fail(st);
  c->partials = static_cast<double*>(ptr);
  if ((st = dev_alloc(c, &ptr, (sgpe::kEnergyRowParts * size_t(kMaxN) + kMaxPartials) * sizeof(double))) !=
      SGPE_OK)
    return fail(st);
  c->epart = static_cast<double*>(ptr);
  if ((st = dev_alloc(c, &ptr, sgpe::norm_blocks() * sizeof(double))) != SGPE_OK) return fail(st);
  c->npart = static_cast<double*>(ptr);
  {
    void* hptr = nullptr;
    void* dptr = nullptr;
    if (hipHostMalloc(&hptr, sizeof(unsigned int), hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
      (void)hipGetLastError();
      return fail(SGPE_ENOMEM);
    }
    c->status_host = static_cast<unsigned int*>(hptr);
    *c->status_host = 0u;
    if (hipHostGetDevicePointer(&dptr, hptr, 0) != hipSuccess) {
      (void)hipGetLastError();
      return fail(SGPE_EDEVICE);
    }
    c->status_dev = static_cast<unsigned int*>(dptr);
  }
  *out = c;
  return SGPE_OK;
}

void sgpe_destroy(sgpe_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  for (void* ptr : c->allocations) (void)hipFree(ptr);
  if (c->host_part) (void)hipHostFree(c->host_part);
  if (c->status_host) (void)hipHostFree(c->status_host);
  if (c->relax_host) (void)hipHostFree(c->relax_host);
  for (hipEvent_t ev : c->relax_ev)
    if (ev) (void)hipEventDestroy(ev);
  (void)hipGetLastError();
  delete c;
}

sgpe_status sgpe_set_col_tile(sgpe_ctx* c, int32_t columns) {
  if (!c || c->prec == SGPE_C128) return SGPE_EINVAL;
  if (const sgpe_status st = check_ctx(c); st != SGPE_OK) return st;   // the pending tail, old schedule
  if (columns == 0) {
    default_schedule(c);
    return SGPE_OK;
  }
  const sgpe_params& p = c->p;
  if (columns < 1) return SGPE_EINVAL;
  int iters = c->col_iters;
  if (!sgpe::col_cols_supported(p.nx, p.ny, columns, iters, c->col_points, c->max_lds)) iters = 1;
  if (!sgpe::col_cols_supported(p.nx, p.ny, columns, iters, c->col_points, c->max_lds)) return SGPE_EINVAL;
  c->cols = columns;
  c->col_iters = iters;
  return SGPE_OK;
}

sgpe_status sgpe_get_schedule(sgpe_ctx* c, sgpe_schedule* out) {
  if (!c || !out) return SGPE_EINVAL;
  *out = get_schedule(c);
  return SGPE_OK;
}

sgpe_status sgpe_set_schedule(sgpe_ctx* c, const sgpe_schedule* s) {
  if (!c) return SGPE_EINVAL;
  if (const sgpe_status st = check_ctx(c); st != SGPE_OK) return st;   // the pending tail, old schedule
  if (c->prec == SGPE_C128) {
    if (!s) {
      default_schedule_c128(c);
      return SGPE_OK;
    }
    return apply_schedule_c128(c, *s);
  }
  if (!s) {
    default_schedule(c);
    return SGPE_OK;
  }
  return apply_schedule(c, *s);
}

sgpe_status sgpe_set_psi(sgpe_ctx* c, const double* h) {
  sgpe_status st = check_ctx_no_flush(c);
  if (st != SGPE_OK) return st;
  if (!h) return SGPE_EINVAL;
  const size_t nx = size_t(c->p.nx), ny = size_t(c->p.ny), npts = nx * ny;
  for (size_t i = 0; i < 4 * npts; ++i)
    if (!std::isfinite(h[i])) return SGPE_ENONFINITE;
  const double* up = h;
  const double* dn = h + 2 * npts;
  hipError_t e;
  if (c->prec == SGPE_C128) {
    std::vector<double4> buf(npts);
    for (size_t i = 0; i < npts; ++i) buf[i] = make_double4(up[2 * i], up[2 * i + 1], dn[2 * i], dn[2 * i + 1]);
    e = hipMemcpyAsync(c->psi64, buf.data(), npts * sizeof(double4), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  } else {
    std::vector<float4> buf(npts);
    for (size_t i = 0; i < npts; ++i)
      buf[i] = make_float4(float(up[2 * i]), float(up[2 * i + 1]), float(dn[2 * i]), float(dn[2 * i + 1]));
    e = hipMemcpyAsync(c->psi, buf.data(), npts * sizeof(float4), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return SGPE_EDEVICE;
  }
  c->has_state = true;
  c->tail_pending = 0;
  c->latched = SGPE_OK;
  if (c->status_host) __atomic_store_n(c->status_host, 0u, __ATOMIC_RELEASE);   // the stream is idle
  return SGPE_OK;
}

sgpe_status sgpe_set_psi_device(sgpe_ctx* c, const void* d) {
  sgpe_status st = check_ctx(c);   // a pending tail completes: d may be the state buffer itself
  if (st != SGPE_OK) return st;
  if (!d || reinterpret_cast<uintptr_t>(d) % 16 != 0) return SGPE_EINVAL;
  const long long npts = (long long)c->p.nx * c->p.ny;
  const int nb = sgpe::norm_blocks();
  const bool c128 = c->prec == SGPE_C128;
  hipError_t e = c128 ? sgpe::launch_nonfinite(static_cast<const double4*>(d), npts, c->npart, nb, c->stream)
                      : sgpe::launch_nonfinite(static_cast<const float4*>(d), npts, c->npart, nb, c->stream);
  if (e != hipSuccess) return status_of(e);
  const double* part = nullptr;
  if ((st = fetch_partials(c, c->npart, size_t(nb), &part)) != SGPE_OK) return st;   // synchronises
  double bad = 0.0;
  for (int b = 0; b < nb; ++b) bad += part[b];
  if (bad != 0.0) return SGPE_ENONFINITE;   // the state is unchanged
  // the stream is idle: no step kernel can set the status word any more
  if (c->status_host) __atomic_store_n(c->status_host, 0u, __ATOMIC_RELEASE);
  void* dst = c128 ? static_cast<void*>(c->psi64) : static_cast<void*>(c->psi);
  const size_t bytes = size_t(npts) * (c128 ? sizeof(double4) : sizeof(float4));
  e = dst == d ? hipSuccess : hipMemcpyAsync(dst, d, bytes, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return SGPE_EDEVICE;
  }
  c->has_state = true;
  c->tail_pending = 0;
  c->latched = SGPE_OK;
  return SGPE_OK;
}

sgpe_status sgpe_get_psi(sgpe_ctx* c, double* h) {
  sgpe_status st = check_ctx(c);
  if (st != SGPE_OK) return st;
  if (!h) return SGPE_EINVAL;
  if (!c->has_state) return SGPE_ESTATE;
  const size_t npts = size_t(c->p.nx) * size_t(c->p.ny);
  bool ok = true;
  double* up = h;
  double* dn = h + 2 * npts;
  auto unpack = [&](const auto& buf) {
    for (size_t i = 0; i < npts; ++i) {
      const auto w = buf[i];
      up[2 * i] = w.x;
      up[2 * i + 1] = w.y;
      dn[2 * i] = w.z;
      dn[2 * i + 1] = w.w;
      ok = ok && std::isfinite(w.x) && std::isfinite(w.y) && std::isfinite(w.z) && std::isfinite(w.w);
    }
  };
  hipError_t e;
  if (c->prec == SGPE_C128) {
    std::vector<double4> buf(npts);
    e = hipMemcpyAsync(buf.data(), c->psi64, npts * sizeof(double4), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) unpack(buf);
  } else {
    std::vector<float4> buf(npts);
    e = hipMemcpyAsync(buf.data(), c->psi, npts * sizeof(float4), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) unpack(buf);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return SGPE_EDEVICE;
  }
  if (!ok) c->latched = SGPE_ENONFINITE;
  return latched_status(c);
}

static sgpe_status step_common(sgpe_ctx* c, int64_t n, bool imag) {
  sgpe_status st = check_ctx_no_flush(c);
  if (st != SGPE_OK) return st;
  if (n < 0) return SGPE_EINVAL;
  if (!c->has_state) return SGPE_ESTATE;
  return run_steps(c, n, imag, nullptr);
}

sgpe_status sgpe_step_real(sgpe_ctx* c, int64_t n) { return step_common(c, n, false); }
sgpe_status sgpe_step_imag(sgpe_ctx* c, int64_t n) { return step_common(c, n, true); }

sgpe_status sgpe_synchronize(sgpe_ctx* c) {
  sgpe_status st = check_ctx(c);
  if (st != SGPE_OK) return st;
  return sync_and_latch(c);
}

sgpe_status sgpe_norm(sgpe_ctx* c, double* out) {
  sgpe_status st = check_ctx(c);
  if (st != SGPE_OK) return st;
  if (!out) return SGPE_EINVAL;
  if (!c->has_state) return SGPE_ESTATE;
  const long long npts = (long long)c->p.nx * c->p.ny;
  const int nb = sgpe::norm_blocks();
  hipError_t e = c->prec == SGPE_C128 ? sgpe::launch_norm(c->psi64, npts, c->npart, nb, c->stream)
                                      : sgpe::launch_norm(c->psi, npts, c->npart, nb, c->stream);
  if (e != hipSuccess) return status_of(e);
  const double* part = nullptr;
  if ((st = fetch_partials(c, c->npart, size_t(nb), &part)) != SGPE_OK) return st;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[b];
  const double dx = 2.0 * c->p.xmax / c->p.nx, dy = 2.0 * c->p.ymax / c->p.ny;
  *out = dx * dy * s;
  if (!std::isfinite(*out)) c->latched = SGPE_ENONFINITE;
  return latched_status(c);
}

sgpe_status sgpe_set_splitting(sgpe_ctx* c, int32_t order, int32_t real_space) {
  if (!c) return SGPE_EINVAL;
  if (const sgpe_status st = check_ctx(c); st != SGPE_OK) return st;   // the pending tail, old scheme
  if ((order != SGPE_SPLIT_KRK && order != SGPE_SPLIT_RKR) ||
      (real_space != SGPE_RSPLIT_FROZEN && real_space != SGPE_RSPLIT_NLN))
    return SGPE_EINVAL;
  if (c->prec == SGPE_C128 && (order != SGPE_SPLIT_KRK || real_space != SGPE_RSPLIT_FROZEN)) return SGPE_EINVAL;
  const int row_groups = c->p.ny / std::min(c->rows, sgpe::row_rows_per_block(c->p.nx, c->p.ny, c->row_points,
                                                                               c->max_lds));
  if (order == SGPE_SPLIT_RKR && row_groups > kMaxPartials) return SGPE_EINVAL;
  c->split_order = order;
  c->split_rs = real_space;
  return SGPE_OK;
}

sgpe_status sgpe_energy(sgpe_ctx* c, double* out) {
  sgpe_status st = check_ctx(c);
  if (st != SGPE_OK) return st;
  if (!out) return SGPE_EINVAL;
  if (!c->has_state) return SGPE_ESTATE;
  const sgpe_params& p = c->p;
  const size_t npts = size_t(p.nx) * size_t(p.ny);
  const double dx = 2.0 * p.xmax / p.nx, dy = 2.0 * p.ymax / p.ny;
  const int nrb = p.ny / sgpe::energy_rows_per_block(p.nx, p.ny);   // row blocks
  constexpr int RP = sgpe::kEnergyRowParts;
  EnergyArgs a = energy_args(c, c->epart, c->epart + RP * nrb);
  const int ncb = p.nx / a.cols;
  hipError_t e = sgpe::launch_energy(a, c->stream);
  if (e != hipSuccess) return status_of(e);
  const double* part = nullptr;
  if ((st = fetch_partials(c, c->epart, RP * size_t(nrb) + ncb, &part)) != SGPE_OK) return st;
  double er = 0.0, ei = 0.0, nr = 0.0, ek = 0.0;
  for (int b = 0; b < nrb; ++b) {
    er += part[RP * b];
    ei += part[RP * b + 1];
    nr += part[RP * b + 2];
  }
  for (int b = 0; b < ncb; ++b) ek += part[RP * nrb + b];
  // per particle of the state rescaled to norm0: quadratic terms over the norm, the interaction
  // (quartic) terms over norm^2 / norm0
  const double w = dx * dy;
  const double nrm = w * nr;
  *out = (w / double(npts) * ek + w * er) / nrm + w * ei * p.norm0 / (nrm * nrm);
  if (!std::isfinite(*out)) c->latched = SGPE_ENONFINITE;
  return latched_status(c);
}

sgpe_status sgpe_profile_steps(sgpe_ctx* c, int32_t imag, int64_t n, double* row_ms, double* col_ms) {
  sgpe_status st = check_ctx(c);
  if (st != SGPE_OK) return st;
  if (n <= 0) return SGPE_EINVAL;
  if (!c->has_state || c->split_order != SGPE_SPLIT_KRK || c->split_rs != SGPE_RSPLIT_FROZEN ||
      c->prec == SGPE_C128)
    return SGPE_ESTATE;
  std::vector<hipEvent_t> ev(3 * size_t(n));
  for (auto& x : ev) {
    if (hipEventCreate(&x) != hipSuccess) {
      (void)hipGetLastError();
      return SGPE_EDEVICE;
    }
  }
  st = run_steps(c, n, imag != 0, &ev);
  if (st == SGPE_OK) st = sync_and_latch(c);
  double tr = 0.0, tc = 0.0;
  if (st == SGPE_OK) {
    for (int64_t i = 0; i < n; ++i) {
      float a = 0.f, b = 0.f;
      (void)hipEventElapsedTime(&a, ev[3 * i], ev[3 * i + 1]);
      (void)hipEventElapsedTime(&b, ev[3 * i + 1], ev[3 * i + 2]);
      tr += a;
      tc += b;
    }
  }
  for (auto& x : ev) (void)hipEventDestroy(x);
  if (st != SGPE_OK) return st;
  if (row_ms) *row_ms = tr / double(n);
  if (col_ms) *col_ms = tc / double(n);
  return SGPE_OK;
}

sgpe_status sgpe_profile_kernels(sgpe_ctx* c, int32_t imag, int64_t n, double* row_ms, double* col_ms) {
  sgpe_status st = check_ctx(c);
  if (st != SGPE_OK) return st;
  if (n <= 0) return SGPE_EINVAL;
  if (!c->has_state || c->split_order != SGPE_SPLIT_KRK || c->split_rs != SGPE_RSPLIT_FROZEN ||
      c->prec == SGPE_C128)
    return SGPE_ESTATE;
  const sgpe_params& p = c->p;
  const size_t bytes = size_t(p.nx) * size_t(p.ny) * sizeof(float4);
  if (!c->scratch) {
    void* ptr = nullptr;
    if ((st = dev_alloc(c, &ptr, bytes)) != SGPE_OK) return st;
    c->scratch = static_cast<float4*>(ptr);
  }
  hipEvent_t ev[4];
  int made = 0;
  for (; made < 4; ++made) {
    if (hipEventCreate(&ev[made]) != hipSuccess) break;
  }
  hipStream_t s = c->stream;
  hipError_t e = made == 4 ? hipSuccess : hipErrorOutOfMemory;
  // keep the state; enter the mixed representation with valid norm partials
  if (e == hipSuccess) e = hipMemcpyAsync(c->scratch, c->psi, bytes, hipMemcpyDeviceToDevice, s);
  RowArgs ra = row_args(c);
  if (e == hipSuccess) e = sgpe::launch_row(ra, sgpe::ROW_FWD, false, false, c->row_iters, c->row_points, s);
  const int steady_norm = imag ? sgpe::NORM_DOT : sgpe::NORM_NONE;
  if (e == hipSuccess) e = sgpe::launch_col(col_args(c, imag != 0, true), sgpe::NORM_DOT, c->col_iters, c->col_points, s);
  RowArgs r = ra;
  r.scale = float(1.0 / (double(p.nx) * double(p.ny)));
  if (imag) {
    r.partials = c->partials;
    r.n_partials = col_groups(c);
  }
  const ColArgs ca = col_args(c, imag != 0, false);
  if (e == hipSuccess) e = hipEventRecord(ev[0], s);
  for (int64_t i = 0; i < n && e == hipSuccess; ++i) e = sgpe::launch_row(r, sgpe::ROW_STEP, imag != 0, c->full2x2, c->row_iters, c->row_points, s);
  if (e == hipSuccess) e = hipEventRecord(ev[1], s);
  if (e == hipSuccess) e = hipEventRecord(ev[2], s);
  for (int64_t i = 0; i < n && e == hipSuccess; ++i) e = sgpe::launch_col(ca, steady_norm, c->col_iters, c->col_points, s);
  if (e == hipSuccess) e = hipEventRecord(ev[3], s);
  if (e == hipSuccess) e = hipMemcpyAsync(c->psi, c->scratch, bytes, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  float a = 0.f, b = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&a, ev[0], ev[1]);
  if (e == hipSuccess) e = hipEventElapsedTime(&b, ev[2], ev[3]);
  for (int i = 0; i < made; ++i) (void)hipEventDestroy(ev[i]);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return status_of(e);
  }
  if (row_ms) *row_ms = double(a) / double(n);
  if (col_ms) *col_ms = double(b) / double(n);
  return latched_status(c);
}

}  // extern "C"
