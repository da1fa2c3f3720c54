// Host side of the spin-Hall pieces (Sec. 6) of the C ABI declared in include/sgpe.h: the spatial
// Raman coupling profile, the annealing update, and the observables (phase separation, population
// radius, circulation).  The kernels are in observables.hip.
#include "sgpe.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "host_internal.hpp"
#include "sgpe_internal.hpp"

using namespace sgpe_host;

extern "C" {

sgpe_status sgpe_set_raman_profile(sgpe_ctx* c, const double* omega_x, const double* omega_y) {
  sgpe_status st = check_ctx(c);
  if (st != SGPE_OK) return st;
  const sgpe_params& p = c->p;
  if (omega_x)
    for (int j = 0; j < p.nx; ++j)
      if (!std::isfinite(omega_x[j])) return SGPE_EINVAL;
  if (omega_y)
    for (int i = 0; i < p.ny; ++i)
      if (!std::isfinite(omega_y[i])) return SGPE_EINVAL;
  if (hipStreamSynchronize(c->stream) != hipSuccess) {
    (void)hipGetLastError();
    return SGPE_EDEVICE;
  }
  if (!omega_x && !omega_y) {
    c->full2x2 = false;
    return SGPE_OK;
  }
  if ((st = raman_tables(c, omega_x, omega_y)) != SGPE_OK) return st;
  c->full2x2 = true;
  return SGPE_OK;
}

// Copies nblocks * per_block partials from c->epart to the host and sums each slot in block order.
static sgpe_status fetch_sums(sgpe_ctx* c, int nblocks, int per_block, double* sums) {
  const double* part = nullptr;
  const sgpe_status st = fetch_partials(c, c->epart, size_t(nblocks) * per_block, &part);
  if (st != SGPE_OK) return st;
  for (int k = 0; k < per_block; ++k) sums[k] = 0.0;
  for (int b = 0; b < nblocks; ++b)
    for (int k = 0; k < per_block; ++k) sums[k] += part[size_t(b) * per_block + k];
  return SGPE_OK;
}

sgpe_status sgpe_add_noise(sgpe_ctx* c, const double* xi, double amplitude) {
  sgpe_status st = check_ctx(c);
  if (st != SGPE_OK) return st;
  if (!xi || !std::isfinite(amplitude)) return SGPE_EINVAL;
  if (!c->has_state) return SGPE_ESTATE;
  const size_t npts = size_t(c->p.nx) * size_t(c->p.ny);
  for (size_t i = 0; i < 4 * npts; ++i)
    if (!std::isfinite(xi[i])) return SGPE_ENONFINITE;
  const double* up = xi;
  const double* dn = xi + 2 * npts;
  hipError_t e;
  if (c->prec == SGPE_C128) {
    if (!c->scratch_q64) {
      void* ptr = nullptr;
      if ((st = dev_alloc(c, &ptr, npts * sizeof(double4))) != SGPE_OK) return st;
      c->scratch_q64 = static_cast<double4*>(ptr);
    }
    std::vector<double4> buf(npts);
    for (size_t i = 0; i < npts; ++i) buf[i] = make_double4(up[2 * i], up[2 * i + 1], dn[2 * i], dn[2 * i + 1]);
    e = hipMemcpyAsync(c->scratch_q64, buf.data(), npts * sizeof(double4), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = sgpe::launch_add_noise(c->psi64, c->scratch_q64, amplitude, (long long)npts, c->stream);
    if (hipStreamSynchronize(c->stream) != hipSuccess) e = hipErrorUnknown;   // buf must outlive the copy
  } else {
    if (!c->scratch) {
      void* ptr = nullptr;
      if ((st = dev_alloc(c, &ptr, npts * sizeof(float4))) != SGPE_OK) return st;
      c->scratch = static_cast<float4*>(ptr);
    }
    std::vector<float4> buf(npts);
    for (size_t i = 0; i < npts; ++i)
      buf[i] = make_float4(float(up[2 * i]), float(up[2 * i + 1]), float(dn[2 * i]), float(dn[2 * i + 1]));
    e = hipMemcpyAsync(c->scratch, buf.data(), npts * sizeof(float4), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = sgpe::launch_add_noise(c->psi, c->scratch, float(amplitude), (long long)npts, c->stream);
    if (hipStreamSynchronize(c->stream) != hipSuccess) e = hipErrorUnknown;   // buf must outlive the copy
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return SGPE_EDEVICE;
  }
  return latched_status(c);
}

sgpe_status sgpe_phase_separation(sgpe_ctx* c, double* out) {
  sgpe_status st = check_ctx(c);
  if (st != SGPE_OK) return st;
  if (!out) return SGPE_EINVAL;
  if (!c->has_state) return SGPE_ESTATE;
  const long long npts = (long long)c->p.nx * c->p.ny;
  const int nb = sgpe::norm_blocks();
  hipError_t e = c->prec == SGPE_C128 ? sgpe::launch_moments(c->psi64, npts, c->epart, nb, c->stream)
                                      : sgpe::launch_moments(c->psi, npts, c->epart, nb, c->stream);
  if (e != hipSuccess) return status_of(e);
  double m[sgpe::kMomentParts];
  if ((st = fetch_sums(c, nb, sgpe::kMomentParts, m)) != SGPE_OK) return st;
  if (!std::isfinite(m[0] + m[1] + m[2])) {
    c->latched = SGPE_ENONFINITE;
    return latched_status(c);
  }
  if (!(m[1] > 0.0) || !(m[2] > 0.0)) return SGPE_ESTATE;
  *out = 1.0 - m[0] / std::sqrt(m[1] * m[2]);
  return latched_status(c);
}

static sgpe_status disk_population(sgpe_ctx* c, double r2, double* out) {
  const sgpe_params& p = c->p;
  const double dx = 2.0 * p.xmax / p.nx, dy = 2.0 * p.ymax / p.ny;
  const int nb = sgpe::norm_blocks();
  hipError_t e =
      c->prec == SGPE_C128
          ? sgpe::launch_disk_population(c->psi64, p.nx, p.ny, -p.xmax, dx, -p.ymax, dy, r2, c->epart, nb, c->stream)
          : sgpe::launch_disk_population(c->psi, p.nx, p.ny, -p.xmax, dx, -p.ymax, dy, r2, c->epart, nb, c->stream);
  if (e != hipSuccess) return status_of(e);
  return fetch_sums(c, nb, 1, out);
}

sgpe_status sgpe_population_radius(sgpe_ctx* c, double fraction, double* radius) {
  sgpe_status st = check_ctx(c);
  if (st != SGPE_OK) return st;
  if (!radius || !(fraction > 0.0 && fraction <= 1.0)) return SGPE_EINVAL;
  if (!c->has_state) return SGPE_ESTATE;
  const sgpe_params& p = c->p;
  double total = 0.0;
  if ((st = disk_population(c, HUGE_VAL, &total)) != SGPE_OK) return st;
  if (!std::isfinite(total)) {
    c->latched = SGPE_ENONFINITE;
    return latched_status(c);
  }
  if (!(total > 0.0)) return SGPE_ESTATE;
  const double target = fraction * total;
  // every grid point lies within the corner radius, so the disc of radius hi holds everything
  double lo = 0.0, hi = std::sqrt(p.xmax * p.xmax + p.ymax * p.ymax);
  for (int it = 0; it < 200 && hi - lo > 1e-12 * hi; ++it) {
    const double mid = 0.5 * (lo + hi);
    double inside = 0.0;
    if ((st = disk_population(c, mid * mid, &inside)) != SGPE_OK) return st;
    if (inside >= target) hi = mid;
    else lo = mid;
  }
  *radius = hi;
  return latched_status(c);
}

sgpe_status sgpe_winding(sgpe_ctx* c, double radius, int32_t* n, double* raw) {
  sgpe_status st = check_ctx(c);
  if (st != SGPE_OK) return st;
  const sgpe_params& p = c->p;
  if (!n || !(radius > 0.0 && radius < std::min(p.xmax, p.ymax))) return SGPE_EINVAL;
  if (!c->has_state) return SGPE_ESTATE;
  const double d = std::min(2.0 * p.xmax / p.nx, 2.0 * p.ymax / p.ny);
  const double mm = std::ceil(4.0 * M_PI * radius / d);
  const int m = mm < 256.0 ? 256 : int(mm);
  hipError_t e = c->prec == SGPE_C128
                     ? sgpe::launch_winding(c->psi64, p.nx, p.ny, p.xmax, p.ymax, radius, m, c->epart, c->stream)
                     : sgpe::launch_winding(c->psi, p.nx, p.ny, p.xmax, p.ymax, radius, m, c->epart, c->stream);
  if (e != hipSuccess) return status_of(e);
  double w[2];
  if ((st = fetch_sums(c, 1, 2, w)) != SGPE_OK) return st;
  if (!std::isfinite(w[0]) || !std::isfinite(w[1])) {
    c->latched = SGPE_ENONFINITE;
    return latched_status(c);
  }
  n[0] = int32_t(std::lround(w[0]));
  n[1] = int32_t(std::lround(w[1]));
  if (raw) {
    raw[0] = w[0];
    raw[1] = w[1];
  }
  return latched_status(c);
}

}  // extern "C"
