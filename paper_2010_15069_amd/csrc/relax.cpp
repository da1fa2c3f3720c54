// sgpe_relax_imag: a ground state by imaginary-time propagation, run until an energy rule is met.
// Propagation in imaginary time approaches the ground state asymptotically, with the atom number
// restored after every step (Sec. 3.2); the spin-Hall ground states of Sec. 6 are found this way.
// The paper fixes no stopping rule; the two rules here are the library's.
//
// The call enqueues chunks of check_every steps, each followed by an energy check: the energy
// kernels, their device-side combination (launch_energy_finish) into a slot of a small device ring,
// an asynchronous copy of that one double into pinned host memory, and an event.  The host reads
// check k while the chunks of checks k+1 .. k+kAhead are already queued behind it, so the device
// does not wait for the host between chunks, and each check costs the energy kernels' own time
// rather than a drained queue.  The price: when check k meets the rule, the queued chunks still run
// (at most kAhead * check_every further steps, which in imaginary time move the state further
// toward the ground state); the result reports both counts.
#include "sgpe.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "host_internal.hpp"
#include "sgpe_internal.hpp"

namespace {

constexpr int kRing = 4;     // device / pinned slots (kAhead + 1 of them are ever in use)
constexpr int64_t kAhead = 2;

static_assert(kAhead + 1 <= kRing, "a slot is reused only after its check has been read");

// The ring (device slots, pinned copies, events), allocated on the first call and kept by the
// context.
sgpe_status relax_buffers(sgpe_ctx* c) {
  if (c->relax_dev) return SGPE_OK;
  for (hipEvent_t& ev : c->relax_ev) {
    if (!ev && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      ev = nullptr;
      return SGPE_EDEVICE;
    }
  }
  if (!c->relax_host) {
    void* h = nullptr;
    if (hipHostMalloc(&h, kRing * sizeof(double), hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return SGPE_ENOMEM;
    }
    c->relax_host = static_cast<double*>(h);
  }
  void* d = nullptr;
  const sgpe_status st = sgpe_host::dev_alloc(c, &d, kRing * sizeof(double));
  if (st != SGPE_OK) return st;
  c->relax_dev = static_cast<double*>(d);
  return SGPE_OK;
}

// The energy check of the state as the stream leaves it, into ring slot `slot`.
hipError_t enqueue_check(sgpe_ctx* c, const sgpe::EnergyArgs& a, int slot) {
  hipError_t e = sgpe::launch_energy(a, c->stream);
  if (e == hipSuccess) e = sgpe::launch_energy_finish(a, c->relax_dev + slot, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->relax_host + slot, c->relax_dev + slot, sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipEventRecord(c->relax_ev[slot], c->stream);
  return e;
}

}  // namespace

extern "C" sgpe_status sgpe_relax_imag(sgpe_ctx* c, int64_t check_every, int64_t max_steps, int32_t rule,
                                       double target, double tol, double* energies, int64_t energies_cap,
                                       sgpe_relax_result* out) {
  sgpe_status st = sgpe_host::check_ctx(c);
  if (st != SGPE_OK) return st;
  // (k check_every stays below 2^63 for every check k up to max_steps / check_every + 1)
  constexpr int64_t kMaxCount = int64_t(1) << 61;
  if (!out || check_every < 1 || max_steps < 0 || check_every > kMaxCount || max_steps > kMaxCount ||
      !std::isfinite(tol) || tol < 0.0 || energies_cap < 0 ||
      (energies_cap > 0 && !energies) || (rule != SGPE_RELAX_TARGET && rule != SGPE_RELAX_DELTA) ||
      (rule == SGPE_RELAX_TARGET && !std::isfinite(target)))
    return SGPE_EINVAL;
  if (!c->has_state) return SGPE_ESTATE;
  if ((st = relax_buffers(c)) != SGPE_OK) return st;
  *out = sgpe_relax_result{};
  out->energy = out->energy_prev = std::nan("");

  const sgpe::EnergyArgs a = sgpe_host::energy_args(c, c->epart, c->epart + sgpe::kEnergyRowParts * c->p.ny);
  // check k is taken after min(k check_every, max_steps) steps; check 0 is the start state
  const int64_t n_checks = 1 + (max_steps + check_every - 1) / check_every;
  auto steps_at = [&](int64_t k) { return std::min(k * check_every, max_steps); };
  int64_t queued = 0;   // checks enqueued so far
  auto enqueue = [&]() -> sgpe_status {
    const int64_t k = queued;
    if (k > 0) {
      sgpe_status s = sgpe_host::run_steps(c, steps_at(k) - steps_at(k - 1), true, nullptr);
      if (s == SGPE_OK) s = sgpe_host::flush_tail(c);   // the check reads the completed state
      if (s != SGPE_OK) return s;
    }
    const hipError_t e = enqueue_check(c, a, int(k % kRing));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return sgpe_host::status_of(e);
    }
    ++queued;
    return SGPE_OK;
  };

  sgpe_status err = SGPE_OK;
  double e_prev = std::nan("");
  for (int64_t k = 0; k < n_checks && err == SGPE_OK; ++k) {
    while (queued < n_checks && queued <= k + kAhead && err == SGPE_OK) err = enqueue();
    if (err != SGPE_OK) break;
    const int slot = int(k % kRing);
    if (hipEventSynchronize(c->relax_ev[slot]) != hipSuccess) {
      (void)hipGetLastError();
      err = SGPE_EDEVICE;
      break;
    }
    const double e = c->relax_host[slot];
    if (k < energies_cap) energies[k] = e;
    out->checks = k + 1;
    out->steps = steps_at(k);
    out->energy = e;
    out->energy_prev = e_prev;
    if (!std::isfinite(e)) {
      c->latched = SGPE_ENONFINITE;
      break;
    }
    const bool met = rule == SGPE_RELAX_TARGET ? std::fabs(e - target) <= tol * std::fabs(target)
                                               : (k > 0 && std::fabs(e - e_prev) < tol * std::fabs(e));
    if (met) {
      out->met = 1;
      break;
    }
    e_prev = e;
  }
  out->steps_taken = queued > 0 ? steps_at(queued - 1) : 0;
  const sgpe_status sync = sgpe_host::sync_and_latch(c);
  return err != SGPE_OK ? err : sync;
}
