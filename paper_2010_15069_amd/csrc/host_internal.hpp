// Host-side internals shared by the single-instance API (api.cpp) and the batch API (batch.cpp):
// the context of one solver instance and the helpers that build its launch arguments.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "sgpe.h"
#include "sgpe_internal.hpp"

// One solver instance: its parameters, device buffers and tables, and its launch schedule.
struct sgpe_ctx {
  sgpe_params p{};
  int device = 0;
  hipStream_t stream = nullptr;
  float4* psi = nullptr;
  bool own_psi = false;
  float4* scratch = nullptr;
  float4* twp_x = nullptr;  // fp32-rounded roots with modulus corrections (step kernels)
  float4* twp_y = nullptr;
  // K tables, index = 2*imag + half  (half: h = dt/2, else h = dt)
  float4* kx_tab[4] = {nullptr, nullptr, nullptr, nullptr};
  float2* ky_tab[4] = {nullptr, nullptr, nullptr, nullptr};
  // spatial Raman coupling Omega_x(x) + Omega_y(y), only with one (full2x2):
  float* hbx = nullptr;     // dt * Omega_x(x_j) / 2
  float* hby = nullptr;     // dt * Omega_y(y_i) / 2
  double* omx = nullptr;    // Omega_x(x_j) (energy)
  double* omy = nullptr;    // Omega_y(y_i)
  double* partials = nullptr;
  double* epart = nullptr;  // energy partials (row: 2 per block, then col: 1 per block)
  double* npart = nullptr;  // norm partials
  size_t max_lds = 0;       // dynamic LDS bytes available per workgroup
  int rows = 1;             // rows per row-pass workgroup
  int cols = 1;             // columns per column-pass workgroup
  int row_iters = 1;        // row groups per row-pass workgroup (the next one prefetched)
  int col_iters = 1;        // column tiles per column-pass workgroup
  int row_points = 16;      // points per lane of the x transforms
  int col_points = 16;      // points per lane of the y transforms
  int n_cu = 1;             // compute units of the device
  // complex128 contexts (prec == SGPE_C128): the state and the step tables in fp64; psi and the
  // fp32 tables are then unused (the schedule fields above apply, with no prefetch)
  int prec = 0;             // sgpe_precision
  double4* psi64 = nullptr;
  double4* twp64_x = nullptr;  // fp64 roots (every context: the energy kernels transform in fp64)
  double4* twp64_y = nullptr;
  double4* kx64[4] = {nullptr, nullptr, nullptr, nullptr};
  double2* ky64[4] = {nullptr, nullptr, nullptr, nullptr};
  double* hbx64 = nullptr;  // dt * Omega_x(x_j) / 2
  double* hby64 = nullptr;  // dt * Omega_y(y_i) / 2
  double4* scratch_q64 = nullptr;  // staging of complex128 inputs (annealing noise)
  bool full2x2 = false;
  int split_order = 0;      // sgpe_split_order
  int split_rs = 0;         // sgpe_real_space_split
  bool has_state = false;
  sgpe_status latched = SGPE_OK;
  // status word the step kernels set when an imaginary-time norm is not finite and positive:
  // fine-grained pinned host memory, mapped into the device's address space
  unsigned int* status_host = nullptr;
  unsigned int* status_dev = nullptr;
  std::vector<void*> allocations;
  double* host_part = nullptr;   // pinned host copy of reduction partials, grown on demand
  size_t host_part_n = 0;
  // A step call of the default schedule (either precision) on a state the context owns leaves its last
  // step's K(dt/2) and the inverse x-transform pending (1: real time, 2: imaginary time, 0: none);
  // the next step call of the same kind merges them with its own first K(dt/2), and every other
  // entry point completes them first (flush_tail, from check_ctx).
  int tail_pending = 0;
  // sgpe_relax_imag's ring of energy checks in flight (allocated on its first call): the energies
  // on the device, their pinned host copies, and an event after each copy
  double* relax_dev = nullptr;
  double* relax_host = nullptr;
  hipEvent_t relax_ev[4] = {nullptr, nullptr, nullptr, nullptr};
};

namespace sgpe {
// Per workgroup of nblocks (sgpe::norm_blocks()), the count of points of psi (npts, device memory)
// with a non-finite value, as doubles in partials.
hipError_t launch_nonfinite(const float4* psi, long long npts, double* partials, int nblocks, hipStream_t s);
hipError_t launch_nonfinite(const double4* psi, long long npts, double* partials, int nblocks, hipStream_t s);
}  // namespace sgpe

namespace sgpe_host {

constexpr int kMaxPartials = 4096;   // norm partials per column pass (one per workgroup)

sgpe_status dev_alloc(sgpe_ctx* c, void** ptr, size_t bytes);
sgpe_status status_of(hipError_t e);
void default_schedule(sgpe_ctx* c);
int default_points(int n, size_t npts);   // points per lane for a transform of length n, npts points in all
int col_groups(const sgpe_ctx* c);
sgpe_status apply_schedule(sgpe_ctx* c, const sgpe_schedule& s);   // validated; EINVAL changes nothing
sgpe_schedule get_schedule(const sgpe_ctx* c);
// Row-pass arguments with the real-space coefficients of a sub-step h (h <= 0: h = dt).
sgpe::RowArgs row_args(const sgpe_ctx* c, double h = 0.0);
sgpe::ColArgs col_args(const sgpe_ctx* c, bool imag, bool half);
// Validates the context and makes its device current, then completes a pending step tail, so
// that the state is in its documented layout: every entry point but the step calls uses this one.
sgpe_status check_ctx(sgpe_ctx* c);
// The same without completing the pending tail (the step calls, which may merge it).
sgpe_status check_ctx_no_flush(sgpe_ctx* c);
// Enqueue the pending step tail, if any (see sgpe_ctx::tail_pending).
sgpe_status flush_tail(sgpe_ctx* c);
// Arguments of the energy kernels for the context's state, with the given partial buffers
// (kEnergyRowParts per row block, then one per column block).
sgpe::EnergyArgs energy_args(const sgpe_ctx* c, double* row_partials, double* col_partials);
// Copies n doubles of reduction partials from the device into the context's pinned host buffer
// (queued on the context's stream, which is then synchronised) and points *host at it.  Returns
// SGPE_ENOMEM if the buffer cannot grow, SGPE_EDEVICE on a device error.  A pinned destination
// avoids the staging copy of pageable memory.
sgpe_status fetch_partials(sgpe_ctx* c, const double* dev, size_t n, const double** host);
// Spatial Raman coupling tables Omega_x(x_j) + Omega_y(y_i) (NULL = zero profile), allocated on first
// use; waits for the stream's queued work before overwriting them.
sgpe_status raman_tables(sgpe_ctx* c, const double* om_x, const double* om_y);
sgpe_status sync_and_latch(sgpe_ctx* c);
// Enqueue n >= 0 steps of the context's scheme (imaginary time if imag) on its stream; with ev, a
// HIP event pair around every pass (the default scheme in complex64 only).
sgpe_status run_steps(sgpe_ctx* c, int64_t n, bool imag, std::vector<hipEvent_t>* ev);
// The context's latched status after the stream has been synchronised: folds in the status word
// the step kernels set on a non-finite norm.
sgpe_status latched_status(sgpe_ctx* c);

}  // namespace sgpe_host
