// sgpe_energy_noalloc: the energy of sgpe_energy with no allocation at call time, for callers that
// cannot allocate (code under HIP graph capture, tight serving loops, harnesses that forbid it).
//
// sgpe_energy writes the energy kernels' partial sums to a device buffer the context allocated and
// brings them back through a pinned host buffer it grows on demand.  Here they live in one static
// device array, `scratch`, of a fixed size: kEnergyRowParts per row block and one per column block,
// for up to kMaxAxis of each (every grid the library accepts).  Each device the library runs on holds
// its own copy until the process ends.  Host code never passes the array's
// name to a kernel or a copy: on a device's first call the address of that device's copy is looked
// up (hipGetSymbolAddress, with the device current) and kept, and only that address is used.  The
// finishing kernel of the energy (launch_energy_finish) sums the partials in a fixed order and
// writes the energy to the caller's device memory, so the call is asynchronous on the context's
// stream and never synchronises.
//
// Every call on a device shares that device's array and leaves its contents behind; the energy
// kernels overwrite every partial the finishing kernel later reads, so nothing needs clearing
// between calls.  Calls that overlap on one device (two streams, or two threads) race on
// the array and must be ordered by the caller.
#include <hip/hip_runtime.h>

#include <mutex>

#include "fft_device.hpp"
#include "host_internal.hpp"
#include "sgpe.h"
#include "sgpe_internal.hpp"

namespace {

constexpr size_t kMaxAxis = 4096;
// kEnergyRowParts partials per row block, then one per column block
constexpr size_t kScratchDoubles = sgpe::kEnergyRowParts * kMaxAxis + kMaxAxis;
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

std::mutex g_mu;
double* g_scratch[kMaxDevices] = {};

// The address of this device's copy of `scratch`, looked up once per device with it current.
double* device_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch[device] = static_cast<double*>(p);
  }
  return g_scratch[device];
}

}  // namespace

extern "C" sgpe_status sgpe_energy_noalloc(sgpe_ctx* c, double* e_dev) {
  sgpe_status st = sgpe_host::check_ctx(c);   // makes the context's device current
  if (st != SGPE_OK) return st;
  if (!e_dev) return SGPE_EINVAL;
  if (!c->has_state) return SGPE_ESTATE;
  const sgpe_params& p = c->p;
  double* base = device_scratch(c->device);
  if (!base) return SGPE_EDEVICE;
  constexpr int RP = sgpe::kEnergyRowParts;
  double* row_parts = base;
  double* col_parts = row_parts + RP * kMaxAxis;
  const sgpe::EnergyArgs a = sgpe_host::energy_args(c, row_parts, col_parts);
  const int nrows = p.ny / a.rows, ncols = p.nx / a.cols;
  if (size_t(nrows) > kMaxAxis || size_t(ncols) > kMaxAxis) return SGPE_ENOMEM;   // beyond the static array
  hipError_t e = sgpe::launch_energy(a, c->stream);
  if (e == hipSuccess) e = sgpe::launch_energy_finish(a, e_dev, c->stream);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return sgpe_host::status_of(e);
  }
  return SGPE_OK;
}
