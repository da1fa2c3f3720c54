// Persistent step kernel for batched parameter sweeps: every steady-state step of every instance of
// a batch in one cooperative launch.
//
// A batch's instances (any mix of grids with 128, 256 or 512 points per axis, diagonal real-space
// operator) are cut into work items of 1024 points per component: a row item is 1024 / nx rows of
// one instance, a column item 1024 / ny columns.  Each item runs in a 256-thread workgroup at 8 points
// per lane, with the same device bodies (row_body, col_body) and the same per-instance arguments
// as the single-instance and per-class launches, so every instance computes exactly what a single
// context with that schedule computes.  The steps of the split step (Sec. 3.2's K(dt/2) R(dt) K(dt/2)
// with the adjacent K halves merged) alternate a row phase (inverse x-FFT, scale, R(dt), forward
// x-FFT for every row item) and a column phase (forward y-FFT, K(dt) and the imaginary-time norm
// partials, inverse y-FFT for every column item), with a barrier after each phase.
//
// The workgroups stay resident for the whole launch.  They form eight groups by blockIdx.x mod 8:
// the dispatcher deals a launch's workgroups to the eight XCDs in turn, so a group is the
// workgroups of one XCD (which one depends on where its rotation stood).  Every instance belongs to one group and is stepped by that group's workgroups alone, so the
// all-to-all between the row and the column phase of its transforms stays within one L2, and a
// barrier joins one group's workgroups only; groups never wait for each other.  Correctness does
// not depend on where a group runs: the barrier counts the group's workgroups, whatever their XCD.
//
// The barrier: after a workgroup's __syncthreads, its first thread makes the workgroup's writes
// visible device-wide (an agent-scope release fence; the state stores go through the L2 as they are
// issued), adds one to its group's counter and waits until the counter reaches the phase's target,
// then takes an agent-scope acquire fence so that its reads see every other workgroup's writes.  The wait is bounded:
// after spin_limit polls a workgroup gives up, sets an abort word that every waiting workgroup also
// polls, records the failure in host-visible memory and returns; every workgroup then leaves at its
// next barrier, and the host reports SGPE_EDEVICE.  A small kernel zeroes the counters and the abort
// word before each launch (graph-replay safe).
#include "col_body.hpp"
#include "row_body.hpp"

namespace sgpe {

// Bounded wait until *w reaches `target` (wrap-safe); false if the wait gave up or another
// workgroup's did.
__device__ __forceinline__ bool persist_wait(const PersistArgs& a, const unsigned* w, unsigned target) {
  for (unsigned spin = 0;; ++spin) {
    const unsigned v = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (static_cast<int>(v - target) >= 0) return true;
    if (__hip_atomic_load(a.barrier + kPersistAbortWord, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)
      return false;
    if (spin >= a.spin_limit) {
      __hip_atomic_store(a.barrier + kPersistAbortWord, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(a.abort_host, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

// Barrier number `nb` (1, 2, ...) of the launch among the workgroups of this one's group.
__device__ __forceinline__ bool persist_barrier(const PersistArgs& a, unsigned nb) {
  __shared__ int ok_s;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned grp = blockIdx.x % kPersistGroups;
    const unsigned members = (gridDim.x - grp + kPersistGroups - 1) / kPersistGroups;
    unsigned* count = a.barrier + kPersistWordStride * grp;
    // release before arriving, acquire after the wait: on this part an agent-scope release is an L2
    // write-back and an acquire an L2 invalidate, so a full fence on both sides would do each twice
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const bool ok = persist_wait(a, count, members * nb);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    ok_s = ok ? 1 : 0;
  }
  __syncthreads();
  return ok_s != 0;
}

// One class's workgroups (in one group) run all the launch's steps of that class's instances in the
// group with the body of its grid size, so only that body's per-lane constants are live in them;
// every workgroup of the group meets at every barrier (one beyond its class's share takes no items).
template <int N, bool IMAG>
__device__ __forceinline__ void persist_class(const PersistArgs& a, const PersistClass& k, int local) {
  constexpr int NORM = IMAG ? NORM_DOT : NORM_NONE;
  const int first = local < k.wg_count ? local : k.n_row + k.n_col;   // past every item: idle
  unsigned nb = 0;
  for (int s = 0; s < a.steps; ++s) {
    const RowArgs* rows = (s == 0 && a.first_is_first) ? a.row_first : a.row_step;
    for (int i = first; i < k.n_row; i += k.wg_count) {
      const int4 it = a.row_items[k.row_begin + i];
      row_body<N, ROW_STEP, IMAG, false, 1, 8, true>(rows[it.x], it.y);
      __syncthreads();
    }
    if (!persist_barrier(a, ++nb)) return;
    for (int i = first; i < k.n_col; i += k.wg_count) {
      const int4 it = a.col_items[k.col_begin + i];
      col_body<N, NORM, 1, 8, true>(a.col[it.x], it.y, it.w);
      __syncthreads();
    }
    if (!persist_barrier(a, ++nb)) return;
  }
}

// Two waves per SIMD: the three grid sizes' bodies and their item loops need ~219 VGPRs; held to
// 168 for three waves they spill 200 bytes per lane, and the sweep ran at 243k instead of 311k
// instance-steps/s.
template <bool IMAG>
__global__ void __launch_bounds__(256, 2) persist_kernel(PersistArgs a) {
  const int grp = static_cast<int>(blockIdx.x % kPersistGroups);
  const int j = static_cast<int>(blockIdx.x / kPersistGroups);
  const PersistClass* cg = a.cls + grp * kPersistClasses;
  if (cg[0].log2n == 0) return;   // a group without instances: nobody waits for it
  int k = 0;
  while (k + 1 < kPersistClasses && cg[k + 1].log2n != 0 && j >= cg[k + 1].wg_begin) ++k;
  const PersistClass c = cg[k];
  const int local = j - c.wg_begin;
  switch (c.log2n) {
    case 7: persist_class<128, IMAG>(a, c, local); break;
    case 8: persist_class<256, IMAG>(a, c, local); break;
    default: persist_class<512, IMAG>(a, c, local); break;
  }
}

__global__ void persist_reset_kernel(unsigned* words) {
  for (int i = threadIdx.x; i < kPersistWords; i += blockDim.x)
    __hip_atomic_store(words + i, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

hipError_t persist_max_grid(bool imag, int n_cu, int* grid) {
  int per_cu = 0;
  const size_t lds = persist_lds_bytes();
  hipError_t e = imag ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persist_kernel<true>, 256, lds)
                      : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persist_kernel<false>, 256, lds);
  if (e != hipSuccess) return e;
  *grid = per_cu * n_cu;
  return *grid > 0 ? hipSuccess : hipErrorInvalidConfiguration;
}

hipError_t launch_persist(const PersistArgs& a, bool imag, int grid, hipStream_t s) {
  hipLaunchKernelGGL(persist_reset_kernel, dim3(1), dim3(256), 0, s, a.barrier);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  PersistArgs args = a;
  void* params[] = {&args};
  const void* fn = imag ? reinterpret_cast<const void*>(persist_kernel<true>)
                        : reinterpret_cast<const void*>(persist_kernel<false>);
  return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(256), params, persist_lds_bytes(), s);
}

// Row items of 1024 / nx rows and column items of 1024 / ny columns at 8 points per lane: both
// 17408 bytes of exchange slots, plus the column pass's k_y row is not staged at 8 points per lane.
size_t persist_lds_bytes() { return row_lds_bytes(512, 2); }

}  // namespace sgpe
