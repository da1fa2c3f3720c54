// Host side of the measurement probe declared in include/sgpe.h (sgpe_probe_exchange).
#include <hip/hip_runtime.h>

#include "sgpe.h"
#include "sgpe_internal.hpp"

namespace {

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

}  // namespace

extern "C" sgpe_status sgpe_probe_exchange(int32_t nx, int32_t ny, int32_t layout_rows, int32_t row_tile,
                                           int32_t col_tile, int32_t write_through, int32_t reps, double* row_ms,
                                           double* col_ms) {
  if (!pow2(nx) || !pow2(ny) || !pow2(layout_rows) || !pow2(row_tile) || !pow2(col_tile) || reps < 1)
    return SGPE_EINVAL;
  if (nx < 16 || ny < 16 || nx > 4096 || ny > 4096 || layout_rows > 8 || ny / 16 < layout_rows ||
      ny % layout_rows != 0 || row_tile > ny || col_tile > nx)
    return SGPE_EINVAL;
  if (2 * row_tile * (nx / 16) > 1024 || 2 * col_tile * (ny / 16) > 1024) return SGPE_EINVAL;
  const size_t bytes = size_t(nx) * size_t(ny) * sizeof(float4);
  void* a = nullptr;
  void* b = nullptr;
  if (hipMalloc(&a, bytes) != hipSuccess || hipMalloc(&b, bytes) != hipSuccess) {
    (void)hipGetLastError();
    if (a) (void)hipFree(a);
    return SGPE_ENOMEM;
  }
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipError_t e = hipEventCreate(&ev[0]);
  if (e == hipSuccess) e = hipEventCreate(&ev[1]);
  if (e == hipSuccess) e = hipMemset(a, 0, bytes);
  if (e == hipSuccess) e = hipMemset(b, 0, bytes);
  double tr = 0.0, tc = 0.0;
  auto* A = static_cast<float4*>(a);
  auto* B = static_cast<float4*>(b);
  const bool wt = write_through != 0;
  // one warm-up round, then reps timed rounds of (row partition A -> B, column partition B -> A)
  for (int i = 0; i <= reps && e == hipSuccess; ++i) {
    float ms = 0.f;
    e = hipEventRecord(ev[0], nullptr);
    if (e == hipSuccess) e = sgpe::launch_probe_rows(A, B, nx, ny, layout_rows, row_tile, wt, nullptr);
    if (e == hipSuccess) e = hipEventRecord(ev[1], nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
    if (i > 0) tr += ms;
    if (e == hipSuccess) e = hipEventRecord(ev[0], nullptr);
    if (e == hipSuccess) e = sgpe::launch_probe_cols(B, A, nx, ny, layout_rows, col_tile, wt, nullptr);
    if (e == hipSuccess) e = hipEventRecord(ev[1], nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
    if (i > 0) tc += ms;
  }
  if (e != hipSuccess) (void)hipGetLastError();
  for (hipEvent_t x : ev)
    if (x) (void)hipEventDestroy(x);
  (void)hipFree(a);
  (void)hipFree(b);
  if (e != hipSuccess) return SGPE_EDEVICE;
  if (row_ms) *row_ms = tr / reps;
  if (col_ms) *col_ms = tc / reps;
  return SGPE_OK;
}
