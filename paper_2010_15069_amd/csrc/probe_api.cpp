// Host side of the measurement probes declared in include/sgpe.h (sgpe_probe_exchange,
// sgpe_probe_placement).
#include <hip/hip_runtime.h>

#include <vector>

#include "sgpe.h"
#include "sgpe_internal.hpp"

namespace {

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

}  // namespace

extern "C" sgpe_status sgpe_probe_exchange(int32_t nx, int32_t ny, int32_t layout_rows, int32_t row_tile,
                                           int32_t col_tile, int32_t flags, int32_t reps, double* row_ms,
                                           double* col_ms, double* pair_ms) {
  const bool wt = (flags & SGPE_PROBE_WRITE_THROUGH) != 0;
  const bool wl = (flags & SGPE_PROBE_WAVE_LOCAL) != 0;
  if ((flags & ~(SGPE_PROBE_WRITE_THROUGH | SGPE_PROBE_WAVE_LOCAL)) != 0) return SGPE_EINVAL;
  if (!pow2(nx) || !pow2(ny) || !pow2(layout_rows) || !pow2(row_tile) || !pow2(col_tile) || reps < 1 || reps > 100000)
    return SGPE_EINVAL;
  if (layout_rows > 8 || ny % layout_rows != 0) return SGPE_EINVAL;
  if (wl) {
    // a wave per line: lengths 512..2048, 1..8 waves per workgroup
    if (nx < 512 || nx > 2048 || ny < 512 || ny > 2048 || row_tile > 8 || col_tile > 8) return SGPE_EINVAL;
  } else {
    if (nx < 16 || ny < 16 || nx > 4096 || ny > 4096 || ny / 16 < layout_rows || row_tile > ny || col_tile > nx)
      return SGPE_EINVAL;
    if (2 * row_tile * (nx / 16) > 1024 || 2 * col_tile * (ny / 16) > 1024) return SGPE_EINVAL;
  }
  const size_t bytes = size_t(nx) * size_t(ny) * sizeof(float4);
  void* a = nullptr;
  void* b = nullptr;
  if (hipMalloc(&a, bytes) != hipSuccess || hipMalloc(&b, bytes) != hipSuccess) {
    (void)hipGetLastError();
    if (a) (void)hipFree(a);
    return SGPE_ENOMEM;
  }
  auto* A = static_cast<float4*>(a);
  auto* B = static_cast<float4*>(b);
  auto rows = [&](const float4* src, float4* dst) {
    return wl ? sgpe::launch_probe_rows_wl(src, dst, nx, ny, layout_rows, row_tile, wt, nullptr)
              : sgpe::launch_probe_rows(src, dst, nx, ny, layout_rows, row_tile, wt, nullptr);
  };
  auto cols = [&](const float4* src, float4* dst) {
    return wl ? sgpe::launch_probe_cols_wl(src, dst, nx, ny, layout_rows, col_tile, wt, nullptr)
              : sgpe::launch_probe_cols(src, dst, nx, ny, layout_rows, col_tile, wt, nullptr);
  };
  std::vector<hipEvent_t> ev(2 * size_t(reps) + 3, nullptr);
  hipError_t e = hipSuccess;
  for (auto& x : ev)
    if (e == hipSuccess) e = hipEventCreate(&x);
  if (e == hipSuccess) e = hipMemset(a, 0, bytes);
  if (e == hipSuccess) e = hipMemset(b, 0, bytes);
  // one untimed round; then reps rounds of (row partition A -> B, column partition B -> A) with an
  // event after every launch (queued, no host wait in between); then the same reps rounds between
  // one event pair
  if (e == hipSuccess) e = rows(A, B);
  if (e == hipSuccess) e = cols(B, A);
  if (e == hipSuccess) e = hipEventRecord(ev[0], nullptr);
  for (int i = 0; i < reps && e == hipSuccess; ++i) {
    e = rows(A, B);
    if (e == hipSuccess) e = hipEventRecord(ev[2 * i + 1], nullptr);
    if (e == hipSuccess) e = cols(B, A);
    if (e == hipSuccess) e = hipEventRecord(ev[2 * i + 2], nullptr);
  }
  const size_t last = 2 * size_t(reps) + 1;
  for (int i = 0; i < reps && e == hipSuccess; ++i) {
    e = rows(A, B);
    if (e == hipSuccess) e = cols(B, A);
  }
  if (e == hipSuccess) e = hipEventRecord(ev[last], nullptr);
  if (e == hipSuccess) e = hipEventSynchronize(ev[last]);
  double tr = 0.0, tc = 0.0, tp = 0.0;
  for (int i = 0; i < reps && e == hipSuccess; ++i) {
    float r = 0.f, c = 0.f;
    e = hipEventElapsedTime(&r, ev[2 * i], ev[2 * i + 1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&c, ev[2 * i + 1], ev[2 * i + 2]);
    tr += r;
    tc += c;
  }
  if (e == hipSuccess) {
    float p = 0.f;
    e = hipEventElapsedTime(&p, ev[2 * size_t(reps)], ev[last]);
    tp = p;
  }
  if (e != hipSuccess) (void)hipGetLastError();
  (void)hipDeviceSynchronize();
  for (hipEvent_t x : ev)
    if (x) (void)hipEventDestroy(x);
  (void)hipFree(a);
  (void)hipFree(b);
  if (e != hipSuccess) return SGPE_EDEVICE;
  if (row_ms) *row_ms = tr / reps;
  if (col_ms) *col_ms = tc / reps;
  if (pair_ms) *pair_ms = tp / reps;
  return SGPE_OK;
}

extern "C" sgpe_status sgpe_probe_placement(int32_t gx, int32_t gy, int32_t threads, uint32_t* xcd) {
  if (!xcd || gx < 1 || gy < 1 || gy > 65535 || threads < 1 || threads > 1024 ||
      int64_t(gx) * int64_t(gy) > (int64_t(1) << 24))
    return SGPE_EINVAL;
  const size_t n = size_t(gx) * size_t(gy);
  void* d = nullptr;
  if (hipMalloc(&d, n * sizeof(unsigned)) != hipSuccess) {
    (void)hipGetLastError();
    return SGPE_ENOMEM;
  }
  hipError_t e = sgpe::launch_probe_xcc(static_cast<unsigned*>(d), gx, gy, threads, nullptr);
  if (e == hipSuccess) e = hipMemcpy(xcd, d, n * sizeof(unsigned), hipMemcpyDeviceToHost);
  (void)hipFree(d);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return SGPE_EDEVICE;
  }
  return SGPE_OK;
}
