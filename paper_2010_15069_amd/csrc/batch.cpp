// Host side of batched parameter sweeps: many independent instances, any mix of grid shapes,
// stepped together.
//
// Instances of one grid shape and one real-space operator form (diagonal, or full 2x2 with a
// spatial Raman coupling) form a class.  Each pass of a class is one launch over all of its
// members (each member's workgroups on one XCD), the members' arguments read from a device table, so a class of
// small grids fills the device where one instance cannot.  Classes run on streams of their own,
// forked from and joined back to the batch stream, so classes of different sizes overlap.  A
// call's whole launch sequence can be captured once into a HIP graph and replayed.  Each member
// computes exactly what a single context with the same schedule computes (the same kernels body,
// the same arguments, the same order of launches).
#include "sgpe.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <utility>
#include <type_traits>
#include <vector>

#include "host_internal.hpp"
#include "sgpe_internal.hpp"

using sgpe::ColArgs;
using sgpe::RowArgs;
using namespace sgpe_host;

namespace {

// Argument table layout of a class with `count` members.
enum RowVariant { ROWTAB_FWD = 0, ROWTAB_SCALE = 1, ROWTAB_PARTIALS = 2, ROWTAB_N = 3 };
// column variants: index 2 * imag + half (half: the K(dt/2) of a call's first and last step)
constexpr int COLTAB_N = 4;

struct BatchClass {
  int nx = 0, ny = 0;
  bool full2x2 = false;
  std::vector<int> members;
  RowArgs* row_tab = nullptr;   // device, [ROWTAB_N][count]
  ColArgs* col_tab = nullptr;   // device, [COLTAB_N][count]
  sgpe::EnergyArgs* e_tab = nullptr;   // device, [count]: the members' energy arguments
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
};

}  // namespace

struct sgpe_batch {
  int device = 0;
  hipStream_t stream = nullptr;       // the caller's stream (may be the null stream)
  hipStream_t graph_stream = nullptr; // graphs are captured and replayed here, ordered after and
                                      // before the caller's stream by events (the null stream
                                      // cannot be captured)
  std::vector<sgpe_ctx*> inst;
  std::vector<BatchClass> cls;
  hipEvent_t fork = nullptr;
  hipEvent_t enter = nullptr, leave = nullptr;
  bool use_graph = true;
  std::map<std::pair<int64_t, int>, hipGraphExec_t> graphs;  // (steps, imag) -> executable graph
  // persistent mode (sgpe_batch_use_persistent): every steady-state step of every instance in one
  // cooperative launch of the persistent kernel
  bool persistent = false;
  bool persist_graph_ok = true;     // cleared if capturing the cooperative launch fails
  RowArgs* p_row_first = nullptr;   // device, [instances]
  RowArgs* p_row_imag = nullptr;    // device, [instances]: scale from the norm partials
  ColArgs* p_col[2] = {nullptr, nullptr};   // device, [instances]: K(dt), real / imaginary time
  int4* p_row_items = nullptr;
  int4* p_col_items = nullptr;
  sgpe::PersistClass* p_cls_dev = nullptr;   // [kPersistGroups][kPersistClasses]
  unsigned* p_words = nullptr;      // device: the grid barrier's words (sgpe::kPersistWords)
  unsigned* p_abort_host = nullptr; // pinned, mapped: a barrier wait gave up
  unsigned* p_abort_host_dev = nullptr;
  int p_grid = 0;                   // workgroups of the persistent launch (all co-resident)
  unsigned p_spin_limit = sgpe::kPersistSpinLimit;
  // sgpe_batch_energies: every instance's energy on the device, and its pinned host copy
  double* e_dev = nullptr;
  double* e_host = nullptr;
};

namespace {

sgpe_status hip_status(hipError_t e) {
  if (e == hipSuccess) return SGPE_OK;
  (void)hipGetLastError();
  return status_of(e);
}

void drop_graphs(sgpe_batch* b) {
  for (auto& g : b->graphs) (void)hipGraphExecDestroy(g.second);
  b->graphs.clear();
}

// Fill the class's argument tables from its members' contexts (which hold the class schedule).
sgpe_status build_tables(BatchClass& k, const std::vector<sgpe_ctx*>& inst) {
  const size_t n = k.members.size();
  std::vector<RowArgs> rows(ROWTAB_N * n);
  std::vector<ColArgs> cols(COLTAB_N * n);
  for (size_t j = 0; j < n; ++j) {
    const sgpe_ctx* c = inst[k.members[j]];
    const RowArgs a = row_args(c);
    RowArgs sc = a;
    sc.scale = float(1.0 / (double(c->p.nx) * double(c->p.ny)));  // exact: a power of two
    RowArgs pa = sc;
    pa.partials = c->partials;
    pa.n_partials = col_groups(c);
    rows[ROWTAB_FWD * n + j] = a;
    rows[ROWTAB_SCALE * n + j] = sc;
    rows[ROWTAB_PARTIALS * n + j] = pa;
    for (int imag = 0; imag < 2; ++imag)
      for (int half = 0; half < 2; ++half) cols[(2 * imag + half) * n + j] = col_args(c, imag != 0, half != 0);
  }
  if (hipMemcpy(k.row_tab, rows.data(), rows.size() * sizeof(RowArgs), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(k.col_tab, cols.data(), cols.size() * sizeof(ColArgs), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    return SGPE_EDEVICE;
  }
  return SGPE_OK;
}

// The fused schedule of n steps for every member of a class, on stream s (the same launch
// sequence as a single context's).
hipError_t enqueue_class(const sgpe_batch* b, const BatchClass& k, int64_t n, bool imag, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int cnt = int(k.members.size());
  const sgpe_ctx* c0 = b->inst[k.members[0]];
  const RowArgs shape_r = row_args(c0);
  const ColArgs shape_c = col_args(c0, imag, false);
  const int rp = c0->row_points, cp = c0->col_points;
  const RowArgs* t_fwd = k.row_tab + ROWTAB_FWD * cnt;
  const RowArgs* t_sc = k.row_tab + ROWTAB_SCALE * cnt;
  const RowArgs* t_pa = k.row_tab + ROWTAB_PARTIALS * cnt;
  auto ctab = [&](bool half) { return k.col_tab + (2 * int(imag) + int(half)) * cnt; };
  hipError_t e = sgpe::launch_row_batch(shape_r, t_fwd, cnt, sgpe::ROW_FWD, false, false, rp, s);
  if (e == hipSuccess) e = sgpe::launch_col_batch(shape_c, ctab(true), cnt, sgpe::NORM_NONE, cp, s);
  for (int64_t i = 1; i <= n && e == hipSuccess; ++i) {
    e = sgpe::launch_row_batch(shape_r, (imag && i > 1) ? t_pa : t_sc, cnt, sgpe::ROW_STEP, imag, k.full2x2, rp, s);
    const bool last = (i == n);
    const int nm = imag ? (last ? sgpe::NORM_SQ : sgpe::NORM_DOT) : sgpe::NORM_NONE;
    if (e == hipSuccess) e = sgpe::launch_col_batch(shape_c, ctab(last), cnt, nm, cp, s);
  }
  if (e == hipSuccess) e = sgpe::launch_row_batch(shape_r, imag ? t_pa : t_sc, cnt, sgpe::ROW_INV, false, false, rp, s);
  return e;
}

// Persistent mode: per class the call's first x transform and half K, then one cooperative launch
// for steps 1..n-1 of every instance, then per class the last step (its row pass, the half K with
// the final norm) and the last inverse x transform.  The same passes, in the same order per
// instance, as the per-class launches.
hipError_t enqueue_persistent(sgpe_batch* b, int64_t n, bool imag, hipStream_t s) {
  hipError_t e = hipSuccess;
  for (const auto& k : b->cls) {
    const int cnt = int(k.members.size());
    const sgpe_ctx* c0 = b->inst[k.members[0]];
    const RowArgs shape_r = row_args(c0);
    const ColArgs shape_c = col_args(c0, imag, false);
    if (e == hipSuccess)
      e = sgpe::launch_row_batch(shape_r, k.row_tab + ROWTAB_FWD * cnt, cnt, sgpe::ROW_FWD, false, false, 8, s);
    if (e == hipSuccess)
      e = sgpe::launch_col_batch(shape_c, k.col_tab + (2 * int(imag) + 1) * cnt, cnt, sgpe::NORM_NONE, 8, s);
  }
  if (e == hipSuccess && n > 1) {
    sgpe::PersistArgs a{};
    a.row_first = b->p_row_first;
    a.row_step = imag ? b->p_row_imag : b->p_row_first;
    a.col = b->p_col[imag ? 1 : 0];
    a.row_items = b->p_row_items;
    a.col_items = b->p_col_items;
    a.cls = b->p_cls_dev;
    a.steps = int(n - 1);
    a.first_is_first = 1;
    a.barrier = b->p_words;
    a.abort_host = b->p_abort_host_dev;
    a.spin_limit = b->p_spin_limit;
    e = sgpe::launch_persist(a, imag, b->p_grid, s);
  }
  for (const auto& k : b->cls) {
    const int cnt = int(k.members.size());
    const sgpe_ctx* c0 = b->inst[k.members[0]];
    const RowArgs shape_r = row_args(c0);
    const ColArgs shape_c = col_args(c0, imag, false);
    const RowArgs* t_sc = k.row_tab + ROWTAB_SCALE * cnt;
    const RowArgs* t_pa = k.row_tab + ROWTAB_PARTIALS * cnt;
    if (e == hipSuccess)
      e = sgpe::launch_row_batch(shape_r, (imag && n > 1) ? t_pa : t_sc, cnt, sgpe::ROW_STEP, imag, false, 8, s);
    if (e == hipSuccess)
      e = sgpe::launch_col_batch(shape_c, k.col_tab + (2 * int(imag) + 1) * cnt, cnt,
                                 imag ? sgpe::NORM_SQ : sgpe::NORM_NONE, 8, s);
    if (e == hipSuccess)
      e = sgpe::launch_row_batch(shape_r, imag ? t_pa : t_sc, cnt, sgpe::ROW_INV, false, false, 8, s);
  }
  return e;
}

// All classes, each on its own stream, forked from and joined back to stream `origin`.
hipError_t enqueue_all(sgpe_batch* b, int64_t n, bool imag, hipStream_t origin) {
  if (b->persistent) return enqueue_persistent(b, n, imag, origin);
  hipError_t e = hipEventRecord(b->fork, origin);
  for (auto& k : b->cls) {
    if (e == hipSuccess) e = hipStreamWaitEvent(k.stream, b->fork, 0);
    if (e == hipSuccess) e = enqueue_class(b, k, n, imag, k.stream);
    if (e == hipSuccess) e = hipEventRecord(k.done, k.stream);
  }
  for (auto& k : b->cls)
    if (e == hipSuccess) e = hipStreamWaitEvent(origin, k.done, 0);
  return e;
}

sgpe_status run(sgpe_batch* b, int64_t n, bool imag) {
  if (n < 0) return SGPE_EINVAL;
  if (n == 0) return SGPE_OK;
  for (const sgpe_ctx* c : b->inst)
    if (!c->has_state) return SGPE_ESTATE;
  if (hipSetDevice(b->device) != hipSuccess) return hip_status(hipErrorInvalidDevice);
  if (!b->use_graph || (b->persistent && !b->persist_graph_ok)) return hip_status(enqueue_all(b, n, imag, b->stream));
  const auto key = std::make_pair(n, int(imag));
  auto it = b->graphs.find(key);
  if (it == b->graphs.end()) {
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(b->graph_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_status(e);
    hipError_t e2 = enqueue_all(b, n, imag, b->graph_stream);
    e = hipStreamEndCapture(b->graph_stream, &g);
    if (e2 != hipSuccess || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      (void)hipGetLastError();
      if (b->persistent) {
        // the runtime could not capture the cooperative launch: run the call directly from now on
        b->persist_graph_ok = false;
        return hip_status(enqueue_all(b, n, imag, b->stream));
      }
      return hip_status(e2 != hipSuccess ? e2 : e);
    }
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_status(e);
    it = b->graphs.emplace(key, x).first;
  }
  hipError_t e = hipEventRecord(b->enter, b->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(b->graph_stream, b->enter, 0);
  if (e == hipSuccess) e = hipGraphLaunch(it->second, b->graph_stream);
  if (e == hipSuccess) e = hipEventRecord(b->leave, b->graph_stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, b->leave, 0);
  return hip_status(e);
}

bool valid_index(const sgpe_batch* b, int32_t i) { return b && i >= 0 && size_t(i) < b->inst.size(); }
bool valid_class(const sgpe_batch* b, int32_t k) { return b && k >= 0 && size_t(k) < b->cls.size(); }

// Apply one schedule to every member of a class (all or none), then rebuild its tables.
sgpe_status set_class_schedule(sgpe_batch* b, BatchClass& k, const sgpe_schedule& s) {
  if (s.row_iters != 1 || s.col_iters != 1) return SGPE_EINVAL;  // batched launches: one tile per workgroup
  std::vector<sgpe_schedule> old;
  for (int m : k.members) old.push_back(get_schedule(b->inst[m]));
  for (size_t j = 0; j < k.members.size(); ++j) {
    if (apply_schedule(b->inst[k.members[j]], s) != SGPE_OK) {
      for (size_t r = 0; r < j; ++r) (void)apply_schedule(b->inst[k.members[r]], old[r]);
      return SGPE_EINVAL;
    }
  }
  drop_graphs(b);
  return build_tables(k, b->inst);
}

// Default for a class: the single-instance rule applied to the class's total point count.
sgpe_schedule class_default(const sgpe_ctx* c0, size_t members) {
  const size_t total = members * size_t(c0->p.nx) * size_t(c0->p.ny);
  sgpe_schedule s{};   // row_tile 0: the default for the points per lane
  s.row_points = default_points(c0->p.nx, total);
  s.col_points = default_points(c0->p.ny, total);
  s.row_iters = 1;
  s.col_iters = 1;
  s.col_tile = sgpe::col_default_cols(c0->p.nx, c0->p.ny, s.col_points, c0->max_lds);
  return s;
}

}  // namespace

extern "C" {

sgpe_status sgpe_batch_create(const sgpe_params* params, int32_t count, void* hip_stream, sgpe_batch** out) {
  if (!out) return SGPE_EINVAL;
  *out = nullptr;
  if (!params || count < 1 || count > 65535) return SGPE_EINVAL;
  for (int32_t i = 0; i < count; ++i) {
    const sgpe_status st = sgpe_validate_params(&params[i]);
    if (st != SGPE_OK) return st;
  }
  sgpe_batch* b = new (std::nothrow) sgpe_batch();
  if (!b) return SGPE_ENOMEM;
  b->stream = static_cast<hipStream_t>(hip_stream);
  auto fail = [&](sgpe_status s) {
    sgpe_batch_destroy(b);
    return s;
  };
  for (int32_t i = 0; i < count; ++i) {
    sgpe_ctx* c = nullptr;
    const sgpe_status st = sgpe_create(&params[i], hip_stream, nullptr, &c);
    if (st != SGPE_OK) return fail(st);
    b->inst.push_back(c);
  }
  b->device = b->inst[0]->device;
  // classes: same grid shape and the same real-space operator form
  for (int32_t i = 0; i < count; ++i) {
    const sgpe_ctx* c = b->inst[i];
    auto it = std::find_if(b->cls.begin(), b->cls.end(), [&](const BatchClass& k) {
      return k.nx == c->p.nx && k.ny == c->p.ny && k.full2x2 == c->full2x2;
    });
    if (it == b->cls.end()) {
      BatchClass k;
      k.nx = c->p.nx;
      k.ny = c->p.ny;
      k.full2x2 = c->full2x2;
      b->cls.push_back(k);
      it = b->cls.end() - 1;
    }
    it->members.push_back(i);
  }
  if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->enter, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->leave, hipEventDisableTiming) != hipSuccess ||
      hipStreamCreateWithFlags(&b->graph_stream, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    return fail(SGPE_EDEVICE);
  }
  for (auto& k : b->cls) {
    const size_t n = k.members.size();
    if (hipStreamCreateWithFlags(&k.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&k.done, hipEventDisableTiming) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&k.row_tab), ROWTAB_N * n * sizeof(RowArgs)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&k.col_tab), COLTAB_N * n * sizeof(ColArgs)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(SGPE_EDEVICE);
    }
    const sgpe_status st = set_class_schedule(b, k, class_default(b->inst[k.members[0]], n));
    if (st != SGPE_OK) return fail(st);
  }
  *out = b;
  return SGPE_OK;
}

void sgpe_batch_destroy(sgpe_batch* b) {
  if (!b) return;
  (void)hipSetDevice(b->device);
  (void)hipStreamSynchronize(b->stream);
  drop_graphs(b);
  for (auto& k : b->cls) {
    if (k.stream) (void)hipStreamSynchronize(k.stream);
    if (k.row_tab) (void)hipFree(k.row_tab);
    if (k.col_tab) (void)hipFree(k.col_tab);
    if (k.e_tab) (void)hipFree(k.e_tab);
    if (k.done) (void)hipEventDestroy(k.done);
    if (k.stream) (void)hipStreamDestroy(k.stream);
  }
  if (b->graph_stream) {
    (void)hipStreamSynchronize(b->graph_stream);
    (void)hipStreamDestroy(b->graph_stream);
  }
  for (void* ptr : {static_cast<void*>(b->p_row_first), static_cast<void*>(b->p_row_imag),
                    static_cast<void*>(b->p_col[0]), static_cast<void*>(b->p_col[1]),
                    static_cast<void*>(b->p_row_items), static_cast<void*>(b->p_col_items),
                    static_cast<void*>(b->p_words), static_cast<void*>(b->p_cls_dev)})
    if (ptr) (void)hipFree(ptr);
  if (b->p_abort_host) (void)hipHostFree(b->p_abort_host);
  if (b->e_dev) (void)hipFree(b->e_dev);
  if (b->e_host) (void)hipHostFree(b->e_host);
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->enter) (void)hipEventDestroy(b->enter);
  if (b->leave) (void)hipEventDestroy(b->leave);
  for (sgpe_ctx* c : b->inst) sgpe_destroy(c);
  (void)hipGetLastError();
  delete b;
}

int32_t sgpe_batch_size(const sgpe_batch* b) { return b ? int32_t(b->inst.size()) : 0; }
int32_t sgpe_batch_class_count(const sgpe_batch* b) { return b ? int32_t(b->cls.size()) : 0; }

sgpe_status sgpe_batch_class_info(const sgpe_batch* b, int32_t k, int32_t* nx, int32_t* ny, int32_t* members) {
  if (!valid_class(b, k)) return SGPE_EINVAL;
  if (nx) *nx = b->cls[k].nx;
  if (ny) *ny = b->cls[k].ny;
  if (members) *members = int32_t(b->cls[k].members.size());
  return SGPE_OK;
}

sgpe_status sgpe_batch_instance_class(const sgpe_batch* b, int32_t index, int32_t* k) {
  if (!valid_index(b, index) || !k) return SGPE_EINVAL;
  for (size_t c = 0; c < b->cls.size(); ++c)
    for (int m : b->cls[c].members)
      if (m == index) {
        *k = int32_t(c);
        return SGPE_OK;
      }
  return SGPE_EINVAL;
}

sgpe_status sgpe_batch_set_psi(sgpe_batch* b, int32_t index, const double* psi) {
  if (!valid_index(b, index)) return SGPE_EINVAL;
  return sgpe_set_psi(b->inst[index], psi);
}

sgpe_status sgpe_batch_set_psi_device(sgpe_batch* b, int32_t index, const void* psi_dev) {
  if (!valid_index(b, index)) return SGPE_EINVAL;
  return sgpe_set_psi_device(b->inst[index], psi_dev);
}

sgpe_status sgpe_batch_get_psi(sgpe_batch* b, int32_t index, double* psi) {
  if (!valid_index(b, index)) return SGPE_EINVAL;
  return sgpe_get_psi(b->inst[index], psi);
}

sgpe_status sgpe_batch_step_real(sgpe_batch* b, int64_t n) { return b ? run(b, n, false) : SGPE_EINVAL; }
sgpe_status sgpe_batch_step_imag(sgpe_batch* b, int64_t n) { return b ? run(b, n, true) : SGPE_EINVAL; }

sgpe_status sgpe_batch_energy(sgpe_batch* b, int32_t index, double* e) {
  if (!valid_index(b, index)) return SGPE_EINVAL;
  return sgpe_energy(b->inst[index], e);
}

sgpe_status sgpe_batch_energies(sgpe_batch* b, double* e) {
  if (!b || !e) return SGPE_EINVAL;
  if (hipSetDevice(b->device) != hipSuccess) return hip_status(hipErrorInvalidDevice);
  for (sgpe_ctx* c : b->inst)
    if (!c->has_state) return SGPE_ESTATE;
  const size_t n = b->inst.size();
  if (!b->e_dev) {
    void* d = nullptr;
    void* h = nullptr;
    if (hipMalloc(&d, n * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      return SGPE_ENOMEM;
    }
    if (hipHostMalloc(&h, n * sizeof(double), hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipFree(d);
      return SGPE_ENOMEM;
    }
    b->e_dev = static_cast<double*>(d);
    b->e_host = static_cast<double*>(h);
  }
  for (auto& k : b->cls) {
    if (!k.e_tab) {   // the members' arguments: their states, tables and partial buffers are fixed
      std::vector<sgpe::EnergyArgs> tab;
      for (int m : k.members) {
        sgpe_ctx* c = b->inst[size_t(m)];
        sgpe::EnergyArgs a = energy_args(c, c->epart, c->epart + sgpe::kEnergyRowParts * c->p.ny);
        a.result = b->e_dev + m;
        tab.push_back(a);
      }
      void* d = nullptr;
      if (hipMalloc(&d, tab.size() * sizeof(sgpe::EnergyArgs)) != hipSuccess) {
        (void)hipGetLastError();
        return SGPE_ENOMEM;
      }
      if (hipMemcpy(d, tab.data(), tab.size() * sizeof(sgpe::EnergyArgs), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(d);
        return SGPE_EDEVICE;
      }
      k.e_tab = static_cast<sgpe::EnergyArgs*>(d);
    }
    const sgpe_ctx* c0 = b->inst[size_t(k.members[0])];
    const hipError_t err = sgpe::launch_energy_batch(k.e_tab, int(k.members.size()), k.nx, k.ny,
                                                     sgpe::energy_rows_per_block(k.nx, k.ny),
                                                     sgpe::energy_cols_per_block(k.nx, k.ny, c0->max_lds), b->stream);
    if (err != hipSuccess) return hip_status(err);
  }
  hipError_t err = hipMemcpyAsync(b->e_host, b->e_dev, n * sizeof(double), hipMemcpyDeviceToHost, b->stream);
  if (err == hipSuccess) err = hipStreamSynchronize(b->stream);
  if (err != hipSuccess) return hip_status(err);
  sgpe_status out = SGPE_OK;
  for (size_t i = 0; i < n; ++i) {
    e[i] = b->e_host[i];
    sgpe_ctx* c = b->inst[i];
    if (!std::isfinite(e[i])) c->latched = SGPE_ENONFINITE;
    if (latched_status(c) != SGPE_OK && out == SGPE_OK) out = c->latched;
  }
  return out;
}

sgpe_status sgpe_batch_norm(sgpe_batch* b, int32_t index, double* n) {
  if (!valid_index(b, index)) return SGPE_EINVAL;
  return sgpe_norm(b->inst[index], n);
}

sgpe_status sgpe_batch_synchronize(sgpe_batch* b) {
  if (!b) return SGPE_EINVAL;
  if (hipSetDevice(b->device) != hipSuccess) return hip_status(hipErrorInvalidDevice);
  const sgpe_status st = hip_status(hipStreamSynchronize(b->stream));
  if (st != SGPE_OK) return st;
  if (b->p_abort_host && __atomic_load_n(b->p_abort_host, __ATOMIC_ACQUIRE) != 0u) {
    // a grid-barrier wait of the persistent kernel gave up: the states are not valid
    __atomic_store_n(b->p_abort_host, 0u, __ATOMIC_RELEASE);
    return SGPE_EDEVICE;
  }
  // an instance whose imaginary-time norm went non-finite is reported (and stays latched in it)
  sgpe_status out = SGPE_OK;
  for (sgpe_ctx* c : b->inst)
    if (latched_status(c) != SGPE_OK && out == SGPE_OK) out = c->latched;
  return out;
}

// Persistent mode: validate the classes, give them the persistent kernel's work-item schedule,
// build the per-instance argument tables and the item lists.
static sgpe_status enable_persistent(sgpe_batch* b) {
  auto supported = [](int n) { return n == 128 || n == 256 || n == 512; };
  if (b->cls.size() > size_t(sgpe::kPersistClasses)) return SGPE_EINVAL;
  for (const auto& k : b->cls)
    if (k.nx != k.ny || !supported(k.nx) || k.full2x2) return SGPE_EINVAL;
  for (const sgpe_ctx* c : b->inst)
    if (c->split_order != SGPE_SPLIT_KRK || c->split_rs != SGPE_RSPLIT_FROZEN) return SGPE_EINVAL;
  if (hipStreamSynchronize(b->stream) != hipSuccess) return hip_status(hipErrorUnknown);
  int coop = 0;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, b->device) != hipSuccess || !coop)
    return hip_status(hipErrorNotSupported);
  // the per-class launches of the first and last step use the same 8-point, 1024-point-item schedule
  for (auto& k : b->cls) {
    sgpe_schedule s{};
    s.row_points = 8;
    s.col_points = 8;
    s.row_iters = 1;
    s.col_iters = 1;
    s.row_tile = 1024 / k.nx;
    s.col_tile = 1024 / k.ny;
    const sgpe_status st = set_class_schedule(b, k, s);
    if (st != SGPE_OK) return st;
  }
  const size_t n = b->inst.size();
  std::vector<RowArgs> first(n), imag(n);
  std::vector<ColArgs> col_r(n), col_i(n);
  for (size_t i = 0; i < n; ++i) {
    const sgpe_ctx* c = b->inst[i];
    RowArgs a = row_args(c);
    a.scale = float(1.0 / (double(c->p.nx) * double(c->p.ny)));
    first[i] = a;
    a.partials = c->partials;
    a.n_partials = col_groups(c);
    imag[i] = a;
    col_r[i] = col_args(c, false, false);
    col_i[i] = col_args(c, true, false);
  }
  auto up = [](auto** dst, const auto& v) {
    using T = std::remove_reference_t<decltype(v[0])>;
    if (!*dst && hipMalloc(reinterpret_cast<void**>(dst), v.size() * sizeof(T)) != hipSuccess) return false;
    return hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) == hipSuccess;
  };
  if (!up(&b->p_row_first, first) || !up(&b->p_row_imag, imag) || !up(&b->p_col[0], col_r) ||
      !up(&b->p_col[1], col_i)) {
    (void)hipGetLastError();
    return SGPE_ENOMEM;
  }
  if (!b->p_words) {
    if (hipMalloc(reinterpret_cast<void**>(&b->p_words), sgpe::kPersistWords * sizeof(unsigned)) != hipSuccess ||
        hipMemset(b->p_words, 0, sgpe::kPersistWords * sizeof(unsigned)) != hipSuccess) {
      (void)hipGetLastError();
      return SGPE_ENOMEM;
    }
    void* h = nullptr;
    void* d = nullptr;
    if (hipHostMalloc(&h, sizeof(unsigned), hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
      (void)hipGetLastError();
      return SGPE_ENOMEM;
    }
    b->p_abort_host = static_cast<unsigned*>(h);
    *b->p_abort_host = 0u;
    if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) {
      (void)hipGetLastError();
      return SGPE_EDEVICE;
    }
    b->p_abort_host_dev = static_cast<unsigned*>(d);
  }
  // workgroups: as many as stay co-resident (the smaller of the two instantiations' limits), in
  // kPersistGroups groups by index mod kPersistGroups
  const int n_cu = b->inst[0]->n_cu;
  int gmax = 0;
  for (int imagi = 0; imagi < 2; ++imagi) {
    int g = 0;
    hipError_t e = sgpe::persist_max_grid(imagi != 0, n_cu, &g);
    if (e != hipSuccess) return hip_status(e);
    gmax = imagi == 0 ? g : std::min(gmax, g);
  }
  constexpr int NG = sgpe::kPersistGroups;
  int members[NG];
  int usable = 0;
  for (int g = 0; g < NG; ++g) {
    members[g] = gmax > g ? (gmax - g + NG - 1) / NG : 0;
    usable += members[g] > 0;
  }
  if (usable == 0) return SGPE_EDEVICE;
  // every instance to one group: a class of a multiple of 8 members in eight equal runs of members
  // (the runs that batched launches place on one XCD each), otherwise each member to the group with
  // the fewest points so far
  std::vector<int> group_of(n, 0);
  double load[NG] = {};
  for (const auto& k : b->cls) {
    const int cnt = int(k.members.size());
    for (int j = 0; j < cnt; ++j) {
      int g = 0;
      if (cnt % NG == 0 && usable == NG) {
        g = j / (cnt / NG);
      } else {
        for (int h = 1; h < NG; ++h)
          if (members[h] > 0 && load[h] < load[g]) g = h;
      }
      group_of[size_t(k.members[j])] = g;
      load[g] += double(k.nx) * double(k.ny);
    }
  }
  // per group: the classes present, their items (row groups of 1024 / n rows and column tiles of
  // 1024 / n columns), and the group's workgroups split among them in proportion to their work
  sgpe::PersistClass pc[NG][sgpe::kPersistClasses] = {};
  std::vector<int4> ri, ci;
  for (int g = 0; g < NG; ++g) {
    int slot = 0;
    double weight[sgpe::kPersistClasses] = {};
    for (const auto& k : b->cls) {
      const int groups = k.nx * k.ny / 1024;
      sgpe::PersistClass c{};
      c.log2n = __builtin_ctz(k.nx);
      c.row_begin = int(ri.size());
      c.col_begin = int(ci.size());
      for (int m : k.members)
        if (group_of[size_t(m)] == g)
          for (int q = 0; q < groups; ++q) {
            ri.push_back(make_int4(m, q, 0, groups));
            ci.push_back(make_int4(m, q, 0, groups));
          }
      c.n_row = int(ri.size()) - c.row_begin;
      c.n_col = int(ci.size()) - c.col_begin;
      if (c.n_row == 0) continue;
      weight[slot] = double(c.n_row) * double(c.log2n);   // an item's cost grows with log2 n
      pc[g][slot++] = c;
    }
    if (slot == 0) continue;
    if (members[g] < slot) return SGPE_EDEVICE;
    double wsum = 0.0;
    for (int k = 0; k < slot; ++k) wsum += weight[k];
    int total = 0;
    for (int k = 0; k < slot; ++k) {
      int w = int(double(members[g]) * weight[k] / wsum);
      w = std::max(1, std::min(w, pc[g][k].n_row));
      pc[g][k].wg_count = w;
      total += w;
    }
    while (total > members[g]) {   // rounding: take back from the largest share
      int kmax = 0;
      for (int k = 1; k < slot; ++k)
        if (pc[g][k].wg_count > pc[g][kmax].wg_count) kmax = k;
      --pc[g][kmax].wg_count;
      --total;
    }
    for (;;) {                      // and hand out the rest where a workgroup has most items
      int kbest = -1;
      double best = 0.0;
      for (int k = 0; k < slot; ++k) {
        if (pc[g][k].wg_count >= pc[g][k].n_row) continue;
        const double per = weight[k] / pc[g][k].wg_count;
        if (kbest < 0 || per > best) kbest = k, best = per;
      }
      if (total >= members[g] || kbest < 0) break;
      ++pc[g][kbest].wg_count;
      ++total;
    }
    int begin = 0;
    for (int k = 0; k < slot; ++k) {
      pc[g][k].wg_begin = begin;
      begin += pc[g][k].wg_count;
    }
  }
  if (b->p_row_items) (void)hipFree(b->p_row_items);
  if (b->p_col_items) (void)hipFree(b->p_col_items);
  b->p_row_items = nullptr;
  b->p_col_items = nullptr;
  if (!up(&b->p_row_items, ri) || !up(&b->p_col_items, ci)) {
    (void)hipGetLastError();
    return SGPE_ENOMEM;
  }
  std::vector<sgpe::PersistClass> flat(&pc[0][0], &pc[0][0] + NG * sgpe::kPersistClasses);
  if (!up(&b->p_cls_dev, flat)) {
    (void)hipGetLastError();
    return SGPE_ENOMEM;
  }
  b->p_grid = gmax;
  // test hook: SGPE_PERSIST_SPIN_LIMIT lowers the bound of the barrier waits, so that a test can
  // make them give up (every workgroup still leaves the kernel normally)
  b->p_spin_limit = sgpe::kPersistSpinLimit;
  if (const char* env = std::getenv("SGPE_PERSIST_SPIN_LIMIT")) b->p_spin_limit = unsigned(std::strtoul(env, nullptr, 10));
  drop_graphs(b);
  b->persistent = true;
  b->persist_graph_ok = true;
  return SGPE_OK;
}

sgpe_status sgpe_batch_use_persistent(sgpe_batch* b, int32_t on) {
  if (!b) return SGPE_EINVAL;
  if (hipSetDevice(b->device) != hipSuccess) return hip_status(hipErrorInvalidDevice);
  if (!on) {
    if (b->persistent) drop_graphs(b);
    b->persistent = false;
    return SGPE_OK;
  }
  return enable_persistent(b);
}

sgpe_status sgpe_batch_use_graph(sgpe_batch* b, int32_t on) {
  if (!b) return SGPE_EINVAL;
  b->use_graph = (on != 0);
  return SGPE_OK;
}

sgpe_status sgpe_batch_get_schedule(const sgpe_batch* b, int32_t k, sgpe_schedule* out) {
  if (!valid_class(b, k) || !out) return SGPE_EINVAL;
  *out = get_schedule(b->inst[b->cls[k].members[0]]);
  return SGPE_OK;
}

sgpe_status sgpe_batch_set_schedule(sgpe_batch* b, int32_t k, const sgpe_schedule* s) {
  if (b && b->persistent) return SGPE_ESTATE;   // the persistent kernel fixes the schedule
  if (!valid_class(b, k)) return SGPE_EINVAL;
  if (hipSetDevice(b->device) != hipSuccess) return hip_status(hipErrorInvalidDevice);
  if (hipStreamSynchronize(b->stream) != hipSuccess) return hip_status(hipErrorUnknown);
  BatchClass& c = b->cls[k];
  return set_class_schedule(b, c, s ? *s : class_default(b->inst[c.members[0]], c.members.size()));
}

sgpe_status sgpe_batch_autotune(sgpe_batch* b, int32_t steps, double* best_ms) {
  if (b && b->persistent) return SGPE_ESTATE;
  if (!b || steps < 1) return SGPE_EINVAL;
  for (const sgpe_ctx* c : b->inst)
    if (!c->has_state) return SGPE_ESTATE;
  if (hipSetDevice(b->device) != hipSuccess) return hip_status(hipErrorInvalidDevice);
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess) {
    if (t0) (void)hipEventDestroy(t0);
    return hip_status(hipErrorOutOfMemory);
  }
  sgpe_status st = SGPE_OK;
  for (size_t ci = 0; ci < b->cls.size() && st == SGPE_OK; ++ci) {
    BatchClass& k = b->cls[ci];
    const sgpe_ctx* c0 = b->inst[k.members[0]];
    const size_t bytes = size_t(c0->p.nx) * size_t(c0->p.ny) * sizeof(float4);
    // keep the members' states: tuning runs real steps on them
    std::vector<void*> saved(k.members.size(), nullptr);
    for (size_t j = 0; j < k.members.size() && st == SGPE_OK; ++j) {
      if (hipMalloc(&saved[j], bytes) != hipSuccess ||
          hipMemcpyAsync(saved[j], b->inst[k.members[j]]->psi, bytes, hipMemcpyDeviceToDevice, b->stream) != hipSuccess)
        st = hip_status(hipErrorOutOfMemory);
    }
    const sgpe_schedule start = get_schedule(c0);
    sgpe_schedule best = start;
    float best_t = -1.0f;
    const int pts[3] = {4, 8, 16};
    const int tiles[5] = {1, 2, 4, 8, 16};
    for (int rp : pts)
      for (int cp : pts)
        for (int ct : tiles) {
          if (st != SGPE_OK) break;
          sgpe_schedule s{};
          s.col_tile = ct;
          s.row_iters = 1;
          s.col_iters = 1;
          s.row_points = rp;
          s.col_points = cp;
          if (hipStreamSynchronize(b->stream) != hipSuccess) {
            st = hip_status(hipErrorUnknown);
            break;
          }
          if (set_class_schedule(b, k, s) != SGPE_OK) continue;  // not valid for this shape
          hipError_t e = enqueue_class(b, k, 2, false, b->stream);
          if (e == hipSuccess) e = hipEventRecord(t0, b->stream);
          if (e == hipSuccess) e = enqueue_class(b, k, steps, false, b->stream);
          if (e == hipSuccess) e = hipEventRecord(t1, b->stream);
          if (e == hipSuccess) e = hipEventSynchronize(t1);
          float ms = 0.0f;
          if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
          if (e != hipSuccess) {
            st = hip_status(e);
            break;
          }
          if (best_t < 0.0f || ms < best_t) {
            best_t = ms;
            best = s;
          }
        }
    if (st == SGPE_OK) st = set_class_schedule(b, k, best_t < 0.0f ? start : best);
    if (best_ms && best_t >= 0.0f) best_ms[ci] = double(best_t) / double(steps);
    for (size_t j = 0; j < k.members.size(); ++j) {
      if (saved[j]) {
        if (st == SGPE_OK &&
            hipMemcpyAsync(b->inst[k.members[j]]->psi, saved[j], bytes, hipMemcpyDeviceToDevice, b->stream) != hipSuccess)
          st = hip_status(hipErrorUnknown);
        if (hipStreamSynchronize(b->stream) != hipSuccess && st == SGPE_OK) st = hip_status(hipErrorUnknown);
        (void)hipFree(saved[j]);
      }
    }
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  drop_graphs(b);
  return st;
}

}  // extern "C"
