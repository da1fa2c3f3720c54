// Internal interface between the host library (api.cpp) and the HIP kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace sgpe {

// Precision of the step kernels: T = float (complex64 state) or double (complex128).  C is the
// complex type of one spinor component, Q that of a grid point (both components, the state's
// element type).
template <class T> struct Cplx;
template <> struct Cplx<float> { using C = float2; using Q = float4; };
template <> struct Cplx<double> { using C = double2; using Q = double4; };
template <class T> using cplx_t = typename Cplx<T>::C;
template <class T> using point_t = typename Cplx<T>::Q;

// Row (x) pass modes.
enum RowMode : int {
  ROW_FWD = 0,   // forward x-FFT only (enter the mixed (k_x, y) representation)
  ROW_INV = 1,   // inverse x-FFT and scale (leave it: real space)
  ROW_STEP = 2,  // inverse x-FFT, scale, real-space exponential R(h), forward x-FFT
  ROW_VAR = 3,   // the general row pass of the splitting variants, steered by RowArgs::var_*
  ROW_STEP_NLN = 4,  // ROW_STEP with R(h) = N(h/2) L(h) N(h/2) (the K-R-K schedule of that split)
};

// Stages of the general row pass (ROW_VAR), run in this order when their flag is set: inverse
// x-FFT and scale, or only the scale; var_r real-space sub-steps R(h) in turn (each in closed form
// with frozen densities, or as N(h/2) L(h) N(h/2) when var_nln); the norm partial; forward x-FFT.
enum RowVarFlags : int {
  VAR_INV = 1,        // inverse x-FFT, then the scale (`scale`, or from the partials)
  VAR_SCALE = 2,      // scale only, from the partials (the state is in real space on entry)
  VAR_NORM_OUT = 4,   // one fp64 partial of sum |psi|^2 per workgroup into partials_out
  VAR_FWD = 8,        // forward x-FFT
  VAR_MID_SCALE = 16, // the scale after the inverse x-FFT is `scale`; the scale from the partials
                      //   is applied after the first real-space sub-step instead
  VAR_NO_STORE = 32,  // the state is not written back (a pass that only produces partials)
};

// Column (y) pass norm accumulation.
enum ColNorm : int {
  NORM_NONE = 0,
  NORM_DOT = 1,  // Re <psik, U psik>: the norm after the first half of U (U hermitian, U = V^2)
  NORM_SQ = 2,   // |U psik|^2
};

template <class T>
struct RowArgsT {
  point_t<T>* psi;       // [ny][nx] state, in place
  int nx, ny;
  int rows_per_block;
  const point_t<T>* tw;  // roots exp(-2 pi i j / nx) as {cos, sin, eta, 0} (rounded to T, see fwd_pass)
  // scale applied after the inverse transform: either `scale`, or computed from partials
  T scale;
  const double* partials;  // NULL => use `scale`
  int n_partials;
  double norm0, parseval_w;  // norm = parseval_w * sum(partials)
  double inv_npts;           // 1/(nx*ny)
  // real-space exponential (all pre-multiplied by the sub-step h)
  T x0, dx, y0, dy;          // x_j = x0 + j dx, y_i = y0 + i dy
  T hvx, hvy;                // h * wx^2 / 2, h * wy^2 / 2
  T hdelta2;                 // h * delta / 2
  T hg_uu, hg_dd, hg_ud;
  const T* hbx;              // h * Omega_x(x_j) / 2, length nx (full 2x2 variant only)
  const T* hby;              // h * Omega_y(y_i) / 2, length ny (full 2x2 variant only);
                             //   the spatial coupling is Omega_x(x) + Omega_y(y)
  // general row pass (ROW_VAR) only:
  int var_flags;             // RowVarFlags
  int var_r;                 // real-space sub-steps R(h) applied in turn (0, 1 or 2)
  int var_nln;               // 1: each R(h) as N(h/2) L(h) N(h/2)
  T hfrac;                   // h / dt: scales the hbx / hby tables (built for h = dt)
  double* partials_out;      // VAR_NORM_OUT: one double per workgroup
  // Status word of the context (host-visible, fine-grained memory) or NULL: workgroup 0 of a
  // pass that rescales by a norm from `partials` stores 1 there when that scale is not finite and
  // positive (the norm was zero, infinite or NaN).  Read by the host at synchronising calls.
  unsigned int* nonfinite;
};
using RowArgs = RowArgsT<float>;

template <class T>
struct ColArgsT {
  point_t<T>* psi;
  int nx, ny;
  int cols;                  // columns per workgroup
  const point_t<T>* tw;      // roots exp(-2 pi i j / ny) as {cos, sin, eta, 0}
  const point_t<T>* kx_tab;  // per k_x: {d11, d12} {d21, d22} as complex (M'(k_x) - 1)
  const cplx_t<T>* ky_tab;   // per k_y: P(k_y) - 1
  double* partials;          // one double per workgroup (norm modes)
};
using ColArgs = ColArgsT<float>;

constexpr int kEnergyRowParts = 3;

struct EnergyArgs {
  const float4* psi;         // the complex64 state, or
  const double4* psi64;      //   the complex128 one (exactly one is set)
  int nx, ny;
  int rows;                  // rows per row-kernel workgroup (energy_rows_per_block)
  int cols;                  // columns per column-kernel workgroup (energy_cols_per_block)
  const double4* twx;        // the fp64 step-kernel roots of length nx ({cos, sin, 0, 0} of 2 pi j / nx)
  const double4* twy;        // the same for ny
  double xmin, dx, ymin, dy;
  double wx2h, wy2h;         // wx^2/2, wy^2/2
  double delta, g_uu, g_dd, g_ud;
  double k_l, omega;
  const double* om_x;        // spatial Raman coupling Omega_x(x_j) (length nx) and Omega_y(y_i)
  const double* om_y;        //   (length ny); both NULL without one
  double dkx, dky;
  double* row_partials;      // kEnergyRowParts per row block: {linear real-space energy and the
                             //   rows' k_x terms, interaction energy, norm}
  double* col_partials;      // 1 per column block: its columns' k_y terms
  double norm0;              // the norm the energy per particle refers to
  double* result;            // batched launches: where the finishing kernel writes this energy
};

// Launchers (return hipSuccess or the launch error).
// Pass geometry.  points: points per lane of the transforms (16; 8 or 4 for lengths up to
// kMaxNSmallP, where more lanes shorten each lane's instruction stream); groups: rows (row pass)
// or columns (column pass) per workgroup; iters: row groups / column tiles per workgroup, 1 or 2
// (the next one prefetched while this one runs; 8 or 16 points per lane, at most 256 threads).
constexpr int kMaxNSmallP = 1024;
inline bool schedule_supported(int n, int groups, int iters, int points) {
  if (points != 16 && !((points == 8 || points == 4) && n <= kMaxNSmallP)) return false;
  if (n < points || groups < 1 || (groups & (groups - 1)) != 0) return false;
  if (iters != 1 && iters != 2) return false;
  if (iters == 2 && points == 4) return false;
  const int threads = 2 * groups * (n / points);
  return threads <= (iters == 2 ? 256 : 512);
}

hipError_t launch_row(const RowArgs& a, int mode, bool imag, bool full2x2, int iters, int points, hipStream_t s);
hipError_t launch_col(const ColArgs& a, int norm_mode, int iters, int points, hipStream_t s);
// complex128: 16 or 8 points per lane (8 for lengths up to kMaxNSmallP), one row group / column
// tile per workgroup, the step modes only
hipError_t launch_row(const RowArgsT<double>& a, int mode, bool imag, bool full2x2, int points, hipStream_t s);
hipError_t launch_col(const ColArgsT<double>& a, int norm_mode, int points, hipStream_t s);
// Batches of instances of one grid shape: `shape` gives the geometry (every table entry must
// share nx, ny, rows_per_block / cols); instance i's arguments are tab[i] (device memory), and
// the launch holds (ny / rows or nx / cols) x count workgroups, and batch_item places all of an
// instance's workgroups on one XCD.  One row group / column tile per workgroup.
hipError_t launch_row_batch(const RowArgs& shape, const RowArgs* tab, int count, int mode, bool imag, bool full2x2,
                            int points, hipStream_t s);
hipError_t launch_col_batch(const ColArgs& shape, const ColArgs* tab, int count, int norm_mode, int points,
                            hipStream_t s);
hipError_t launch_energy(const EnergyArgs& a, hipStream_t s);
// The energy per particle from the partials launch_energy wrote (a's buffers), combined on the
// device in a fixed order and written to out (one double, device memory).
hipError_t launch_energy_finish(const EnergyArgs& a, double* out, hipStream_t s);
// The energies of `count` complex64 states of one grid shape, one launch per kernel: tab (device)
// holds each state's arguments (rows and cols as energy_rows/cols_per_block give them for that
// shape), and each energy is written to its tab[i].result.
hipError_t launch_energy_batch(const EnergyArgs* tab, int count, int nx, int ny, int rows, int cols, hipStream_t s);
hipError_t launch_norm(const float4* psi, long long npts, double* partials, int nblocks, hipStream_t s);
hipError_t launch_norm(const double4* psi, long long npts, double* partials, int nblocks, hipStream_t s);

// Observables and state updates (observables.hip).  Grid-stride reductions write one partial (or
// `kMomentParts` partials) per block, summed on the host in block order.
constexpr int kMomentParts = 3;
// psi += amp * xi, both components (xi in the state's layout).
hipError_t launch_add_noise(float4* psi, const float4* xi, float amp, long long npts, hipStream_t s);
hipError_t launch_add_noise(double4* psi, const double4* xi, double amp, long long npts, hipStream_t s);
// per block: sum n_u n_d, sum n_u^2, sum n_d^2
hipError_t launch_moments(const float4* psi, long long npts, double* partials, int nblocks, hipStream_t s);
hipError_t launch_moments(const double4* psi, long long npts, double* partials, int nblocks, hipStream_t s);
// per block: sum of n_u + n_d over the points with x^2 + y^2 <= r2
hipError_t launch_disk_population(const float4* psi, int nx, int ny, double x0, double dx, double y0, double dy,
                                  double r2, double* partials, int nblocks, hipStream_t s);
hipError_t launch_disk_population(const double4* psi, int nx, int ny, double x0, double dx, double y0, double dy,
                                  double r2, double* partials, int nblocks, hipStream_t s);
// Phase increments of both components along the closed lattice path of `m` samples of the circle
// of this radius about the origin; out[c] = (sum of increments) / (2 pi).  One workgroup.
hipError_t launch_winding(const float4* psi, int nx, int ny, double xmax, double ymax, double radius, int m,
                          double* out, hipStream_t s);
hipError_t launch_winding(const double4* psi, int nx, int ny, double xmax, double ymax, double radius, int m,
                          double* out, hipStream_t s);

// Persistent step kernel of a batch (persist.hip).  Square grids of n = 128, 256 or 512 points per
// axis, one class per n.  Work items are int4 {instance, group, -, groups of that instance in the
// pass}; a row item is 1024 / n rows, a column item 1024 / n columns, 8 points per lane, 256
// threads.  The workgroups form kPersistGroups groups by blockIdx.x mod kPersistGroups (one XCD
// each); every instance belongs to one group, whose workgroups alone step it and meet at the
// group's barriers.  Within a group the workgroups are split among the classes present in
// proportion to their work; a workgroup takes its class's items round-robin.
constexpr int kPersistClasses = 3;
constexpr int kPersistGroups = 8;
struct PersistClass {
  int log2n;                  // 0: unused slot (the group's classes come first)
  int wg_begin, wg_count;     // this class's workgroups, by index within the group
  int row_begin, n_row;       // its row items in row_items
  int col_begin, n_col;       // its column items in col_items
};
struct PersistArgs {
  const RowArgs* row_first;   // per instance: the row pass of a call's first step (fixed scale)
  const RowArgs* row_step;    // per instance: later steps (imaginary time: scale from the partials)
  const ColArgs* col;         // per instance: K(dt), norm partials in imaginary time
  const int4* row_items;
  const int4* col_items;
  const PersistClass* cls;    // [kPersistGroups][kPersistClasses], device memory
  int steps;                  // steady-state steps in this launch
  int first_is_first;         // 1: the launch's first step is the call's first (row_first)
  unsigned* barrier;          // device words of the group barriers, kPersistWords (zeroed per launch)
  unsigned* abort_host;       // host-visible: a barrier wait gave up
  unsigned spin_limit;        // polls before a barrier wait gives up
};
constexpr unsigned kPersistSpinLimit = 4u << 20;   // ~4M polls of ~0.5 us or more: seconds, not a hang
// barrier words, each on its own 256-byte line: one counter per group, then the abort word
constexpr int kPersistWordStride = 64;
constexpr int kPersistAbortWord = kPersistWordStride * kPersistGroups;
constexpr int kPersistWords = kPersistWordStride * (kPersistGroups + 1);
size_t persist_lds_bytes();
// Largest co-resident grid of the persistent kernel on a device with n_cu compute units.
hipError_t persist_max_grid(bool imag, int n_cu, int* grid);
// Zero the barrier words, then launch cooperatively (all workgroups resident) on stream s.
hipError_t launch_persist(const PersistArgs& a, bool imag, int grid, hipStream_t s);

// Measurement probes (probes.hip): the data movement of the row and column partitions with no
// arithmetic, on a layout with `layout_rows` interleaved rows (1 = the state's layout).
hipError_t launch_probe_rows(const float4* src, float4* dst, int nx, int ny, int layout_rows, int row_tile,
                             bool write_through, hipStream_t s);
hipError_t launch_probe_cols(const float4* src, float4* dst, int nx, int ny, int layout_rows, int col_tile,
                             bool write_through, hipStream_t s);
// the same with a wave owning a whole row (column), both components per lane; `waves` lines per
// workgroup; lengths 512, 1024, 2048
// One record per workgroup of a gx x gy grid of `threads`: the XCD that ran it.
hipError_t launch_probe_xcc(unsigned* out, int gx, int gy, int threads, hipStream_t s);
hipError_t launch_probe_rows_wl(const float4* src, float4* dst, int nx, int ny, int layout_rows, int waves,
                                bool write_through, hipStream_t s);
hipError_t launch_probe_cols_wl(const float4* src, float4* dst, int nx, int ny, int layout_rows, int waves,
                                bool write_through, hipStream_t s);

// Workgroup geometry helpers (shared with the host so that partial counts match).
// max_lds: the device's LDS bytes per workgroup (minus the kernels' static LDS).
int row_rows_per_block(int nx, int ny, int points, size_t max_lds);
int col_default_cols(int nx, int ny, int points, size_t max_lds);
bool col_cols_supported(int nx, int ny, int cols, int iters, int points, size_t max_lds);
bool energy_fits(int nx, int ny, size_t max_lds);
int energy_rows_per_block(int nx, int ny);
int energy_cols_per_block(int nx, int ny, size_t max_lds);
size_t energy_lds_bytes(int n, int lines);
size_t row_lds_bytes(int nx, int rows);
size_t col_lds_bytes(int ny, int cols);
size_t col_lds_bytes_c128(int ny, int cols, int points);
int norm_blocks();

}  // namespace sgpe
