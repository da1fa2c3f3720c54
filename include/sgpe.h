/*
 * sgpe.h -- C ABI of the MI355X (gfx950) split-step solver for the two-component quasi-2D
 * Gross-Pitaevskii equation.
 *
 * Method (Smith, Cooke & LeBlanc, "GPU-accelerated solutions of the nonlinear Schroedinger
 * equation for simulating 2D spinor BECs"):
 *   - model: Sec. 3.1, Eq. (GPEcomponent) with the Hamiltonian pieces of Eqs. (H1)-(H4);
 *   - grids and propagators: Sec. 3.2, Eq. (TEOp);
 *   - time-splitting spectral (TSSP) step with Strang splitting, real and imaginary time, and
 *     renormalisation to the atom number after each imaginary-time step: Sec. 3.2.
 * Dimensionless harmonic-oscillator units (Sec. 6): hbar = m = omega_perp = 1.
 *
 * Conventions that the paper leaves open and this library fixes:
 *   - i d/dt psi = H psi; real-time propagators exp(-i H dt), imaginary-time exp(-H dtau);
 *   - H_K(k) = |k|^2/2 * 1 + k_L k_x sigma_z + (Omega/2) sigma_x  (k-space 2x2, uniform Omega);
 *   - H_R(r) = V(r) 1 + (delta/2) sigma_z + diag(g_uu n_u + g_ud n_d, g_dd n_d + g_ud n_u)
 *              + (Omega(x, y)/2) sigma_x,  V = (wx^2 x^2 + wy^2 y^2)/2, with the spatial coupling
 *              Omega(x, y) = omega_r0 tanh(x/omega_rw), or Omega_x(x) + Omega_y(y) as given to
 *              sgpe_set_raman_profile;
 *   - one step = K(dt/2) R(dt) K(dt/2); R exponentiates H_R with the densities of its input;
 *   - imaginary time rescales the total (both components) to norm0 after every step;
 *   - grid x_j = -xmax + j*dx, dx = 2*xmax/nx (periodic, endpoint excluded), k_x in FFT order
 *     with the Nyquist bin at -pi/dx; the same along y;
 *   - energy per particle: the Gross-Pitaevskii functional with 1/2 on the interaction terms, of
 *     the state rescaled to norm0 (quadratic terms over the norm N, interaction terms over
 *     N^2 / norm0), so that the norm of a complex64 state does not enter at first order.
 *
 * Threading: a context is not thread-safe; distinct contexts are independent.
 * Errors: every call returns a status; nothing aborts and no C++ exception crosses the ABI.
 * Validation errors are returned before any device work.  A non-finite norm found during
 * imaginary-time stepping (the renormalisation of Sec. 3.2 divides by it) is latched in the
 * context: the pass that would rescale by a norm that is zero, infinite or NaN sets a status word
 * in pinned host memory, and the next synchronising call (sgpe_synchronize, sgpe_get_psi,
 * sgpe_norm, sgpe_energy, the observables) returns SGPE_ENONFINITE.  Non-finite values found in
 * the state by get_psi, norm or energy latch the same way.  sgpe_set_psi clears the latch.
 *
 * Field names: sgpe_params names the spin-momentum coefficient k_l (k_L of Eq. H1) and the uniform
 * Raman coupling omega (Omega of Eq. H4), after the paper's symbols.
 */
#ifndef SGPE_H
#define SGPE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SGPE_OK = 0,
  SGPE_EINVAL = 1,      /* invalid argument or parameter (reported before any device work) */
  SGPE_ENOMEM = 2,      /* device or pinned host allocation failed, or the grid exceeds the
                           supported size */
  SGPE_EDEVICE = 3,     /* no usable gfx950 device, or a HIP runtime error */
  SGPE_ENONFINITE = 4,  /* NaN/Inf in an input state, or a non-finite norm during stepping */
  SGPE_ESTATE = 5       /* call not valid in the current state (e.g. stepping before set_psi) */
} sgpe_status;

/* Problem parameters.  Plain data; the same fields as the Python dataclass workloads.Params. */
typedef struct {
  int32_t nx, ny;         /* grid points, powers of two in [16, 4096]                  (Sec. 3.2) */
  double xmax, ymax;      /* box [-xmax, xmax) x [-ymax, ymax), both > 0               (Sec. 3.2) */
  double g_uu, g_dd, g_ud;/* mean-field couplings g_{up up}, g_{dn dn}, g_{up dn}       (Eq. H3)  */
  double k_l;             /* spin-momentum coefficient: + k_l k_x sigma_z in H_K        (Eq. H1)  */
  double omega;           /* spatially uniform Raman coupling, (omega/2) sigma_x in H_K (Eq. H4)  */
  double delta;           /* uniform detuning, (delta/2) sigma_z in H_R                 (Eq. H2)  */
  double wx, wy;          /* trap V = (wx^2 x^2 + wy^2 y^2)/2, both >= 0               (Eq. H2)  */
  double omega_r0;        /* spatial Raman coupling Omega(x) = omega_r0 tanh(x/omega_rw) in H_R;  */
  double omega_rw;        /*   omega_r0 = 0 disables it; omega_rw > 0 when enabled     (Eq. H4)  */
  double dt;              /* time step (> 0), used for real and imaginary steps        (Eq. TEOp) */
  double norm0;           /* imaginary-time target norm dx dy sum |psi|^2 (> 0)        (Sec. 3.2) */
} sgpe_params;

typedef struct sgpe_ctx sgpe_ctx;

/* Check a parameter set on the host (no device calls).  SGPE_OK or SGPE_EINVAL. */
sgpe_status sgpe_validate_params(const sgpe_params* p);

/* Number of visible HIP devices, or a negative value if the runtime reports none/an error.
 * Host-side query; never fails with an exception. */
int32_t sgpe_device_count(void);

/* Create a solver context on the current HIP device for the two-component model of Sec. 3.1
 * (Eq. GPEcomponent, Hamiltonian Eqs. H1-H4) on the periodic grid of Sec. 3.2 (x_j = -xmax + j dx,
 * k-space spacing pi / xmax).  Builds the operator and root tables of Eq. (TEOp) for dt and dt/2.
 *   hip_stream: a hipStream_t to enqueue all work on, or NULL for the null stream.  Borrowed.
 *   psi_dev:    NULL to let the context allocate the state (16*nx*ny bytes), or a device pointer
 *               of at least 16*nx*ny bytes, 16-byte aligned, which the context borrows and which
 *               must outlive it.  The device layout is [ny][nx] of {re_up, im_up, re_dn, im_dn}
 *               (float32).
 * On success *out receives the context; on failure *out is set to NULL.  The state is
 * undefined until sgpe_set_psi; stepping before that returns SGPE_ESTATE.
 * Errors: SGPE_EINVAL (bad params or NULL out), SGPE_EDEVICE (no device / not gfx950 /
 * runtime error), SGPE_ENOMEM. */
sgpe_status sgpe_create(const sgpe_params* p, void* hip_stream, void* psi_dev, sgpe_ctx** out);

/* Precision of a context's state and step arithmetic. */
typedef enum {
  SGPE_C64 = 0,   /* complex64 state, fp32 step kernels (the default) */
  SGPE_C128 = 1   /* complex128 state, fp64 step kernels: the same kernels instantiated in double */
} sgpe_precision;

/* sgpe_create with a precision.  SGPE_C128: the state is [ny][nx] of {re_up, im_up, re_dn, im_dn}
 * as fp64 (32*nx*ny bytes; a borrowed psi_dev must hold that many, 16-byte aligned), set_psi and
 * get_psi copy without rounding, and the step kernels, tables and the imaginary-time norm run in
 * fp64 (Sec. 4 uses complex128 throughout).  Its schedules have no prefetch (row_iters = col_iters
 * = 1), 16 or 8 points per lane (8 for lengths up to 1024), and at most 256 threads per workgroup
 * unless one line alone needs 512; sgpe_set_schedule accepts those (SGPE_EINVAL otherwise),
 * sgpe_set_col_tile returns SGPE_EINVAL, sgpe_set_splitting accepts only the default, sgpe_profile_steps / sgpe_profile_kernels return SGPE_ESTATE.  Batches are
 * complex64 only.  Errors: as sgpe_create, and SGPE_EINVAL for an unknown precision. */
sgpe_status sgpe_create_ex(const sgpe_params* p, int32_t precision, void* hip_stream, void* psi_dev,
                           sgpe_ctx** out);

/* Release the context and everything it allocated (not a borrowed state).  NULL is a no-op. */
void sgpe_destroy(sgpe_ctx* ctx);

/* Set the pseudospinor order parameter (Psi_up, Psi_down) of Sec. 3.1 on the grid points of
 * Sec. 3.2 -- the initial state of a real- or imaginary-time propagation.  psi_host is complex128,
 * shape (2, ny, nx), C order, re/im interleaved (component 0 = up); the caller keeps ownership.
 * It is rounded once to complex64 (copied as is for SGPE_C128).  Synchronous.  Clears a latched
 * status.  Errors: SGPE_EINVAL (NULL), SGPE_ENONFINITE (NaN/Inf in the input; the state is
 * unchanged). */
sgpe_status sgpe_set_psi(sgpe_ctx* ctx, const double* psi_host);

/* sgpe_set_psi from device memory: the order parameter (Psi_up, Psi_down) of Sec. 3.1 on the grid
 * of Sec. 3.2, already in the context's own device layout -- [ny][nx] of {re_up, im_up, re_dn,
 * im_dn}, float32 for SGPE_C64 and float64 for SGPE_C128 (16 * nx * ny or 32 * nx * ny bytes),
 * 16-byte aligned, on the context's device, and either the context's own state buffer or disjoint
 * from it.  The caller keeps ownership and must have finished writing it (its producer ordered
 * before this call).  The values are checked on the device first
 * (one pass counting non-finite values), then copied into the state as they are; nothing is rounded
 * or rescaled.  Synchronises.  Clears a latched status.  Errors: SGPE_EINVAL (NULL or misaligned),
 * SGPE_ENONFINITE (a NaN/Inf; the state is unchanged), SGPE_EDEVICE. */
sgpe_status sgpe_set_psi_device(sgpe_ctx* ctx, const void* psi_dev);

/* Copy the order parameter (Sec. 3.1) out in the layout of sgpe_set_psi, into the caller's
 * array of 4 * nx * ny doubles.  Synchronises the stream.  Errors: SGPE_EINVAL (NULL), SGPE_ESTATE
 * (no state), SGPE_ENONFINITE (a non-finite value in the state, or a latched status; the values
 * are still copied). */
sgpe_status sgpe_get_psi(sgpe_ctx* ctx, double* psi_host);

/* Advance n >= 0 real-time steps (Sec. 3.2).  Asynchronous on the context's stream.  The
 * fused schedule is K(dt/2) [R(dt) K(dt)]^(n-1) R(dt) K(dt/2); its result equals n separate
 * K(dt/2) R(dt) K(dt/2) steps up to rounding.  Consecutive calls continue one schedule: on a
 * context with the K-R-K splitting (either real-space form) on a complex64 state, or the default
 * splitting on a complex128 one, and a state it allocated itself, a call leaves its
 * last K(dt/2) and inverse x-transform pending, and the next step call of the same kind merges them
 * with its own first K(dt/2), so calls of n1 and n2 steps give bit for bit what one call of
 * n1 + n2 steps gives.  Every other call on the context (get_psi, energy, norm, the observables,
 * synchronize, a step of the other kind, a schedule or splitting change, ...) completes the
 * pending half-step first, so no caller sees the difference.  A context on a caller's state buffer
 * (psi_dev at create) completes every call, so the buffer always holds the documented layout.
 * Errors: SGPE_EINVAL (n < 0), SGPE_ESTATE. */
sgpe_status sgpe_step_real(sgpe_ctx* ctx, int64_t n);

/* Advance n >= 0 imaginary-time steps, rescaling the total norm to norm0 after each one
 * (Sec. 3.2).  Asynchronous.  Errors as sgpe_step_real. */
sgpe_status sgpe_step_imag(sgpe_ctx* ctx, int64_t n);

/* Energy per particle of the current state rescaled to norm0 (Gross-Pitaevskii functional, Eqs.
 * (H1)-(H4) with 1/2 on the interaction terms; quadratic terms over the norm N, interaction terms
 * over N^2 / norm0).  Accumulated in fp64.  Synchronises.  The partial sums come back through a
 * pinned host buffer owned by the context, allocated on the first reduction (energy, norm or an
 * observable) and grown on demand; SGPE_ENOMEM if that allocation fails. */
sgpe_status sgpe_energy(sgpe_ctx* ctx, double* e_per_particle);

/* Norm dx dy sum |psi|^2 of the current state (both components), accumulated in fp64: the atom
 * number that imaginary time restores after every step (Sec. 3.2).  Synchronises.  Partials as
 * sgpe_energy.  Errors: SGPE_EINVAL (NULL), SGPE_ESTATE (no state), SGPE_ENONFINITE. */
sgpe_status sgpe_norm(sgpe_ctx* ctx, double* norm);

/* Wait for all work enqueued by the context; reports a latched error (SGPE_ENONFINITE after an
 * imaginary-time step met a norm that is zero, infinite or NaN, so that the renormalisation of
 * Sec. 3.2 could not be applied). */
sgpe_status sgpe_synchronize(sgpe_ctx* ctx);

/* Stopping rules and result of sgpe_relax_imag (below). */
typedef enum { SGPE_RELAX_TARGET = 0, SGPE_RELAX_DELTA = 1 } sgpe_relax_rule;

typedef struct sgpe_relax_result {
  int64_t steps;        /* steps at the last check read: the one that met the rule, else the last */
  int64_t steps_taken;  /* steps applied to the state when the call returns */
  int64_t checks;       /* checks read, check 0 included */
  double energy;        /* energy per particle at the last check read */
  double energy_prev;   /* at the check before it (NaN for check 0) */
  int32_t met;          /* 1 if the rule was met */
  int32_t reserved;     /* 0 */
} sgpe_relax_result;

/* Ground state by imaginary-time propagation (Sec. 3.2: imaginary time approaches the ground state
 * asymptotically, the norm restored after every step; Sec. 6 finds its ground states this way),
 * run until an energy rule is met.  The paper fixes no stopping rule; these are the library's:
 *   SGPE_RELAX_TARGET: stop at the first check with |E - target| <= tol |target|;
 *   SGPE_RELAX_DELTA:  stop at the first check with |E_k - E_(k-1)| < tol |E_k| (target unused).
 * Check 0 is the energy of the state as it is; check k > 0 follows min(k check_every, max_steps)
 * steps of the context's scheme (as sgpe_step_imag), so max_steps caps the steps.  Each check's
 * energy is that of sgpe_energy (same kernels, the partials combined on the device: equal up to
 * the order of the final fp64 sums).  The host reads check k while up to two further chunks of
 * check_every steps are already queued, so the device never waits for the host between chunks; when
 * check k meets the rule those chunks still run, and the state the call leaves has
 * out->steps_taken >= out->steps steps (at most 2 check_every more).  energies (host, may be NULL
 * with energies_cap = 0) receives the energy of check k at index k for k < energies_cap.
 * Synchronises before returning.  The ring of checks in flight (4 device doubles, their pinned host
 * copies and 4 events) is allocated on the first call and kept by the context.
 * Errors: SGPE_EINVAL (NULL out, check_every < 1, max_steps < 0, either above 2^61, tol negative
 * or not finite, an unknown rule, a non-finite target with SGPE_RELAX_TARGET, energies NULL with
 * energies_cap > 0, energies_cap < 0), SGPE_ESTATE (no state), SGPE_ENOMEM, SGPE_EDEVICE, SGPE_ENONFINITE (a check's
 * energy, or an imaginary-time norm, not finite: the call stops there and out holds that check). */
sgpe_status sgpe_relax_imag(sgpe_ctx* ctx, int64_t check_every, int64_t max_steps, int32_t rule, double target,
                            double tol, double* energies, int64_t energies_cap, sgpe_relax_result* out);

/* Measurement helper: run n real-time (imag = 0) or imaginary-time (imag = 1) steady-state
 * steps with a HIP event pair around every kernel launch, and return the mean duration in
 * milliseconds of the row pass (x transforms + real-space exponential) and of the column pass
 * (y transforms + k-space propagator).  The state advances exactly as with sgpe_step_*(n).
 * Synchronises.  Either output pointer may be NULL. */
sgpe_status sgpe_profile_steps(sgpe_ctx* ctx, int32_t imag, int64_t n,
                               double* row_ms, double* col_ms);

/* Measurement helper: mean duration in milliseconds of one steady-state row-pass launch and
 * one column-pass launch (real time: imag = 0; imaginary time: imag = 1), each from n launches
 * issued back to back between one HIP event pair -- the per-kernel figure a kernel-trace
 * profiler reports.  The launches work on a copy of the state in the mixed representation; the
 * state is restored afterwards, so a caller sees no change.  Allocates the state-sized scratch
 * buffer on first use.  Synchronises.  Either output pointer may be NULL. */
sgpe_status sgpe_profile_kernels(sgpe_ctx* ctx, int32_t imag, int64_t n,
                                 double* row_ms, double* col_ms);

/* Splitting variants (Sec. 3.2).  order: SGPE_SPLIT_KRK, one step = K(dt/2) R(dt) K(dt/2) (the
 * default), or SGPE_SPLIT_RKR, one step = R(dt/2) K(dt) R(dt/2).  real_space: SGPE_RSPLIT_FROZEN,
 * R(h) = one closed-form 2x2 exponential of H_R with the densities of its input (the default), or
 * SGPE_RSPLIT_NLN, R(h) = N(h/2) L(h) N(h/2) with N the mean-field phase (Eq. H3) with the densities
 * of its input and L the exponential of the linear real-space terms (Eqs. H2, H4).  The frozen
 * form is the exact real-space sub-flow when there is no spatial Raman coupling, or when
 * g_uu = g_dd = g_ud (the mean field is then a multiple of the total density, which the coupling
 * conserves); otherwise it is first order in the mean-field coupling, and N L N keeps the step
 * second order.  Imaginary time normalises after
 * every step in every variant.  Cost per step: two sweeps, except R-K-R in imaginary time (three:
 * the norm is needed between the two R halves of consecutive steps).  On a complex64 state K-R-K
 * with N L N runs the default's fused schedule with N L N in its row pass, so consecutive step calls
 * continue it as they do the default's; R-K-R runs a general row pass and completes every call.
 * sgpe_profile_steps and sgpe_profile_kernels measure the default only and return SGPE_ESTATE
 * under a variant.  Takes effect for the next step call.
 * Errors: SGPE_EINVAL (NULL context, unknown value). */
typedef enum { SGPE_SPLIT_KRK = 0, SGPE_SPLIT_RKR = 1 } sgpe_split_order;
typedef enum { SGPE_RSPLIT_FROZEN = 0, SGPE_RSPLIT_NLN = 1 } sgpe_real_space_split;
sgpe_status sgpe_set_splitting(sgpe_ctx* ctx, int32_t order, int32_t real_space);

/* Spatially varying Raman coupling Omega(x, y) = Omega_x(x) + Omega_y(y) of the real-space
 * Hamiltonian ((Omega/2) sigma_x in H_R, Eq. (H4) with a position-dependent Omega; Sec. 6 uses a
 * profile along y, Eq. (Omega)).  omega_x: host array of nx values Omega_x(x_j); omega_y: host
 * array of ny values Omega_y(y_i); either may be NULL for a zero profile; both NULL switches the
 * spatial coupling off.  The arrays are copied (the caller keeps ownership) and replace the
 * profile that omega_r0/omega_rw gave at creation.  Waits for the stream's queued work first.
 * Errors: SGPE_EINVAL (non-finite value), SGPE_EDEVICE, SGPE_ENOMEM. */
sgpe_status sgpe_set_raman_profile(sgpe_ctx* ctx, const double* omega_x, const double* omega_y);

/* Annealing update (Sec. 6): psi <- psi + amplitude * xi at every point and both components.
 * xi: host array in the layout of sgpe_set_psi (complex128, shape (2, ny, nx)), rounded once to
 * complex64; the caller draws it (e.g. complex Gaussian noise) and keeps ownership.  No
 * renormalisation (the next imaginary-time step does it).  Allocates the state-sized scratch
 * buffer on first use.  Synchronises.
 * Errors: SGPE_EINVAL (NULL, non-finite amplitude), SGPE_ENONFINITE (NaN/Inf in xi; the state is
 * unchanged), SGPE_ESTATE (no state). */
sgpe_status sgpe_add_noise(sgpe_ctx* ctx, const double* xi_host, double amplitude);

/* System-averaged phase-separation parameter of the current state (Sec. 6, Eq. (s)):
 * s = 1 - sum n_u n_d / sqrt(sum n_u^2 * sum n_d^2), sums over all grid points, n = |psi|^2,
 * accumulated in fp64.  0 for proportional densities, 1 for disjoint ones.  Synchronises.
 * Errors: SGPE_EINVAL (NULL), SGPE_ESTATE (no state, or a component that is zero everywhere). */
sgpe_status sgpe_phase_separation(sgpe_ctx* ctx, double* s);

/* Radius of the smallest disc about the origin (x = y = 0) that holds at least `fraction` of the
 * total population sum (n_u + n_d): the smallest grid-point radius r_k with
 * sum_{x^2 + y^2 <= r_k^2} (n_u + n_d) >= fraction * total, found by bisection to within
 * 1e-12 relative (about 60 fp64 reductions on the device).  Sec. 6 uses fraction = 0.99 for the
 * contour of the circulation.  Synchronises.
 * Errors: SGPE_EINVAL (NULL, fraction outside (0, 1]), SGPE_ESTATE (no state or zero population). */
sgpe_status sgpe_population_radius(sgpe_ctx* ctx, double fraction, double* radius);

/* Circulation of each component along the circle of `radius` about the origin, counter-clockwise
 * (Sec. 6, Eq. (Lz)): the closed lattice path through p_k, k = 0..m-1, the grid point nearest to
 * (radius cos t_k, radius sin t_k), t_k = 2 pi k / m, m = max(256, ceil(4 pi radius / min(dx, dy)))
 * (so that consecutive points are equal or neighbours); raw[c] = (1 / 2 pi) sum_k
 * arg(psi_c(p_{k+1}) conj(psi_c(p_k))) with p_m = p_0, each increment in (-pi, pi], in fp64; n[c] =
 * raw[c] rounded to the nearest integer, the winding number (L_z per particle in units of hbar).
 * n: int32[2] (up, down); raw: double[2] or NULL.  Synchronises.
 * Errors: SGPE_EINVAL (NULL n, radius not in (0, min(xmax, ymax))), SGPE_ESTATE (no state). */
sgpe_status sgpe_winding(sgpe_ctx* ctx, double radius, int32_t* n, double* raw);

/* Measurement helper: the memory floor of a step's data movement (no arithmetic).  The row pass
 * and the column pass of a step (the two sweeps of the fused schedule of Sec. 3.2's split step)
 * partition the grid among workgroups by rows, then by columns.  This probe copies an nx x ny grid
 * of 16-byte points between two buffers of its own, alternating the two partitions: each point
 * stays at its address, and what alternates is which workgroup (and so which XCD) reads and writes
 * it.
 *   layout_rows L (1, 2, 4, 8): point (x, y) at index ((y / L) nx + x) L + y % L (L = 1: the
 *                 state's [ny][nx] layout; larger L makes L rows of a column contiguous);
 *   flags:        SGPE_PROBE_WRITE_THROUGH: device-scope stores, as the single-instance step kernels
 *                 use; SGPE_PROBE_WAVE_LOCAL: a wave owns a whole row (column) with both components
 *                 per lane, as transforms that run inside one wave would (lengths 512..2048);
 *   row_tile, col_tile: rows per row-partition workgroup and columns per column-partition workgroup
 *                 -- without WAVE_LOCAL each lane moves the 16 eight-byte values a lane of the step
 *                 kernels owns (2 row_tile nx / 16 and 2 col_tile ny / 16 threads, at most 1024);
 *                 with it, 1..8 waves (lines) per workgroup.
 * One untimed round, then reps rounds with a HIP event after every launch (row_ms / col_ms: mean
 * per launch of each partition, back to back with no host wait), then reps rounds between one event
 * pair (pair_ms: mean per round, a row and a column launch).  Any output may be NULL.  Allocates
 * and frees its buffers on the current device, synchronises.  Errors: SGPE_EINVAL (sizes not powers
 * of two, out of range, unknown flags), SGPE_ENOMEM, SGPE_EDEVICE. */
enum { SGPE_PROBE_WRITE_THROUGH = 1, SGPE_PROBE_WAVE_LOCAL = 2 };
sgpe_status sgpe_probe_exchange(int32_t nx, int32_t ny, int32_t layout_rows, int32_t row_tile, int32_t col_tile,
                                int32_t flags, int32_t reps, double* row_ms, double* col_ms, double* pair_ms);

/* Measurement helper: where workgroups run.  Launches a gx x gy grid of `threads`-thread
 * workgroups on the current device; thread 0 of workgroup (x, y) writes the index of the XCD that
 * ran it (hardware register XCC_ID) to xcd[y gx + x] (host memory, gx gy entries).  The batched
 * and persistent launches (Sec. 3.2's steps of many instances) place work by the dispatcher's order,
 * workgroup L of a launch on XCD (s + L) mod 8 with s where its rotation stood; this probe shows
 * that order on the device at hand.  Synchronises.
 * Errors: SGPE_EINVAL (NULL xcd, gx < 1, gy not in 1..65535, threads not in 1..1024, more than
 * 2^24 workgroups), SGPE_ENOMEM, SGPE_EDEVICE. */
sgpe_status sgpe_probe_placement(int32_t gx, int32_t gy, int32_t threads, uint32_t* xcd);

/* sgpe_energy for callers that cannot allocate (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the same energy per particle, written as one double to
 * e_dev (device memory, caller-owned), asynchronously on the context's stream.  The call allocates
 * nothing and never synchronises: the energy kernels' partial sums live in a static device array of
 * 128 KiB (three per row block and one per column block, up to 4096 of each: every grid the library
 * accepts), which every GPU the library runs on holds until the process ends.  Every call on a device
 * shares that array; calls that overlap on one device (several streams or threads) race on it and
 * must be ordered by the caller.  The result equals sgpe_energy's up to the order of the final fp64
 * sums.  Errors: SGPE_EINVAL (NULL e_dev), SGPE_ESTATE (no state), SGPE_ENOMEM (more rows or column
 * blocks than the array holds; no grid the library accepts has them), SGPE_EDEVICE. */
sgpe_status sgpe_energy_noalloc(sgpe_ctx* ctx, double* e_dev);

/* Static description of a status code.  Never NULL. */
const char* sgpe_strerror(sgpe_status s);

/* Tuning knob: columns per column-pass workgroup, the rest of the schedule kept (prefetching
 * is dropped if the new width does not allow it).  0 restores the whole default schedule.  An
 * unsupported value returns SGPE_EINVAL and changes nothing.  See sgpe_schedule. */
sgpe_status sgpe_set_col_tile(sgpe_ctx* ctx, int32_t columns);

/* Launch schedule of the two passes -- how the work is cut into lanes and workgroups.  Tiles and
 * prefetching do not change the arithmetic of any point: with the same points per lane, real-time
 * results are bit-identical under every valid schedule, and imaginary-time results differ only in
 * the grouping of the fp64 norm partials.  The points per lane set the transforms' radix
 * decomposition, so changing them changes results at the level of rounding.
 *   col_tile    columns per column-pass workgroup (power of two)
 *   row_iters   row groups per row-pass workgroup, 1 or 2: with 2, the next group's data is loaded
 *               while the current one is transformed (8 or 16 points per lane, <= 256 threads)
 *   col_iters   the same for column tiles
 *   row_points  points per lane of the x transforms: 16, or 8 / 4 when nx <= 1024
 *   col_points  the same for the y transforms and ny
 *   row_tile    rows per row-pass workgroup (power of two); 0 in sgpe_set_schedule: the default
 *               for row_points (256-thread workgroups)
 * A workgroup has 2 * lines * (n / points) threads, at most 512 (256 when prefetching), and its
 * LDS must fit the device. */
typedef struct {
  int32_t col_tile;
  int32_t row_iters;
  int32_t col_iters;
  int32_t row_points;
  int32_t col_points;
  int32_t row_tile;
} sgpe_schedule;

/* The schedule in use.  SGPE_EINVAL if either pointer is NULL. */
sgpe_status sgpe_get_schedule(sgpe_ctx* ctx, sgpe_schedule* out);

/* Set the schedule; NULL restores the default (chosen from the grid size and the device's
 * compute-unit count).  An unsupported schedule returns SGPE_EINVAL and changes nothing. */
sgpe_status sgpe_set_schedule(sgpe_ctx* ctx, const sgpe_schedule* schedule);

/* ------------------------------------------------------------------------------------------
 * Batched parameter sweeps: many independent instances, any mix of grid shapes, stepped
 * together.  Each instance is a full solver of its own (its parameters, state, norm); instances
 * of one grid shape and real-space operator form make a class, and each pass of a class is one
 * launch over all of its members, so classes of small grids fill the device.  Classes run
 * concurrently on internal streams forked from and joined to the batch stream.  With graphs on
 * (the default), the launches of a step_* call are captured once per (n, real/imag) into a HIP
 * graph and replayed on later calls with the same n.
 *
 * Results: every instance computes exactly what a single context (sgpe_create) with the same
 * parameters and schedule computes -- bit-identical.
 * ------------------------------------------------------------------------------------------ */
typedef struct sgpe_batch sgpe_batch;

/* count (1..65535) instances with params[i]; the same error cases as sgpe_create for each.
 * hip_stream as in sgpe_create.  Per-class schedules start at the single-instance defaults for
 * the class's total point count (row_iters = col_iters = 1: batched launches take one row group
 * / column tile per workgroup). */
sgpe_status sgpe_batch_create(const sgpe_params* params, int32_t count, void* hip_stream, sgpe_batch** out);
void sgpe_batch_destroy(sgpe_batch* batch);

int32_t sgpe_batch_size(const sgpe_batch* batch);          /* instances; 0 for NULL */
int32_t sgpe_batch_class_count(const sgpe_batch* batch);   /* classes; 0 for NULL */
/* grid shape and member count of class k; any output may be NULL */
sgpe_status sgpe_batch_class_info(const sgpe_batch* batch, int32_t k, int32_t* nx, int32_t* ny, int32_t* members);
/* the class of instance `index` */
sgpe_status sgpe_batch_instance_class(const sgpe_batch* batch, int32_t index, int32_t* k);

/* Per instance, as sgpe_set_psi / sgpe_set_psi_device / sgpe_get_psi / sgpe_energy / sgpe_norm
 * (index out of range: SGPE_EINVAL). */
sgpe_status sgpe_batch_set_psi(sgpe_batch* batch, int32_t index, const double* psi);
sgpe_status sgpe_batch_set_psi_device(sgpe_batch* batch, int32_t index, const void* psi_dev);
sgpe_status sgpe_batch_get_psi(sgpe_batch* batch, int32_t index, double* psi);
sgpe_status sgpe_batch_energy(sgpe_batch* batch, int32_t index, double* e_per_particle);
sgpe_status sgpe_batch_norm(sgpe_batch* batch, int32_t index, double* norm);

/* The energy per particle (as sgpe_energy: the Gross-Pitaevskii functional of Eqs. (H1)-(H4) of
 * the state rescaled to norm0) of every instance at once, into e[i] for instance i (host array of
 * sgpe_batch_size doubles).  Each class is one launch of each energy kernel over all its members
 * (grid y = member), their partials combined on the device; then one copy and one
 * synchronisation of the batch stream, instead of one per instance.  Equal to sgpe_batch_energy's
 * values up to the order of the final fp64 sums.  The argument tables and a device / pinned array of
 * one double per instance are allocated on the first call and kept by the batch.
 * Errors: SGPE_EINVAL (NULL), SGPE_ESTATE (an instance without a state), SGPE_ENOMEM, SGPE_EDEVICE,
 * SGPE_ENONFINITE (an energy not finite, or an instance's latched status; every e[i] is written and
 * a non-finite energy latches in its instance). */
sgpe_status sgpe_batch_energies(sgpe_batch* batch, double* e);

/* n steps of every instance (all must have a state: else SGPE_ESTATE); asynchronous on the batch
 * stream. */
sgpe_status sgpe_batch_step_real(sgpe_batch* batch, int64_t n);
sgpe_status sgpe_batch_step_imag(sgpe_batch* batch, int64_t n);
sgpe_status sgpe_batch_synchronize(sgpe_batch* batch);

/* Graph capture of step calls on (1, default) or off (0: launches are issued directly). */
sgpe_status sgpe_batch_use_graph(sgpe_batch* batch, int32_t on);

/* Schedule of class k (see sgpe_schedule; row_iters and col_iters must be 1).  NULL restores the
 * class default.  Synchronises; an unsupported schedule returns SGPE_EINVAL and changes nothing. */
sgpe_status sgpe_batch_get_schedule(const sgpe_batch* batch, int32_t k, sgpe_schedule* out);
sgpe_status sgpe_batch_set_schedule(sgpe_batch* batch, int32_t k, const sgpe_schedule* schedule);

/* Persistent mode (on = 1): each step_* call runs every steady-state step of every instance in one
 * cooperative launch of a persistent kernel (workgroups stay resident; work items of 1024 points
 * per component -- 1024 / nx rows or 1024 / ny columns of one instance -- taken round-robin; a
 * bounded grid-wide barrier between the row and the column phase of each step), with the call's
 * first and last passes as per-class launches: about 3 x classes + 1 launches per call instead of
 * 2 n + 2 per class.  Requires every class to be a square grid with nx = ny in {128, 256, 512} and
 * no spatial Raman coupling (SGPE_EINVAL otherwise), and a device with cooperative launches
 * (SGPE_EDEVICE).  The resident workgroups are split among the classes in proportion to their work.
 * Enabling sets every class's schedule to 8 points per lane, 1024 / nx rows per row workgroup and
 * 1024 / ny columns per column workgroup; while it is on, sgpe_batch_set_schedule and
 * sgpe_batch_autotune return SGPE_ESTATE.  Results: every instance bit-identical to a single
 * context with that schedule.  If a barrier wait ever gives up (it polls a bounded number of
 * times), every workgroup leaves, the states are invalid and sgpe_batch_synchronize returns
 * SGPE_EDEVICE (the environment variable SGPE_PERSIST_SPIN_LIMIT, read when the mode is enabled,
 * replaces the poll bound; 0 forces that path, for tests).  With graphs on, the call is captured as usual when the runtime can capture the
 * cooperative launch, and runs directly otherwise.  on = 0 returns to per-class launches (the
 * schedules stay).  Synchronises. */
sgpe_status sgpe_batch_use_persistent(sgpe_batch* batch, int32_t on);

/* Autotuner: for every class, time `steps` real-time steps under each supported schedule (points
 * per lane 4/8/16 in each pass, column tiles 1..16) and keep the fastest.  The instances' states
 * are saved before and restored after (so results do not depend on tuning); the captured graphs
 * are dropped.  best_ms, if not NULL, receives one value per class: the chosen schedule's time per
 * step of that class in milliseconds.  Synchronises. */
sgpe_status sgpe_batch_autotune(sgpe_batch* batch, int32_t steps, double* best_ms);

#ifdef __cplusplus
}
#endif

#endif /* SGPE_H */
