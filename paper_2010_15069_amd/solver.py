"""Python face of the C ABI: one Solver per context.  Every step runs in libsgpe's HIP kernels;
this module only marshals arguments and owns the optional torch buffer/stream handles."""
from __future__ import annotations

import ctypes

import numpy as np

from ._lib import RELAX_RULES, RelaxResult, Schedule, SgpeParams, check, lib


class Solver:
    """Split-step solver context on the current HIP device.

    ``params``: any object (or dict) with the fields of ``workloads.Params`` / ``sgpe_params``.
    ``stream``: a raw hipStream_t handle (int) or None for the null stream; e.g.
    ``torch.cuda.current_stream().cuda_stream``.
    ``psi_dev``: optional device pointer (int) of >= 16*nx*ny bytes (32*nx*ny for complex128) that
    the context borrows, e.g. ``t.data_ptr()`` of a torch float32 tensor of shape (ny, nx, 4).
    ``precision``: "c64" (complex64 state, fp32 kernels) or "c128" (complex128, fp64 kernels).
    """

    PRECISIONS = {"c64": 0, "c128": 1}

    def __init__(self, params, stream=None, psi_dev=None, precision="c64"):
        self._lib = lib()
        self.params = params
        self._cp = SgpeParams.from_obj(params)
        self.nx, self.ny = int(self._cp.nx), int(self._cp.ny)
        if precision not in self.PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(self.PRECISIONS)}")
        self.precision = precision
        self._ctx = ctypes.c_void_p()
        check(self._lib.sgpe_create_ex(ctypes.byref(self._cp), self.PRECISIONS[precision],
                                       ctypes.c_void_p(stream or 0), ctypes.c_void_p(psi_dev or 0),
                                       ctypes.byref(self._ctx)),
              "sgpe_create_ex")

    # -- lifetime --------------------------------------------------------------------------
    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            self._lib.sgpe_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- state -----------------------------------------------------------------------------
    def set_psi(self, psi):
        a = np.ascontiguousarray(np.asarray(psi), dtype=np.complex128)
        if a.shape != (2, self.ny, self.nx):
            raise ValueError(f"psi must have shape (2, {self.ny}, {self.nx}), got {a.shape}")
        check(self._lib.sgpe_set_psi(self._ctx, a.ctypes.data_as(ctypes.c_void_p)), "sgpe_set_psi")
        return self

    def set_psi_device(self, t):
        """The state from a device tensor in the context's own layout (sgpe_set_psi_device): shape
        (ny, nx, 4) of (re_up, im_up, re_dn, im_dn), float32 (complex64 context) or float64
        (complex128), contiguous.  The tensor's current stream is synchronised first, so whatever
        produced it has finished."""
        _check_device_state(t, self.ny, self.nx, self.precision)
        import torch
        torch.cuda.current_stream(t.device).synchronize()
        check(self._lib.sgpe_set_psi_device(self._ctx, ctypes.c_void_p(t.data_ptr())), "sgpe_set_psi_device")
        return self

    def get_psi(self):
        out = np.empty((2, self.ny, self.nx), dtype=np.complex128)
        check(self._lib.sgpe_get_psi(self._ctx, out.ctypes.data_as(ctypes.c_void_p)), "sgpe_get_psi")
        return out

    # -- stepping --------------------------------------------------------------------------
    def step_real(self, n):
        check(self._lib.sgpe_step_real(self._ctx, int(n)), "sgpe_step_real")
        return self

    def step_imag(self, n):
        check(self._lib.sgpe_step_imag(self._ctx, int(n)), "sgpe_step_imag")
        return self

    def synchronize(self):
        check(self._lib.sgpe_synchronize(self._ctx), "sgpe_synchronize")

    def relax_imag(self, check_every=50, max_steps=200000, target=None, tol=1e-6, rule=None,
                   record_energies=False) -> dict:
        """Imaginary-time steps until an energy rule is met (sgpe_relax_imag): rule "target" (the
        default when a target energy is given) stops at |E - target| <= tol |target|, rule "delta"
        at |E_k - E_(k-1)| < tol |E_k|, the energy checked every `check_every` steps.  Returns the
        result fields, and with record_energies the energy of every check read."""
        rule = rule or ("target" if target is not None else "delta")
        n_checks = 1 + (int(max_steps) + int(check_every) - 1) // int(check_every)
        energies = np.full(n_checks, np.nan) if record_energies else None
        res = RelaxResult()
        ptr = energies.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if record_energies else None
        check(self._lib.sgpe_relax_imag(self._ctx, int(check_every), int(max_steps), RELAX_RULES[rule],
                                        float(target if target is not None else 0.0), float(tol), ptr,
                                        n_checks if record_energies else 0, ctypes.byref(res)),
              "sgpe_relax_imag")
        out = {f: getattr(res, f) for f, _ in RelaxResult._fields_ if f != "reserved"}
        out["met"] = bool(out["met"])
        if record_energies:
            out["energies"] = energies[:res.checks]
        return out

    # -- observables -----------------------------------------------------------------------
    def energy(self) -> float:
        v = ctypes.c_double()
        check(self._lib.sgpe_energy(self._ctx, ctypes.byref(v)), "sgpe_energy")
        return v.value

    def norm(self) -> float:
        v = ctypes.c_double()
        check(self._lib.sgpe_norm(self._ctx, ctypes.byref(v)), "sgpe_norm")
        return v.value

    def set_splitting(self, order="krk", real_space="frozen"):
        """Splitting variant: order "krk" (K(dt/2) R(dt) K(dt/2)) or "rkr" (R(dt/2) K(dt) R(dt/2));
        real_space "frozen" (one closed-form exponential) or "nln" (N(h/2) L(h) N(h/2))."""
        orders, splits = {"krk": 0, "rkr": 1}, {"frozen": 0, "nln": 1}
        if order not in orders or real_space not in splits:
            raise ValueError(f"unknown splitting {order!r}, {real_space!r}")
        check(self._lib.sgpe_set_splitting(self._ctx, orders[order], splits[real_space]), "sgpe_set_splitting")
        return self

    # -- spatial coupling, annealing and observables (Sec. 6) -------------------------------
    def set_raman_profile(self, omega_x=None, omega_y=None):
        """Spatial Raman coupling Omega_x(x_j) + Omega_y(y_i) (arrays of nx / ny values, or None
        for zero); both None switches it off."""
        def arr(v, n, name):
            if v is None:
                return None
            a = np.ascontiguousarray(np.asarray(v), dtype=np.float64)
            if a.shape != (n,):
                raise ValueError(f"{name} must have shape ({n},), got {a.shape}")
            return a
        ax, ay = arr(omega_x, self.nx, "omega_x"), arr(omega_y, self.ny, "omega_y")
        px = ax.ctypes.data_as(ctypes.c_void_p) if ax is not None else None
        py = ay.ctypes.data_as(ctypes.c_void_p) if ay is not None else None
        check(self._lib.sgpe_set_raman_profile(self._ctx, px, py), "sgpe_set_raman_profile")
        return self

    def add_noise(self, xi, amplitude):
        """psi <- psi + amplitude * xi (xi complex, shape (2, ny, nx))."""
        a = np.ascontiguousarray(np.asarray(xi), dtype=np.complex128)
        if a.shape != (2, self.ny, self.nx):
            raise ValueError(f"xi must have shape (2, {self.ny}, {self.nx}), got {a.shape}")
        check(self._lib.sgpe_add_noise(self._ctx, a.ctypes.data_as(ctypes.c_void_p), float(amplitude)),
              "sgpe_add_noise")
        return self

    def phase_separation(self) -> float:
        v = ctypes.c_double()
        check(self._lib.sgpe_phase_separation(self._ctx, ctypes.byref(v)), "sgpe_phase_separation")
        return v.value

    def population_radius(self, fraction=0.99) -> float:
        v = ctypes.c_double()
        check(self._lib.sgpe_population_radius(self._ctx, float(fraction), ctypes.byref(v)),
              "sgpe_population_radius")
        return v.value

    def winding(self, radius):
        """(n_up, n_down, raw_up, raw_down): winding numbers along the circle of this radius and
        the unrounded phase sums over 2 pi."""
        n = (ctypes.c_int32 * 2)()
        raw = (ctypes.c_double * 2)()
        check(self._lib.sgpe_winding(self._ctx, float(radius), n, raw), "sgpe_winding")
        return int(n[0]), int(n[1]), float(raw[0]), float(raw[1])

    # -- measurement / tuning --------------------------------------------------------------
    def profile_steps(self, n, imag=False):
        """Mean per-launch milliseconds of (row pass, column pass) over n steady-state steps."""
        r, c = ctypes.c_double(), ctypes.c_double()
        check(self._lib.sgpe_profile_steps(self._ctx, 1 if imag else 0, int(n), ctypes.byref(r),
                                           ctypes.byref(c)), "sgpe_profile_steps")
        return r.value, c.value

    def profile_kernels(self, n, imag=False):
        """Mean milliseconds of one (row pass, column pass) launch, each from n back-to-back
        launches; the state is left unchanged."""
        r, c = ctypes.c_double(), ctypes.c_double()
        check(self._lib.sgpe_profile_kernels(self._ctx, 1 if imag else 0, int(n), ctypes.byref(r),
                                             ctypes.byref(c)), "sgpe_profile_kernels")
        return r.value, c.value

    def get_schedule(self) -> dict:
        sc = Schedule()
        check(self._lib.sgpe_get_schedule(self._ctx, ctypes.byref(sc)), "sgpe_get_schedule")
        return {name: int(getattr(sc, name)) for name, _ in Schedule._fields_}

    def set_schedule(self, schedule=None, **fields):
        """Set the launch schedule from a dict and/or keyword fields, the unnamed fields kept;
        set_schedule(None) with no fields restores the default."""
        if schedule is None and not fields:
            check(self._lib.sgpe_set_schedule(self._ctx, None), "sgpe_set_schedule")
            return self
        cur = self.get_schedule()
        changes = dict(schedule or {}, **fields)
        if "row_points" in changes and "row_tile" not in changes:
            cur["row_tile"] = 0          # the default tile for the new points per lane
        cur.update(changes)
        sc = Schedule(**{k: int(v) for k, v in cur.items()})
        check(self._lib.sgpe_set_schedule(self._ctx, ctypes.byref(sc)), "sgpe_set_schedule")
        return self

    def set_col_tile(self, columns):
        check(self._lib.sgpe_set_col_tile(self._ctx, int(columns)), "sgpe_set_col_tile")
        return self


class Batch:
    """Many independent solver instances (any mix of grid shapes) stepped together; see the
    sgpe_batch_* calls in include/sgpe.h.  ``params``: a sequence of parameter objects/dicts."""

    def __init__(self, params, stream=None):
        self._lib = lib()
        self.params = list(params)
        n = len(self.params)
        arr = (SgpeParams * n)(*[SgpeParams.from_obj(p) for p in self.params])
        self._shapes = [(int(a.ny), int(a.nx)) for a in arr]
        self._b = ctypes.c_void_p()
        check(self._lib.sgpe_batch_create(arr, n, ctypes.c_void_p(stream or 0), ctypes.byref(self._b)),
              "sgpe_batch_create")

    def close(self):
        if getattr(self, "_b", None) is not None and self._b.value:
            self._lib.sgpe_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __len__(self):
        return int(self._lib.sgpe_batch_size(self._b))

    def classes(self):
        """[(nx, ny, members)] per class."""
        out = []
        for k in range(int(self._lib.sgpe_batch_class_count(self._b))):
            nx, ny, m = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
            check(self._lib.sgpe_batch_class_info(self._b, k, ctypes.byref(nx), ctypes.byref(ny),
                                                  ctypes.byref(m)), "sgpe_batch_class_info")
            out.append((nx.value, ny.value, m.value))
        return out

    def instance_class(self, i):
        k = ctypes.c_int32()
        check(self._lib.sgpe_batch_instance_class(self._b, int(i), ctypes.byref(k)), "sgpe_batch_instance_class")
        return k.value

    def set_psi(self, i, psi):
        ny, nx = self._shapes[i]
        a = np.ascontiguousarray(np.asarray(psi), dtype=np.complex128)
        if a.shape != (2, ny, nx):
            raise ValueError(f"psi must have shape (2, {ny}, {nx}), got {a.shape}")
        check(self._lib.sgpe_batch_set_psi(self._b, int(i), a.ctypes.data_as(ctypes.c_void_p)), "sgpe_batch_set_psi")
        return self

    def set_psi_device(self, i, t):
        """Instance i's state from a device tensor, as Solver.set_psi_device (complex64)."""
        ny, nx = self._shapes[i]
        _check_device_state(t, ny, nx, "c64")
        import torch
        torch.cuda.current_stream(t.device).synchronize()
        check(self._lib.sgpe_batch_set_psi_device(self._b, int(i), ctypes.c_void_p(t.data_ptr())),
              "sgpe_batch_set_psi_device")
        return self

    def get_psi(self, i):
        ny, nx = self._shapes[i]
        out = np.empty((2, ny, nx), dtype=np.complex128)
        check(self._lib.sgpe_batch_get_psi(self._b, int(i), out.ctypes.data_as(ctypes.c_void_p)),
              "sgpe_batch_get_psi")
        return out

    def step_real(self, n):
        check(self._lib.sgpe_batch_step_real(self._b, int(n)), "sgpe_batch_step_real")
        return self

    def step_imag(self, n):
        check(self._lib.sgpe_batch_step_imag(self._b, int(n)), "sgpe_batch_step_imag")
        return self

    def synchronize(self):
        check(self._lib.sgpe_batch_synchronize(self._b), "sgpe_batch_synchronize")
        return self

    def energy(self, i) -> float:
        v = ctypes.c_double()
        check(self._lib.sgpe_batch_energy(self._b, int(i), ctypes.byref(v)), "sgpe_batch_energy")
        return v.value

    def energies(self):
        """Every instance's energy per particle at once (sgpe_batch_energies), as a numpy array."""
        out = np.empty(len(self), dtype=np.float64)
        check(self._lib.sgpe_batch_energies(self._b, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
              "sgpe_batch_energies")
        return out

    def norm(self, i) -> float:
        v = ctypes.c_double()
        check(self._lib.sgpe_batch_norm(self._b, int(i), ctypes.byref(v)), "sgpe_batch_norm")
        return v.value

    def use_persistent(self, on=True):
        """Every steady-state step of every instance in one cooperative persistent launch per call
        (see sgpe_batch_use_persistent)."""
        check(self._lib.sgpe_batch_use_persistent(self._b, int(bool(on))), "sgpe_batch_use_persistent")
        return self

    def use_graph(self, on=True):
        check(self._lib.sgpe_batch_use_graph(self._b, 1 if on else 0), "sgpe_batch_use_graph")
        return self

    def get_schedule(self, k) -> dict:
        sc = Schedule()
        check(self._lib.sgpe_batch_get_schedule(self._b, int(k), ctypes.byref(sc)), "sgpe_batch_get_schedule")
        return {name: int(getattr(sc, name)) for name, _ in Schedule._fields_}

    def set_schedule(self, k, schedule=None, **fields):
        if schedule is None and not fields:
            check(self._lib.sgpe_batch_set_schedule(self._b, int(k), None), "sgpe_batch_set_schedule")
            return self
        cur = self.get_schedule(k)
        changes = dict(schedule or {}, **fields)
        if "row_points" in changes and "row_tile" not in changes:
            cur["row_tile"] = 0          # the default tile for the new points per lane
        cur.update(changes)
        sc = Schedule(**{key: int(v) for key, v in cur.items()})
        check(self._lib.sgpe_batch_set_schedule(self._b, int(k), ctypes.byref(sc)), "sgpe_batch_set_schedule")
        return self

    def autotune(self, steps=10):
        """Per class: the fastest schedule over the supported set (states kept); returns the
        chosen per-class time per step in ms."""
        ms = (ctypes.c_double * max(1, len(self.classes())))()
        check(self._lib.sgpe_batch_autotune(self._b, int(steps), ms), "sgpe_batch_autotune")
        return list(ms)


def _check_device_state(t, ny, nx, precision):
    import torch
    want = torch.float64 if precision == "c128" else torch.float32
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == want and t.is_contiguous()
            and tuple(t.shape) == (ny, nx, 4)):
        raise ValueError(f"expected a contiguous {want} device tensor of shape ({ny}, {nx}, 4)")


def device_count() -> int:
    return int(lib().sgpe_device_count())


def validate_params(params) -> int:
    p = SgpeParams.from_obj(params)
    return int(lib().sgpe_validate_params(ctypes.byref(p)))


def probe_exchange(nx, ny, layout_rows=1, row_tile=1, col_tile=4, write_through=True, wave_local=False, reps=50):
    """sgpe_probe_exchange: mean milliseconds of (row-partition launch, column-partition launch,
    row + column round back to back) of the arithmetic-free copy with a step's data movement (see
    include/sgpe.h)."""
    r, c, pr = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    flags = (1 if write_through else 0) | (2 if wave_local else 0)
    check(lib().sgpe_probe_exchange(int(nx), int(ny), int(layout_rows), int(row_tile), int(col_tile), flags,
                                    int(reps), ctypes.byref(r), ctypes.byref(c), ctypes.byref(pr)),
          "sgpe_probe_exchange")
    return r.value, c.value, pr.value


def probe_placement(gx, gy=1, threads=256):
    """sgpe_probe_placement: the XCD index that ran each workgroup of a gx x gy grid, as a numpy
    array of shape (gy, gx)."""
    out = (ctypes.c_uint32 * (int(gx) * int(gy)))()
    check(lib().sgpe_probe_placement(int(gx), int(gy), int(threads), out), "sgpe_probe_placement")
    return np.frombuffer(out, dtype=np.uint32).reshape(int(gy), int(gx)).copy()
