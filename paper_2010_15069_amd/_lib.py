"""ctypes binding of libsgpe.so (include/sgpe.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes
import importlib.util
import os

_PKG_DIR = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG_DIR, "libsgpe.so")

SGPE_OK, SGPE_EINVAL, SGPE_ENOMEM, SGPE_EDEVICE, SGPE_ENONFINITE, SGPE_ESTATE = range(6)
STATUS_NAMES = {0: "SGPE_OK", 1: "SGPE_EINVAL", 2: "SGPE_ENOMEM", 3: "SGPE_EDEVICE",
                4: "SGPE_ENONFINITE", 5: "SGPE_ESTATE"}


class SgpeParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("xmax", ctypes.c_double), ("ymax", ctypes.c_double),
        ("g_uu", ctypes.c_double), ("g_dd", ctypes.c_double), ("g_ud", ctypes.c_double),
        ("k_l", ctypes.c_double), ("omega", ctypes.c_double), ("delta", ctypes.c_double),
        ("wx", ctypes.c_double), ("wy", ctypes.c_double),
        ("omega_r0", ctypes.c_double), ("omega_rw", ctypes.c_double),
        ("dt", ctypes.c_double), ("norm0", ctypes.c_double),
    ]

    @classmethod
    def from_obj(cls, p) -> "SgpeParams":
        """From any object (or dict) with the fields of workloads.Params."""
        get = (lambda k: p[k]) if isinstance(p, dict) else (lambda k: getattr(p, k))
        out = cls()
        for name, ctype in cls._fields_:
            v = get(name)
            setattr(out, name, int(v) if ctype is ctypes.c_int32 else float(v))
        return out


class Schedule(ctypes.Structure):
    """sgpe_schedule: launch schedule of the two passes (see include/sgpe.h)."""
    _fields_ = [("col_tile", ctypes.c_int32), ("row_iters", ctypes.c_int32),
                ("col_iters", ctypes.c_int32), ("row_points", ctypes.c_int32),
                ("col_points", ctypes.c_int32), ("row_tile", ctypes.c_int32)]


class RelaxResult(ctypes.Structure):
    """sgpe_relax_result: where sgpe_relax_imag stopped (see include/sgpe.h)."""
    _fields_ = [("steps", ctypes.c_int64), ("steps_taken", ctypes.c_int64), ("checks", ctypes.c_int64),
                ("energy", ctypes.c_double), ("energy_prev", ctypes.c_double), ("met", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


RELAX_RULES = {"target": 0, "delta": 1}


class SgpeError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = int(status)
        msg = _lib().sgpe_strerror(self.status).decode() if _LIB is not None else ""
        super().__init__(f"{where}: {STATUS_NAMES.get(self.status, self.status)} ({msg})")


_LIB = None

EXPORTS = [
    "sgpe_validate_params", "sgpe_device_count", "sgpe_create", "sgpe_destroy", "sgpe_set_psi",
    "sgpe_get_psi", "sgpe_step_real", "sgpe_step_imag", "sgpe_energy", "sgpe_norm",
    "sgpe_synchronize", "sgpe_profile_steps", "sgpe_profile_kernels", "sgpe_strerror",
    "sgpe_set_col_tile", "sgpe_get_schedule", "sgpe_set_schedule",
    "sgpe_batch_create", "sgpe_batch_destroy", "sgpe_batch_size", "sgpe_batch_class_count",
    "sgpe_batch_class_info", "sgpe_batch_instance_class", "sgpe_batch_set_psi", "sgpe_batch_get_psi",
    "sgpe_batch_energy", "sgpe_batch_norm", "sgpe_batch_step_real", "sgpe_batch_step_imag",
    "sgpe_batch_synchronize", "sgpe_batch_use_graph", "sgpe_batch_get_schedule",
    "sgpe_batch_set_schedule", "sgpe_batch_autotune", "sgpe_batch_use_persistent",
    "sgpe_set_raman_profile", "sgpe_add_noise", "sgpe_phase_separation", "sgpe_population_radius",
    "sgpe_winding", "sgpe_set_splitting", "sgpe_create_ex", "sgpe_probe_exchange", "sgpe_energy_noalloc",
    "sgpe_probe_placement", "sgpe_relax_imag", "sgpe_batch_energies", "sgpe_set_psi_device",
    "sgpe_batch_set_psi_device",
]


def _preload_hip_runtime():
    """PyTorch ships its own HIP runtime (SONAME libamdhip64.so.7, file libamdhip64.so).  Load
    that file first so that libsgpe's dependency resolves to it whether or not torch is imported
    before or after us: one process must never hold two HIP runtimes."""
    spec = importlib.util.find_spec("torch")
    if spec is None or not spec.submodule_search_locations:
        return
    path = os.path.join(list(spec.submodule_search_locations)[0], "lib", "libamdhip64.so")
    if os.path.exists(path):
        ctypes.CDLL(path, mode=ctypes.RTLD_GLOBAL)


def _lib():
    """Load libsgpe.so; raises if it has not been built (there is no fallback path)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2010_15069_amd.build`")
    _preload_hip_runtime()
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    st = ctypes.c_int
    lib.sgpe_validate_params.argtypes = [P(SgpeParams)]
    lib.sgpe_validate_params.restype = st
    lib.sgpe_device_count.argtypes = []
    lib.sgpe_device_count.restype = ctypes.c_int32
    lib.sgpe_create.argtypes = [P(SgpeParams), vp, vp, P(vp)]
    lib.sgpe_create.restype = st
    lib.sgpe_destroy.argtypes = [vp]
    lib.sgpe_destroy.restype = None
    lib.sgpe_set_psi.argtypes = [vp, vp]
    lib.sgpe_set_psi.restype = st
    lib.sgpe_get_psi.argtypes = [vp, vp]
    lib.sgpe_get_psi.restype = st
    lib.sgpe_step_real.argtypes = [vp, ctypes.c_int64]
    lib.sgpe_step_real.restype = st
    lib.sgpe_step_imag.argtypes = [vp, ctypes.c_int64]
    lib.sgpe_step_imag.restype = st
    lib.sgpe_energy.argtypes = [vp, P(ctypes.c_double)]
    lib.sgpe_energy.restype = st
    lib.sgpe_norm.argtypes = [vp, P(ctypes.c_double)]
    lib.sgpe_norm.restype = st
    lib.sgpe_synchronize.argtypes = [vp]
    lib.sgpe_synchronize.restype = st
    lib.sgpe_profile_steps.argtypes = [vp, ctypes.c_int32, ctypes.c_int64, P(ctypes.c_double),
                                       P(ctypes.c_double)]
    lib.sgpe_profile_steps.restype = st
    lib.sgpe_profile_kernels.argtypes = [vp, ctypes.c_int32, ctypes.c_int64, P(ctypes.c_double),
                                         P(ctypes.c_double)]
    lib.sgpe_profile_kernels.restype = st
    lib.sgpe_get_schedule.argtypes = [vp, P(Schedule)]
    lib.sgpe_get_schedule.restype = st
    lib.sgpe_set_schedule.argtypes = [vp, P(Schedule)]
    lib.sgpe_set_schedule.restype = st
    lib.sgpe_strerror.argtypes = [ctypes.c_int]
    lib.sgpe_strerror.restype = ctypes.c_char_p
    lib.sgpe_set_col_tile.argtypes = [vp, ctypes.c_int32]
    lib.sgpe_set_col_tile.restype = st
    i32, i64, PI32 = ctypes.c_int32, ctypes.c_int64, P(ctypes.c_int32)
    batch_sigs = {
        "sgpe_batch_create": ([P(SgpeParams), i32, vp, P(vp)], st),
        "sgpe_batch_destroy": ([vp], None),
        "sgpe_batch_size": ([vp], i32),
        "sgpe_batch_class_count": ([vp], i32),
        "sgpe_batch_class_info": ([vp, i32, PI32, PI32, PI32], st),
        "sgpe_batch_instance_class": ([vp, i32, PI32], st),
        "sgpe_batch_set_psi": ([vp, i32, vp], st),
        "sgpe_batch_get_psi": ([vp, i32, vp], st),
        "sgpe_batch_energy": ([vp, i32, P(ctypes.c_double)], st),
        "sgpe_batch_norm": ([vp, i32, P(ctypes.c_double)], st),
        "sgpe_batch_step_real": ([vp, i64], st),
        "sgpe_batch_step_imag": ([vp, i64], st),
        "sgpe_batch_synchronize": ([vp], st),
        "sgpe_batch_use_graph": ([vp, i32], st),
        "sgpe_batch_get_schedule": ([vp, i32, P(Schedule)], st),
        "sgpe_batch_set_schedule": ([vp, i32, P(Schedule)], st),
        "sgpe_batch_autotune": ([vp, i32, P(ctypes.c_double)], st),
        "sgpe_batch_use_persistent": ([vp, i32], st),
    }
    batch_sigs.update({
        "sgpe_set_raman_profile": ([vp, vp, vp], st),
        "sgpe_add_noise": ([vp, vp, ctypes.c_double], st),
        "sgpe_phase_separation": ([vp, P(ctypes.c_double)], st),
        "sgpe_population_radius": ([vp, ctypes.c_double, P(ctypes.c_double)], st),
        "sgpe_winding": ([vp, ctypes.c_double, PI32, P(ctypes.c_double)], st),
        "sgpe_set_splitting": ([vp, i32, i32], st),
        "sgpe_create_ex": ([P(SgpeParams), i32, vp, vp, P(vp)], st),
        "sgpe_probe_exchange": ([i32, i32, i32, i32, i32, i32, i32, P(ctypes.c_double), P(ctypes.c_double),
                                 P(ctypes.c_double)], st),
        "sgpe_energy_noalloc": ([vp, vp], st),
        "sgpe_probe_placement": ([i32, i32, i32, P(ctypes.c_uint32)], st),
        "sgpe_relax_imag": ([vp, ctypes.c_int64, ctypes.c_int64, i32, ctypes.c_double, ctypes.c_double,
                             P(ctypes.c_double), ctypes.c_int64, P(RelaxResult)], st),
        "sgpe_batch_energies": ([vp, P(ctypes.c_double)], st),
        "sgpe_set_psi_device": ([vp, vp], st),
        "sgpe_batch_set_psi_device": ([vp, i32, vp], st),
    })
    for name, (args, res) in batch_sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _LIB = lib
    return lib


def lib():
    return _lib()


def check(status: int, where: str) -> None:
    if status != SGPE_OK:
        raise SgpeError(status, where)
