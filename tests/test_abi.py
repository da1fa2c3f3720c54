"""Host-side checks of the C ABI: the library loads, exports every function include/sgpe.h
declares, validates parameters without a device, and reports the absence of a GPU."""
import ctypes
import os
import re

import pytest

from workloads import PRESETS, Params

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sgpe.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sgpe_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2010_15069_amd import _lib
    return _lib.lib()


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["sgpe_create", "sgpe_destroy", "sgpe_set_psi", "sgpe_get_psi", "sgpe_step_real",
              "sgpe_step_imag", "sgpe_energy", "sgpe_norm", "sgpe_strerror"]:
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_covers_every_declared_symbol():
    from paper_2010_15069_amd import _lib
    assert sorted(_lib.EXPORTS) == _declared()


def test_struct_layout_matches_header():
    # 2 int32 + 14 doubles, naturally aligned
    from paper_2010_15069_amd import SgpeParams
    assert ctypes.sizeof(SgpeParams) == 8 + 14 * 8
    assert SgpeParams.xmax.offset == 8
    body = re.search(r"typedef struct \{(.*?)\} sgpe_params;", open(HEADER).read(), flags=re.S).group(1)
    header_fields = re.findall(r"^\s*(?:int32_t|double)\s+([^;]+);", body, flags=re.M)
    names = [n.strip() for f in header_fields for n in f.split(",")]
    assert names == [f[0] for f in SgpeParams._fields_]
    assert names == list(Params().as_dict().keys())


@pytest.mark.parametrize("name", sorted(PRESETS))
def test_presets_validate(name):
    from paper_2010_15069_amd import validate_params
    assert validate_params(PRESETS[name]) == 0


@pytest.mark.parametrize("bad", [
    dict(nx=48), dict(ny=8), dict(nx=8192), dict(ny=0), dict(nx=-64),
    dict(xmax=0.0), dict(ymax=-1.0), dict(dt=0.0), dict(dt=-1e-3), dict(norm0=0.0),
    dict(wx=-1.0), dict(omega_r0=1.0, omega_rw=0.0), dict(g_uu=float("nan")),
    dict(dt=float("inf")), dict(k_l=float("nan")),
])
def test_invalid_params_rejected(bad):
    from paper_2010_15069_amd import validate_params
    assert validate_params(Params().replace(**bad)) == 1  # SGPE_EINVAL


def test_strerror_never_null(lib):
    for s in range(-1, 8):
        assert isinstance(lib.sgpe_strerror(s), bytes)


def test_null_arguments(lib):
    assert lib.sgpe_validate_params(None) == 1
    from paper_2010_15069_amd import SgpeParams
    p = SgpeParams.from_obj(Params())
    assert lib.sgpe_create(ctypes.byref(p), None, None, None) == 1
    # NULL context: every entry point returns SGPE_EINVAL, destroy is a no-op
    lib.sgpe_destroy(None)
    assert lib.sgpe_step_real(None, 1) == 1
    assert lib.sgpe_step_imag(None, 1) == 1
    assert lib.sgpe_set_psi(None, None) == 1
    assert lib.sgpe_get_psi(None, None) == 1
    d = ctypes.c_double()
    assert lib.sgpe_energy(None, ctypes.byref(d)) == 1
    assert lib.sgpe_norm(None, ctypes.byref(d)) == 1
    assert lib.sgpe_synchronize(None) == 1


def test_invalid_params_rejected_before_device_work(lib):
    from paper_2010_15069_amd import SgpeParams
    p = SgpeParams.from_obj(Params(nx=100))
    out = ctypes.c_void_p(1234)
    assert lib.sgpe_create(ctypes.byref(p), None, None, ctypes.byref(out)) == 1
    assert out.value is None


def test_no_device_reports_edevice(lib):
    if lib.sgpe_device_count() > 0:
        pytest.skip("a GPU is visible")
    from paper_2010_15069_amd import SgpeParams
    p = SgpeParams.from_obj(PRESETS["tiny"])
    out = ctypes.c_void_p()
    assert lib.sgpe_create(ctypes.byref(p), None, None, ctypes.byref(out)) == 3  # SGPE_EDEVICE
    assert out.value is None


def test_one_hip_runtime_in_process(lib):
    import torch  # noqa: F401  -- torch ships its own HIP runtime; libsgpe must reuse it
    maps = open("/proc/self/maps").read()
    hip = {l.split()[-1] for l in maps.splitlines() if "libamdhip64" in l}
    assert len(hip) == 1, hip


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    from paper_2010_15069_amd import _lib
    monkeypatch.setattr(_lib, "_LIB", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "libsgpe.so"))
    with pytest.raises(ImportError):
        _lib.lib()


def test_schedule_struct_matches_header():
    from paper_2010_15069_amd._lib import Schedule
    body = re.search(r"typedef struct \{([^{}]*)\} sgpe_schedule;", open(HEADER).read()).group(1)
    names = [n.strip() for n in re.findall(r"^\s*int32_t\s+([^;]+);", body, flags=re.M)]
    assert names == [f[0] for f in Schedule._fields_]
    assert ctypes.sizeof(Schedule) == 4 * len(names)


def test_batch_null_and_invalid_arguments(lib):
    from paper_2010_15069_amd import SgpeParams
    out = ctypes.c_void_p(1234)
    assert lib.sgpe_batch_create(None, 1, None, ctypes.byref(out)) == 1
    p = (SgpeParams * 2)(SgpeParams.from_obj(Params()), SgpeParams.from_obj(Params(nx=100)))
    out = ctypes.c_void_p(1234)
    assert lib.sgpe_batch_create(p, 2, None, ctypes.byref(out)) == 1      # second instance invalid
    assert out.value is None
    assert lib.sgpe_batch_create(p, 0, None, ctypes.byref(out)) == 1      # empty batch
    lib.sgpe_batch_destroy(None)
    assert lib.sgpe_batch_size(None) == 0 and lib.sgpe_batch_class_count(None) == 0
    assert lib.sgpe_batch_step_imag(None, 1) == 1
    assert lib.sgpe_batch_step_real(None, 1) == 1
    assert lib.sgpe_batch_synchronize(None) == 1
    assert lib.sgpe_batch_set_psi(None, 0, None) == 1
    d = ctypes.c_double()
    assert lib.sgpe_batch_energy(None, 0, ctypes.byref(d)) == 1
    assert lib.sgpe_batch_autotune(None, 1, None) == 1


def test_sweep_instances_are_seeded_and_in_range():
    from workloads import sweep_instances
    a, b = sweep_instances(seed=4), sweep_instances(seed=4)
    assert [x.as_dict() for x in a] == [x.as_dict() for x in b]
    assert [p.nx for p in a] == [128] * 32 + [256] * 32 + [512] * 32
    for p in a:
        assert 1.0 <= p.g_uu <= 100.0 and p.g_uu == p.g_dd == p.g_ud
        assert 0.0 <= p.omega <= 3.0 and -0.5 <= p.delta <= 0.5
        assert p.k_l == 2.0 and p.dt == 1e-3 and p.omega_r0 == 0.0
    assert len({p.g_uu for p in a}) == 96


def test_new_entry_points_reject_null_and_invalid_arguments(lib):
    # all of these fail before any device call
    from paper_2010_15069_amd import SgpeParams
    d = ctypes.c_double()
    n = (ctypes.c_int32 * 2)()
    assert lib.sgpe_set_splitting(None, 0, 0) == 1
    assert lib.sgpe_set_raman_profile(None, None, None) == 1
    assert lib.sgpe_add_noise(None, None, 1.0) == 1
    assert lib.sgpe_phase_separation(None, ctypes.byref(d)) == 1
    assert lib.sgpe_population_radius(None, 0.99, ctypes.byref(d)) == 1
    assert lib.sgpe_winding(None, 1.0, n, None) == 1
    out = ctypes.c_void_p(1234)
    p = SgpeParams.from_obj(Params())
    for prec in (-1, 2, 7):
        assert lib.sgpe_create_ex(ctypes.byref(p), prec, None, None, ctypes.byref(out)) == 1
        assert out.value is None
    assert lib.sgpe_create_ex(ctypes.byref(p), 1, None, None, None) == 1
    from paper_2010_15069_amd._lib import RelaxResult
    res = RelaxResult()
    assert lib.sgpe_relax_imag(None, 50, 100, 0, -1.0, 1e-6, None, 0, ctypes.byref(res)) == 1
    assert lib.sgpe_set_psi_device(None, None) == 1
    assert lib.sgpe_batch_set_psi_device(None, 0, None) == 1


def test_header_documents_precision_and_splitting_enums():
    h = open(HEADER).read()
    for name in ("SGPE_C64 = 0", "SGPE_C128 = 1", "SGPE_SPLIT_KRK = 0", "SGPE_SPLIT_RKR = 1",
                 "SGPE_RSPLIT_FROZEN = 0", "SGPE_RSPLIT_NLN = 1"):
        assert name in h, name


def _comment_before(decl_name):
    """The comment block that ends right before the declaration of decl_name."""
    text = open(HEADER).read()
    m = re.search(r"/\*((?:(?!\*/).)*)\*/\s*(?:typedef[^;]*;\s*)*(?:sgpe_status|void|int32_t|const char\*)\s+"
                  + decl_name + r"\s*\(", text, flags=re.S)
    assert m, decl_name
    return m.group(1)


@pytest.mark.parametrize("name", ["sgpe_create", "sgpe_create_ex", "sgpe_set_psi", "sgpe_get_psi",
                                  "sgpe_step_real", "sgpe_step_imag", "sgpe_energy", "sgpe_norm",
                                  "sgpe_synchronize", "sgpe_set_splitting", "sgpe_set_raman_profile",
                                  "sgpe_add_noise", "sgpe_phase_separation", "sgpe_winding",
                                  "sgpe_relax_imag", "sgpe_set_psi_device"])
def test_boundary_calls_cite_the_paper(name):
    # every call of the solver boundary names the passage that defines what it computes
    doc = _comment_before(name)
    assert re.search(r"\b(Sec\.|Eq\.|Eqs\.)", doc), f"{name}: no citation in {doc!r}"


def test_header_documents_the_nonfinite_latch():
    h = open(HEADER).read()
    assert "SGPE_ENONFINITE" in _comment_before("sgpe_synchronize")
    assert "clears" in _comment_before("sgpe_set_psi").lower()
    assert "status word" in h


def test_probe_rejects_invalid_arguments_before_device_work(lib):
    d = ctypes.c_double()
    assert lib.sgpe_probe_exchange(1000, 1024, 1, 1, 4, 0, 10, None, None, None) == 1   # not a power of two
    assert lib.sgpe_probe_exchange(1024, 1024, 3, 1, 4, 0, 10, None, None, None) == 1   # layout
    assert lib.sgpe_probe_exchange(1024, 1024, 1, 1, 4, 4, 10, None, None, None) == 1   # unknown flag
    assert lib.sgpe_probe_exchange(1024, 1024, 1, 16, 4, 0, 10, None, None, None) == 1  # 2048 threads
    assert lib.sgpe_probe_exchange(256, 1024, 1, 1, 1, 2, 10, None, None, None) == 1    # wave-local: >= 512
    assert lib.sgpe_probe_exchange(1024, 1024, 1, 1, 4, 0, 0, ctypes.byref(d), None, None) == 1   # reps
    out = (ctypes.c_uint32 * 8)()
    assert lib.sgpe_probe_placement(8, 1, 64, None) == 1            # NULL output
    assert lib.sgpe_probe_placement(0, 1, 64, out) == 1             # empty grid
    assert lib.sgpe_probe_placement(8, 70000, 64, out) == 1         # gy beyond the 2D limit
    assert lib.sgpe_probe_placement(8, 1, 2048, out) == 1           # more than 1024 threads
