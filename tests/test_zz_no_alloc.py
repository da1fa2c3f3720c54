"""sgpe_energy_noalloc (the allocation-free variant of sgpe_energy, for callers that cannot allocate)
against sgpe_energy, through the C ABI, on two calls in a row, the second on a smaller grid; on large
and extreme grids; and its error paths."""
import ctypes

import numpy as np
import pytest

from workloads import initial_state, preset

pytestmark = pytest.mark.gpu

SGPE_OK, SGPE_ESTATE = 0, 5


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2010_15069_amd import _lib, device_count
    if device_count() <= 0 or not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch, _lib.lib()


def _noalloc_energy(torch, lib, solver):
    out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    st = lib.sgpe_energy_noalloc(solver._ctx, ctypes.c_void_p(out.data_ptr()))
    assert st == SGPE_OK, st
    torch.cuda.synchronize()
    return float(out.cpu()[0])


def test_matches_energy_on_two_calls_second_smaller(env):
    torch, lib = env
    from paper_2010_15069_amd import Solver
    for n, seed in ((512, 0), (128, 1)):
        p = preset("ground_256", nx=n, ny=n)
        print(f"case: {n}x{n} energy_noalloc vs energy", flush=True)
        s = Solver(p).set_psi(initial_state(p, "tf", seed=seed))
        s.step_imag(20)
        e_ref = s.energy()
        e = _noalloc_energy(torch, lib, s)
        assert abs(e - e_ref) <= 1e-12 * abs(e_ref), (n, e, e_ref)
        s.close()


def test_spatial_raman_and_ragged_grid(env):
    torch, lib = env
    from paper_2010_15069_amd import Solver
    p = preset("ground_2048", nx=256, ny=64)
    s = Solver(p).set_psi(initial_state(p, "tf", seed=2))
    s.step_imag(10)
    e_ref = s.energy()
    assert abs(_noalloc_energy(torch, lib, s) - e_ref) <= 1e-12 * abs(e_ref)


def test_large_and_extreme_grids(env):
    # the static array holds only partial sums (three per row block, one per column block), so every grid
    # the library accepts fits: a full-size 2048 x 1024 grid and a 4096-point axis
    torch, lib = env
    from paper_2010_15069_amd import Solver
    for nx, ny in ((2048, 1024), (4096, 64), (64, 4096)):
        p = preset("ground_256", nx=nx, ny=ny)
        print(f"case: {nx}x{ny} energy_noalloc vs energy", flush=True)
        s = Solver(p).set_psi(initial_state(p, "tf", seed=0))
        s.step_imag(5)
        e_ref = s.energy()
        assert abs(_noalloc_energy(torch, lib, s) - e_ref) <= 1e-12 * abs(e_ref), (nx, ny)
        assert lib.sgpe_energy_noalloc(s._ctx, None) == 1      # SGPE_EINVAL
        s.close()


def test_no_state_is_an_error(env):
    torch, lib = env
    from paper_2010_15069_amd import Solver
    s = Solver(preset("tiny"))
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    assert lib.sgpe_energy_noalloc(s._ctx, ctypes.c_void_p(out.data_ptr())) == SGPE_ESTATE
