"""GPU parity of the complex128 instantiation of the step kernels (precision as a template
parameter of the same kernels) against the FP64 oracle, through the C ABI.

Both sides compute in fp64, so the bar is rounding: psi relative L2 <= 1e-12 and energies within
1e-11 (the two FFT algorithms round differently; measured after hundreds of steps: 2e-14 to 7e-14).  Cases: the tiny workload as written (64^2, complex128, imaginary then real time), the
512^2 real-time physics, the spatial Raman full 2x2 exponential, ragged and extreme shapes, the
full 1024^2 grid, 8 points per lane, unitarity, observables, and the complex128 schedule's limits."""
import os

import numpy as np
import pytest

import oracle
from oracle import OracleGPE
from workloads import Params, complex_noise, initial_state, preset, spin_hall_params, spin_hall_profile, vortex_state

pytestmark = pytest.mark.gpu

WORKERS = max(1, min(16, len(os.sched_getaffinity(0))))


@pytest.fixture(scope="module")
def Solver():
    from paper_2010_15069_amd import Solver, device_count
    if device_count() <= 0:
        pytest.skip("no HIP device")
    return Solver


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def pair(Solver, p, psi0):
    o = OracleGPE(p, workers=WORKERS)
    o.set_psi(psi0)
    s = Solver(p, precision="c128")
    s.set_psi(psi0)
    return o, s


def check(o, s, tol=1e-12, e_tol=1e-11):
    err = rel_l2(s.get_psi(), o.psi)
    assert err <= tol, f"psi rel L2 {err:.3e} > {tol:.0e}"
    eo, eg = o.energy(), s.energy()
    assert abs(eg - eo) <= e_tol * abs(eo), (eg, eo)
    no, ng = o.norm(), s.norm()
    assert abs(ng - no) <= 1e-12 * no, (ng, no)
    print(f"psi rel L2 {err:.2e}")


def test_tiny_as_written_complex128(Solver):
    p = preset("tiny")
    psi0 = initial_state(p, "gauss", seed=0)
    o, s = pair(Solver, p, psi0)
    o.step_imag(200)
    s.step_imag(200)
    check(o, s)
    o.step_real(200)
    s.step_real(200)
    check(o, s)


def test_state_round_trip_is_exact(Solver):
    p = preset("tiny")
    psi0 = initial_state(p, "gauss", seed=1) * (1 + 1e-9j)   # values not representable in complex64
    s = Solver(p, precision="c128").set_psi(psi0)
    assert np.array_equal(s.get_psi(), psi0)


def test_realtime_512(Solver):
    p = preset("realtime_512")
    o, s = pair(Solver, p, initial_state(p, "tf", seed=0))
    o.step_real(200)
    s.step_real(200)
    check(o, s)


@pytest.mark.parametrize("kind", ["imag", "real"])
def test_spatial_raman_full_2x2(Solver, kind):
    p = preset("ground_2048", nx=128, ny=128)
    o, s = pair(Solver, p, initial_state(p, "tf", seed=2))
    getattr(o, f"step_{kind}")(300)
    getattr(s, f"step_{kind}")(300)
    check(o, s)


@pytest.mark.parametrize("nx,ny", [(16, 16), (32, 256), (256, 32), (2048, 16), (16, 2048), (4096, 16), (16, 4096),
                                   (64, 4096), (128, 512)])
def test_ragged_shapes(Solver, nx, ny):
    p = Params(nx=nx, ny=ny, xmax=8.0, ymax=6.0, g_uu=3.0, g_dd=4.0, g_ud=2.0, k_l=1.3, omega=0.7, delta=0.2,
               dt=1e-3)
    o, s = pair(Solver, p, initial_state(p, "tf", seed=3))
    o.step_imag(50)
    s.step_imag(50)
    o.step_real(50)
    s.step_real(50)
    check(o, s)


SCHEDULES_C128 = [dict(row_points=16, col_points=16, col_tile=1), dict(row_points=8, col_points=16, col_tile=1),
                  dict(row_points=16, col_points=8, col_tile=1), dict(row_points=8, col_points=8, col_tile=2)]


# every (shape, schedule) pair the bounds allow: two 8-point columns of 1024 points would take 512
# threads, beyond the 256 a complex128 tile may use where one column needs fewer
POINTS_CASES = [(nx, ny, k) for nx, ny in [(1024, 1024), (64, 512), (512, 32)] for k in range(len(SCHEDULES_C128))
                if not (ny == 1024 and k == 3)]


@pytest.mark.parametrize("nx,ny,sched", POINTS_CASES)
def test_points_per_lane_schedules(Solver, nx, ny, sched):
    # the transforms at 16 and 8 points per lane in either pass (different radix decompositions,
    # the same bar); the default (8 up to 1024 points) runs in every other test here
    p = Params(nx=nx, ny=ny, xmax=10.0, ymax=9.0, g_uu=8.0, g_dd=6.0, g_ud=7.0, k_l=2.0, omega=1.0, delta=0.2,
               dt=1e-3)
    psi0 = initial_state(p, "tf", seed=7)
    o, s = pair(Solver, p, psi0)
    s.set_schedule(**SCHEDULES_C128[sched], row_tile=0)
    print(f"case: c128 {nx}x{ny} schedule {s.get_schedule()}", flush=True)
    steps = 5 if nx * ny >= 1 << 20 else 100
    o.step_imag(steps)
    s.step_imag(steps)
    o.step_real(steps)
    s.step_real(steps)
    check(o, s)


def test_full_size_1024(Solver):
    p = preset("metric_1024")
    o, s = pair(Solver, p, initial_state(p, "tf", seed=0))
    o.step_real(5)
    s.step_real(5)
    check(o, s)
    o.step_imag(5)
    s.step_imag(5)
    check(o, s)


def test_unitarity_1000_real_steps(Solver):
    p = preset("tiny")
    s = Solver(p, precision="c128").set_psi(initial_state(p, "gauss", seed=0))
    n0 = s.norm()
    s.step_real(1000)
    assert abs(s.norm() - n0) <= 1e-12 * n0


def test_observables_and_annealing(Solver):
    p = spin_hall_params(n=128, ratio=0.3)
    psi0 = vortex_state(p, n_vortices=5, seed=2)
    o = OracleGPE(p, workers=WORKERS)
    o.set_raman_profile(None, spin_hall_profile(p))
    o.set_psi(psi0)
    s = Solver(p, precision="c128").set_raman_profile(omega_y=spin_hall_profile(p)).set_psi(psi0)
    xi = complex_noise(p, seed=[2, 0])
    o.add_noise(xi, 1e-3)
    s.add_noise(xi, 1e-3)
    o.step_imag(100)
    s.step_imag(100)
    check(o, s)
    psi = s.get_psi()
    assert abs(s.phase_separation() - oracle.phase_separation(psi)) <= 1e-12
    r = s.population_radius(0.99)
    assert abs(r - oracle.population_radius(psi, p.xmax, p.ymax, 0.99)) <= 1e-9 * r
    (nu, nd), _ = oracle.winding(psi, p.xmax, p.ymax, r)
    assert s.winding(r)[:2] == (nu, nd)


def test_fixed_schedule_and_limits(Solver):
    from paper_2010_15069_amd import SgpeError
    from paper_2010_15069_amd._lib import lib
    p = preset("tiny")
    s = Solver(p, precision="c128").set_psi(initial_state(p, "gauss", seed=0))
    # 8 points per lane up to 1024 points per axis by default
    assert s.get_schedule()["row_points"] == 8 and s.get_schedule()["row_iters"] == 1
    default = s.get_schedule()
    # no prefetch, 16 or 8 points per lane only, at most 256 threads where a line needs fewer
    for bad in (dict(row_iters=2), dict(col_iters=2), dict(row_points=4), dict(col_points=4),
                dict(col_tile=64), dict(row_tile=64)):
        with pytest.raises(SgpeError, match="SGPE_EINVAL"):
            s.set_schedule(**bad)
        assert s.get_schedule() == default, bad
    with pytest.raises(SgpeError, match="SGPE_EINVAL"):
        s.set_col_tile(2)
    s.set_schedule(row_points=16, col_points=16, col_tile=1)
    assert s.get_schedule()["row_points"] == 16
    s.set_schedule(None)
    assert s.get_schedule() == default
    q = Params(nx=2048, ny=16, xmax=8.0, ymax=6.0)
    with pytest.raises(SgpeError, match="SGPE_EINVAL"):
        Solver(q, precision="c128").set_schedule(row_points=8)   # 8 points per lane up to 1024
    with pytest.raises(SgpeError, match="SGPE_EINVAL"):
        s.set_splitting("rkr", "frozen")
    with pytest.raises(SgpeError, match="SGPE_ESTATE"):
        s.profile_steps(5)
    with pytest.raises(ValueError):
        Solver(p, precision="c256")
    # complex128 columns of 4096 points run (their k_y values are read per point, not staged)
