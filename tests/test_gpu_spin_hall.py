"""GPU parity of the spin-Hall pieces (Sec. 6) against the FP64 oracle, through the C ABI:
the spatial Raman coupling along y in the real-space exponential (imaginary and real time, a
small grid and the full 1024^2 one), the annealing update, the observables (phase separation,
99 % population radius, winding numbers) on a shared state, one whole trial protocol at a small
size, and the error paths of the new entry points.

Bars: psi relative L2 <= 1e-5 (1e-6 after a few steps at full size), energies within 1e-6,
integer winding numbers exactly equal, real-valued observables to the precision their fp64
reductions allow."""
import math
import os

import numpy as np
import pytest

import oracle
from oracle import OracleGPE
from workloads import complex_noise, round_to_c64, spin_hall_params, spin_hall_profile, vortex_state

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
    prof = spin_hall_profile(p)
    o = OracleGPE(p, workers=WORKERS)
    o.set_raman_profile(None, prof)
    o.set_psi(psi0)
    s = Solver(p)
    s.set_raman_profile(omega_y=prof)
    s.set_psi(psi0)
    return o, s


def check(o, s, psi_tol, e_tol=1e-6):
    err = rel_l2(s.get_psi(), o.psi)
    assert err <= psi_tol, f"psi rel L2 {err:.3e} > {psi_tol:.1e}"
    eo, eg = o.energy(), s.energy()
    assert abs(eg - eo) <= e_tol * abs(eo), (eg, eo)
    return err


@pytest.mark.parametrize("ratio", [0.1, 0.8])
def test_y_profile_imag_then_real_256(Solver, ratio):
    p = spin_hall_params(n=256, ratio=ratio)
    o, s = pair(Solver, p, vortex_state(p, n_vortices=10, seed=1))
    o.step_imag(300)
    s.step_imag(300)
    check(o, s, 1e-5)
    o.step_real(200)
    s.step_real(200)
    check(o, s, 1e-5)


def test_y_profile_ragged_grid(Solver):
    p = spin_hall_params(n=128, ratio=0.3).replace(ny=64, ymax=12.0)
    o, s = pair(Solver, p, vortex_state(p, n_vortices=6, seed=2))
    o.step_imag(200)
    s.step_imag(200)
    check(o, s, 1e-5)


def test_x_and_y_profiles_together(Solver):
    # a tanh profile along x through the tables, added to the Sec. 6 profile along y
    p = spin_hall_params(n=128, ratio=0.2)
    x = -p.xmax + (2 * p.xmax / p.nx) * np.arange(p.nx)
    ox = 3.0 * np.tanh(x / 2.0)
    oy = spin_hall_profile(p)
    psi0 = vortex_state(p, n_vortices=8, seed=3)
    o = OracleGPE(p, workers=WORKERS)
    o.set_raman_profile(ox, oy)
    o.set_psi(psi0)
    s = Solver(p)
    s.set_raman_profile(ox, oy)
    s.set_psi(psi0)
    o.step_imag(150)
    s.step_imag(150)
    check(o, s, 1e-5)
    # switching the spatial coupling off again gives the plain diagonal exponential
    o.set_raman_profile(None, None)
    s.set_raman_profile(None, None)
    o.step_real(100)
    s.step_real(100)
    check(o, s, 1e-5)


def test_spin_hall_full_size_1024(Solver):
    p = spin_hall_params(n=1024, ratio=0.1)
    o, s = pair(Solver, p, vortex_state(p, n_vortices=50, seed=0))
    o.step_imag(5)
    s.step_imag(5)
    check(o, s, 1e-6)
    o.step_real(5)
    s.step_real(5)
    check(o, s, 1e-6)


def test_add_noise_parity(Solver):
    p = spin_hall_params(n=256, ratio=0.1)
    psi0 = vortex_state(p, n_vortices=5, seed=4)
    xi = complex_noise(p, seed=[4, 0])
    o, s = pair(Solver, p, psi0)
    o.add_noise(xi, 0.003)
    s.add_noise(xi, 0.003)
    assert rel_l2(s.get_psi(), o.psi) <= 1e-6
    before = s.get_psi()
    s.add_noise(xi, 0.0)
    assert np.array_equal(s.get_psi(), before)
    o.step_imag(100)
    s.step_imag(100)
    check(o, s, 1e-5)


@pytest.mark.parametrize("n", [256, 1024])
def test_observables_on_a_shared_state(Solver, n):
    p = spin_hall_params(n=n, ratio=0.2)
    o = OracleGPE(p, workers=WORKERS)
    o.set_raman_profile(None, spin_hall_profile(p))
    o.set_psi(vortex_state(p, n_vortices=12, seed=5))
    o.step_imag(3)
    psi = round_to_c64(o.psi)            # both sides see the same complex64 values
    s = Solver(p)
    s.set_psi(psi)
    sep_o = oracle.phase_separation(psi)
    assert abs(s.phase_separation() - sep_o) <= 1e-12 * max(1.0, abs(sep_o)) + 1e-14
    for f in (0.5, 0.9, 0.99):
        r_o = oracle.population_radius(psi, p.xmax, p.ymax, f)
        r_g = s.population_radius(f)
        assert abs(r_g - r_o) <= 1e-9 * r_o, (f, r_g, r_o)
    r99 = oracle.population_radius(psi, p.xmax, p.ymax, 0.99)
    (nu, nd), (ru, rd) = oracle.winding(psi, p.xmax, p.ymax, r99)
    gu, gd, graw_u, graw_d = s.winding(r99)
    assert (gu, gd) == (nu, nd) == (12, -12)
    assert abs(graw_u - ru) < 1e-9 and abs(graw_d - rd) < 1e-9
    for radius in (0.5, 2.0, 0.9 * p.xmax):
        (nu, nd), _ = oracle.winding(psi, p.xmax, p.ymax, radius)
        gu, gd, _, _ = s.winding(radius)
        assert (gu, gd) == (nu, nd), radius


def test_trial_protocol_matches_the_oracle(Solver):
    from paper_2010_15069_amd.spin_hall import run_trial
    n, seed, ratio = 128, 7, 0.3
    res = run_trial(ratio=ratio, seed=seed, n=n, segments=(600, 300), anneal_every=200, n_vortices=8,
                    return_psi=True)
    # unequal couplings with a spatial Raman profile: the driver takes the N L N real-space split
    assert res["real_space"] == "nln"
    # the same protocol on the oracle: anneal after 200 and 400 steps with amplitudes
    # amp0 (1 - 1/3) and amp0 (1 - 2/3) (the third anneal has amplitude zero), 300 plain steps
    p = spin_hall_params(n=n, ratio=ratio)
    psi0 = vortex_state(p, n_vortices=8, seed=seed)
    amp0 = 0.05 * float(np.abs(psi0).max())
    o = OracleGPE(p, workers=WORKERS)
    o.set_splitting("krk", "nln")
    o.set_raman_profile(None, spin_hall_profile(p))
    o.set_psi(psi0)
    for k, amp in enumerate((amp0 * 2 / 3, amp0 / 3)):
        o.step_imag(200)
        o.add_noise(complex_noise(p, seed=[seed, k]), amp)
    o.step_imag(200 + 300)
    err = rel_l2(res["psi"], o.psi)
    assert err <= 1e-5, err
    eo = o.energy()
    assert abs(res["energy"] - eo) <= 1e-6 * abs(eo)
    assert abs(res["phase_separation"] - oracle.phase_separation(o.psi)) <= 1e-5
    r99 = oracle.population_radius(o.psi, p.xmax, p.ymax, 0.99)
    assert abs(res["radius_99"] - r99) <= 2.0 * (2 * p.xmax / p.nx)
    (nu, nd), _ = oracle.winding(o.psi, p.xmax, p.ymax, res["radius_99"])
    assert (res["winding_up"], res["winding_down"]) == (nu, nd)


def test_error_paths(Solver):
    from paper_2010_15069_amd import SgpeError
    p = spin_hall_params(n=64, ratio=0.1)
    s = Solver(p)
    with pytest.raises(SgpeError, match="SGPE_ESTATE"):
        s.phase_separation()
    with pytest.raises(SgpeError, match="SGPE_ESTATE"):
        s.winding(1.0)
    with pytest.raises(SgpeError, match="SGPE_ESTATE"):
        s.add_noise(np.zeros((2, 64, 64), complex), 1.0)
    bad = spin_hall_profile(p).copy()
    bad[3] = np.nan
    with pytest.raises(SgpeError, match="SGPE_EINVAL"):
        s.set_raman_profile(omega_y=bad)
    psi0 = vortex_state(p, n_vortices=2, seed=0)
    s.set_psi(psi0)
    with pytest.raises(SgpeError, match="SGPE_EINVAL"):
        s.winding(p.xmax)
    with pytest.raises(SgpeError, match="SGPE_EINVAL"):
        s.winding(0.0)
    with pytest.raises(SgpeError, match="SGPE_EINVAL"):
        s.population_radius(0.0)
    with pytest.raises(SgpeError, match="SGPE_EINVAL"):
        s.population_radius(1.5)
    xi = np.zeros((2, 64, 64), complex)
    xi[1, 5, 5] = np.inf
    with pytest.raises(SgpeError, match="SGPE_ENONFINITE"):
        s.add_noise(xi, 1.0)
    assert np.array_equal(s.get_psi(), round_to_c64(psi0))   # unchanged
    with pytest.raises(SgpeError, match="SGPE_EINVAL"):
        s.add_noise(np.zeros((2, 64, 64), complex), math.inf)
    zero_dn = psi0.copy()
    zero_dn[1] = 0.0
    s.set_psi(zero_dn)
    with pytest.raises(SgpeError, match="SGPE_ESTATE"):
        s.phase_separation()
