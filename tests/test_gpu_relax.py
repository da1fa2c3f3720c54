"""sgpe_relax_imag -- imaginary-time propagation to a ground state (Sec. 3.2) until an energy rule is
met, with the energy checks pipelined behind the steps -- against the same steps and checks made
one call at a time, and against the oracle's converged energy of the time-to-solution workload."""
import ctypes
import json
import os

import numpy as np
import pytest

from workloads import initial_state, preset

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
SGPE_EINVAL, SGPE_ENONFINITE, SGPE_ESTATE = 1, 4, 5


@pytest.fixture(scope="module")
def api():
    from paper_2010_15069_amd import Solver, _lib, device_count
    if device_count() <= 0:
        pytest.skip("no HIP device")
    return Solver, _lib.lib()


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_delta_rule_matches_checks_made_one_call_at_a_time(api, precision):
    Solver, _ = api
    p = preset("ground_256", nx=64, ny=64)
    psi0 = initial_state(p, "tf", seed=4)
    every, tol, cap = 50, 1e-5, 20000
    print(f"case: 64^2 {precision} relax_imag(delta {tol:g}, every {every}) vs step_imag + energy", flush=True)
    a = Solver(p, precision=precision).set_psi(psi0)
    r = a.relax_imag(check_every=every, max_steps=cap, rule="delta", tol=tol, record_energies=True)
    b = Solver(p, precision=precision).set_psi(psi0)
    es, steps = [b.energy()], 0
    while steps < cap:
        b.step_imag(every)
        steps += every
        es.append(b.energy())
        if abs(es[-1] - es[-2]) < tol * abs(es[-1]):
            break
    print(f"relax stopped at {r['steps']} steps ({r['checks']} checks), one call at a time at {steps}")
    assert r["met"] and r["steps"] == steps < cap and r["checks"] == len(es)
    # the same energies up to the order of the final fp64 sums (device vs host)
    np.testing.assert_allclose(r["energies"], es, rtol=1e-13, atol=0)
    assert r["energy"] == r["energies"][-1] and r["energy_prev"] == r["energies"][-2]
    # the chunks queued behind the stopping check ran: the same state as the same chunks one by one
    assert steps <= r["steps_taken"] <= steps + 2 * every and r["steps_taken"] % every == 0
    for _ in range((r["steps_taken"] - steps) // every):
        b.step_imag(every)
        b.synchronize()      # each of the driver's chunks is completed for its energy check
    assert np.array_equal(a.get_psi(), b.get_psi())
    a.close()
    b.close()


def test_target_rule_reaches_the_oracle_energy(api):
    Solver, _ = api
    ref = json.load(open(os.path.join(GOLDEN, "ground_energy.json")))
    p = preset(ref["workload"])
    e_ref = float(ref["energy"])
    print(f"case: {ref['workload']} relax_imag(target = oracle E_ref, 1e-6)", flush=True)
    s = Solver(p).set_psi(initial_state(p, "tf", seed=0))
    r = s.relax_imag(check_every=50, max_steps=200000, target=e_ref, tol=1e-6)
    assert r["met"] and abs(r["energy"] - e_ref) <= 1e-6 * abs(e_ref)
    assert abs(r["energy_prev"] - e_ref) > 1e-6 * abs(e_ref)      # the first check inside
    # the state left behind (up to two chunks further) is still there, and so is its norm
    e_now = s.energy()
    assert abs(e_now - e_ref) <= 1e-6 * abs(e_ref) and e_now <= r["energy"] + 1e-8 * abs(e_ref)
    assert abs(s.norm() - p.norm0) <= 1e-5 * p.norm0
    s.close()


def test_max_steps_caps_a_rule_that_is_never_met(api):
    Solver, _ = api
    p = preset("tiny")
    s = Solver(p).set_psi(initial_state(p, "gauss", seed=1))
    r = s.relax_imag(check_every=50, max_steps=120, rule="delta", tol=0.0, record_energies=True)
    # checks after 0, 50, 100 and 120 steps
    assert not r["met"] and r["checks"] == 4 and r["steps"] == 120 and r["steps_taken"] == 120
    assert abs(r["energies"][-1] - s.energy()) <= 1e-14 * abs(r["energies"][-1])
    r0 = s.relax_imag(check_every=7, max_steps=0, rule="delta", tol=1.0)
    assert r0["checks"] == 1 and r0["steps"] == 0 and r0["steps_taken"] == 0 and not r0["met"]
    s.close()


def test_overflowing_norm_stops_the_call(api):
    Solver, lib = api
    from paper_2010_15069_amd._lib import RelaxResult
    p = preset("tiny")
    good = initial_state(p, "gauss", seed=0)
    s = Solver(p)
    print("case: tiny 64^2, |psi| ~ 1e20, relax_imag", flush=True)
    s.set_psi(good * 1e20)          # finite in fp32; |psi|^2 ~ 1e40 is not
    res = RelaxResult()
    st = lib.sgpe_relax_imag(s._ctx, 10, 1000, 1, 0.0, 0.0, None, 0, ctypes.byref(res))
    assert st == SGPE_ENONFINITE
    assert res.met == 0 and res.checks <= 2 and res.steps_taken <= 30
    assert lib.sgpe_synchronize(s._ctx) == SGPE_ENONFINITE
    s.set_psi(good)
    assert s.relax_imag(check_every=10, max_steps=20, rule="delta", tol=0.0)["steps_taken"] == 20


def test_invalid_arguments(api):
    Solver, lib = api
    from paper_2010_15069_amd._lib import RelaxResult
    p = preset("tiny")
    s = Solver(p)
    res = RelaxResult()
    assert lib.sgpe_relax_imag(s._ctx, 10, 100, 1, 0.0, 0.0, None, 0, ctypes.byref(res)) == SGPE_ESTATE
    s.set_psi(initial_state(p, "gauss", seed=0))
    e = (ctypes.c_double * 4)()
    bad = [(0, 100, 1, 0.0, 0.0, None, 0, ctypes.byref(res)),            # check_every < 1
           (10, -1, 1, 0.0, 0.0, None, 0, ctypes.byref(res)),            # max_steps < 0
           (1 << 62, 100, 1, 0.0, 0.0, None, 0, ctypes.byref(res)),      # check_every above 2^61
           (10, 1 << 62, 1, 0.0, 0.0, None, 0, ctypes.byref(res)),       # max_steps above 2^61
           (10, 100, 2, 0.0, 0.0, None, 0, ctypes.byref(res)),           # unknown rule
           (10, 100, 0, float("nan"), 1e-6, None, 0, ctypes.byref(res)),  # target not finite
           (10, 100, 1, 0.0, -1.0, None, 0, ctypes.byref(res)),          # tol < 0
           (10, 100, 1, 0.0, float("inf"), None, 0, ctypes.byref(res)),  # tol not finite
           (10, 100, 1, 0.0, 0.0, None, 3, ctypes.byref(res)),           # NULL energies with a capacity
           (10, 100, 1, 0.0, 0.0, e, -1, ctypes.byref(res)),             # negative capacity
           (10, 100, 1, 0.0, 0.0, None, 0, None)]                        # NULL out
    for args in bad:
        assert lib.sgpe_relax_imag(s._ctx, *args) == SGPE_EINVAL, args
    s.close()
