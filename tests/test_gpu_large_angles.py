"""GPU parity, against the FP64 oracle, of the real-space exponential (Eqs. (H2)-(H4), Eq. (TEOp))
on the branches that large phases take.

Per point, the real-time row pass needs (cos(phi) - 1, sin(phi), sin(phi)/phi) of the real-space
angles.  |phi| <= pi/4 takes a short polynomial; beyond, a reduction by pi/2 (every quadrant, and
whole turns, where sin(r)/r of the reduced angle is not sin(phi)/phi).  In imaginary time the full
2x2 form takes cosh and sinh from exponentials once h|B| >= 0.25.  Each wave picks one routine per
point index by a vote of its lanes.  The workloads below put those angles where the state lives:

* a box [-16, 16)^2 with the harmonic trap and dt = 1/32 (exact in binary): h V reaches 8 rad at
  the corners, so |phi| runs from ~0 in the cloud through pi/4 (the circle r ~ 7.1, where the waves
  that cross it split their vote) to 2 pi and beyond; the 1e-3 seeded noise puts weight there;
* the same box with a spatial Raman profile Omega_x(x) + Omega_y(y) that is zero for |x|, |y| <= 4
  and grows quadratically outside, so that h|B| of the full 2x2 form reaches 7 rad;
* imaginary time with Omega(x) = 50 tanh(x / 4) and dt = 2e-2: h|B| = h Omega / 2 up to 0.5, at least
  0.25 on three quarters of the grid.  (Omega_0 = 200 with dt = 5e-3 reaches the same angles but is
  ill-conditioned for any complex64 transform: the oracle's own step with its FFTs taken in single
  precision, everything else exact, moves the state by 1e-3 within 100 steps.  The case here moves
  by 3e-6 under that emulation after 300 steps.)

Bars: complex64 psi relative L2 <= 1e-5 after 200 steps and energy within 1e-6; complex128 1e-12
and 1e-11.  The angles are rounded once to fp32 on the GPU (the oracle works in fp64), and that
rounding repeats every step: over 200 steps a phase of 8 rad drifts by up to ~1e-4 rad where it
acts.  Those points hold the noise (~1e-3 of the peak amplitude), so the drift contributes about
2e-6 of relative L2; a wrong branch (an O(1) error there) contributes ~1e-2.
"""
import math
import os

import numpy as np
import pytest

from oracle import OracleGPE
from workloads import Params, grid_axes, initial_state, preset

pytestmark = pytest.mark.gpu

WORKERS = max(1, min(16, len(os.sched_getaffinity(0))))
DT = 1.0 / 32.0
STEPS = 200


@pytest.fixture(scope="module")
def Solver():
    from paper_2010_15069_amd import Solver, device_count
    if device_count() <= 0:
        pytest.skip("no HIP device")
    return Solver


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def wide_box(**kw):
    base = dict(nx=128, ny=128, xmax=16.0, ymax=16.0, g_uu=10.0, g_dd=10.0, g_ud=10.0, delta=0.3, dt=DT)
    base.update(kw)
    return Params(**base)


def edge_profile(p):
    """Omega_x, Omega_y: zero for |coordinate| <= 4, 1.6 (|coordinate| - 4)^2 beyond."""
    x, y, _, _ = grid_axes(p)
    f = lambda u: 1.6 * np.maximum(np.abs(u) - 4.0, 0.0) ** 2
    return f(x), f(y)


def run_pair(Solver, p, psi0, kind, steps, precision, profile=None, splitting=None):
    o = OracleGPE(p, workers=WORKERS)
    s = Solver(p, precision=precision)
    if profile is not None:
        o.set_raman_profile(*profile)
        s.set_raman_profile(*profile)
    if splitting is not None:
        o.set_splitting(*splitting)
        s.set_splitting(*splitting)
    o.set_psi(psi0)
    s.set_psi(psi0)
    print(f"case: {p.nx}x{p.ny} {kind} {steps} steps {precision}", flush=True)
    getattr(o, f"step_{kind}")(steps)
    getattr(s, f"step_{kind}")(steps)
    return o, s


def check(o, s, psi_tol, e_tol):
    err = rel_l2(s.get_psi(), o.psi)
    eo, eg = o.energy(), s.energy()
    print(f"psi rel L2 {err:.3e}, energy {eg!r} vs {eo!r}")
    assert err <= psi_tol, f"psi rel L2 {err:.3e} > {psi_tol:.0e}"
    assert abs(eg - eo) <= e_tol * abs(eo), (eg, eo)


TOL = {"c64": (1e-5, 1e-6), "c128": (1e-12, 1e-11)}


def test_premise_angles_span_the_branches():
    # the workloads reach the angles the docstring names (fp64, from the parameters alone)
    p = wide_box()
    x, y, _, _ = grid_axes(p)
    X, Y = np.meshgrid(x, y)
    hv = p.dt * 0.5 * (X ** 2 + Y ** 2)
    assert hv.max() > 2 * math.pi + 1.0 and np.mean(hv > math.pi / 4) > 0.5
    ox, oy = edge_profile(p)
    th = p.dt * 0.5 * (ox[None, :] + oy[:, None])
    assert th.max() > 2 * math.pi and np.mean(th > math.pi / 4) > 0.3
    g = cosh_case()
    xg, _, _, _ = grid_axes(g)
    thi = g.dt * np.sqrt((0.5 * g.omega_r0 * np.tanh(xg / g.omega_rw)) ** 2 + (0.5 * g.delta) ** 2)
    assert thi.max() > 0.45 and np.mean(thi >= 0.25) > 0.5


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_real_time_diagonal_large_phases(Solver, precision):
    p = wide_box()
    o, s = run_pair(Solver, p, initial_state(p, "tf", seed=3), "real", STEPS, precision)
    check(o, s, *TOL[precision])


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_real_time_full_2x2_large_rotation(Solver, precision):
    p = wide_box(g_uu=10.0, g_dd=8.0, g_ud=6.0)
    o, s = run_pair(Solver, p, initial_state(p, "tf", seed=4), "real", STEPS, precision,
                    profile=edge_profile(p))
    check(o, s, *TOL[precision])


def test_real_time_full_2x2_nln_large_rotation(Solver):
    p = wide_box(g_uu=10.0, g_dd=8.0, g_ud=6.0)
    o, s = run_pair(Solver, p, initial_state(p, "tf", seed=5), "real", STEPS, "c64",
                    profile=edge_profile(p), splitting=("krk", "nln"))
    check(o, s, *TOL["c64"])


def cosh_case():
    return preset("ground_2048", nx=128, ny=128, omega_r0=50.0, dt=2e-2, delta=0.4)


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_imaginary_time_full_2x2_cosh_branch(Solver, precision):
    p = cosh_case()
    o, s = run_pair(Solver, p, initial_state(p, "tf", seed=6), "imag", 300, precision)
    check(o, s, *TOL[precision])
