"""Pins of the oracle's splitting variants (Sec. 3.2): the R(dt/2) K(dt) R(dt/2) ordering and the
second-order real-space split N(h/2) L(h) N(h/2), against results fixed independently of them.

* the real-space sub-step against a high-order ODE integration (scipy's DOP853) of
  i psi' = H_R(n(psi)) psi at one point: local error O(h^3) for N L N, O(h^2) for frozen densities
  (the caveat that motivates the variant: unequal couplings and a spatial Raman term);
* the R-K-R step on a plane wave against a 2x2 matrix power built with scipy.linalg.expm;
* the R-K-R imaginary-time fixed point of a linear problem against numpy.linalg.eigh;
* second-order convergence in dt of whole trajectories.
Planted mutants are caught."""
import math

import numpy as np
import pytest
import scipy.linalg as sla
from scipy.integrate import solve_ivp

import oracle.gpe as og
from oracle import OracleGPE
from workloads import Params, gaussian_state, grid_axes

from .test_oracle_pins import _dense_hamiltonian


def _uniform_point_case():
    p = Params(nx=16, ny=16, wx=0.0, wy=0.0, g_uu=3.0, g_dd=1.0, g_ud=2.0, delta=0.4)
    o = OracleGPE(p)
    o.set_raman_profile(np.full(16, 1.3), None)
    u0, d0 = 0.8 + 0.1j, 0.3 - 0.5j
    psi0 = np.stack([np.full((16, 16), u0), np.full((16, 16), d0)])

    def exact(h):
        def f(t, y):
            u, d = y[0] + 1j * y[1], y[2] + 1j * y[3]
            nu, nd = abs(u) ** 2, abs(d) ** 2
            du = -1j * ((p.delta / 2 + p.g_uu * nu + p.g_ud * nd) * u + 0.65 * d)
            dd = -1j * ((-p.delta / 2 + p.g_dd * nd + p.g_ud * nu) * d + 0.65 * u)
            return [du.real, du.imag, dd.real, dd.imag]
        y = solve_ivp(f, (0.0, h), [u0.real, u0.imag, d0.real, d0.imag], rtol=1e-13, atol=1e-14,
                      method="DOP853").y[:, -1]
        return np.array([y[0] + 1j * y[1], y[2] + 1j * y[3]])
    return o, psi0, exact


def _local_error_ratio(real_space):
    o, psi0, exact = _uniform_point_case()
    o.set_splitting("krk", real_space)
    e = [np.abs(o.apply_R(psi0, h, False)[:, 0, 0] - exact(h)).max() for h in (0.1, 0.05)]
    return e[0] / e[1]


def test_nln_real_space_split_is_locally_third_order():
    assert 7.0 < _local_error_ratio("nln") < 9.5


def test_frozen_densities_are_locally_second_order_only():
    assert 3.5 < _local_error_ratio("frozen") < 4.5


def test_nln_equals_frozen_without_spatial_coupling_in_real_time():
    # with Omega(r) = 0 every real-space piece is a diagonal phase that keeps the densities
    p = Params(nx=32, ny=16, g_uu=3.0, g_dd=1.5, g_ud=2.0, delta=0.3, k_l=1.1, omega=0.6, dt=2e-3)
    psi0 = gaussian_state(p, noise=0.05, seed=2)
    a, b = OracleGPE(p), OracleGPE(p)
    a.set_splitting("krk", "frozen")
    b.set_splitting("krk", "nln")
    a.set_psi(psi0)
    b.set_psi(psi0)
    a.step_real(30)
    b.step_real(30)
    assert np.max(np.abs(a.psi - b.psi)) < 1e-12


def test_rkr_plane_wave_matrix_power():
    # V = 0, no spatial coupling, equal couplings: the total density of a plane wave stays uniform
    # and constant, so one R-K-R step at k0 is D U_K(dt) D with D the mean-field/detuning phase of
    # dt/2 and U_K = expm(-i dt H_K(k0)).
    g, delta, k_l, om = 1.7, 0.35, 1.2, 0.9
    p = Params(nx=16, ny=16, xmax=4.0, ymax=3.0, wx=0.0, wy=0.0, g_uu=g, g_dd=g, g_ud=g, delta=delta,
               k_l=k_l, omega=om, dt=3e-3)
    x, y, _, _ = grid_axes(p)
    X, Y = np.meshgrid(x, y)
    k0x, k0y = 2 * math.pi / p.xmax, -math.pi / p.ymax
    a, b = 0.6 + 0.2j, -0.3 + 0.5j
    ph = np.exp(1j * (k0x * X + k0y * Y))
    o = OracleGPE(p)
    o.set_splitting("rkr", "frozen")
    o.set_psi(np.stack([a * ph, b * ph]))
    n = 50
    o.step_real(n)
    ntot = abs(a) ** 2 + abs(b) ** 2
    sz, sx = np.diag([1.0, -1.0]), np.array([[0.0, 1.0], [1.0, 0.0]])
    HK = 0.5 * (k0x ** 2 + k0y ** 2) * np.eye(2) + k_l * k0x * sz + 0.5 * om * sx
    D = np.diag(np.exp(-0.5j * p.dt * (g * ntot + 0.5 * delta * np.array([1.0, -1.0]))))
    M = D @ sla.expm(-1j * p.dt * HK) @ D
    want = np.linalg.matrix_power(M, n) @ np.array([a, b])
    got = np.array([o.psi[0, 3, 5] / ph[3, 5], o.psi[1, 3, 5] / ph[3, 5]])
    assert np.max(np.abs(got - want)) < 1e-12


@pytest.mark.parametrize("real_space", ["frozen", "nln"])
def test_rkr_linear_ground_state_matches_eigh(real_space):
    p = Params(nx=16, ny=16, xmax=6.0, ymax=6.0, wx=1.0, wy=1.3, k_l=0.9, omega=0.7,
               delta=0.25, omega_r0=0.6, omega_rw=2.0, dt=2e-3)
    w = np.linalg.eigvalsh(_dense_hamiltonian(p))
    o = OracleGPE(p)
    o.set_splitting("rkr", real_space)
    o.set_psi(gaussian_state(p, sigma=1.5, noise=1e-2, seed=7))
    o.step_imag(15000)
    assert abs(o.energy() - w[0]) < 1e-8, (o.energy(), w[0])


def _order(order, real_space, p, psi0, t_end=0.3):
    sols = []
    for dt in (4e-3, 2e-3, 1e-3):
        o = OracleGPE(p.replace(dt=dt))
        o.set_raman_profile(1.4 * np.tanh(grid_axes(p)[0] / 1.5), None)
        o.set_splitting(order, real_space)
        o.set_psi(psi0)
        o.step_real(int(round(t_end / dt)))
        sols.append(o.psi)
    return math.log2(np.linalg.norm(sols[0] - sols[1]) / np.linalg.norm(sols[1] - sols[2]))


@pytest.mark.parametrize("order", ["krk", "rkr"])
def test_second_order_in_dt_with_unequal_couplings_and_spatial_raman(order):
    p = Params(nx=32, ny=32, xmax=5.0, ymax=5.0, g_uu=30.0, g_dd=10.0, g_ud=20.0, k_l=1.0, omega=0.5,
               delta=0.3)
    psi0 = gaussian_state(p, sigma=1.2, noise=0.02, seed=5)
    assert abs(_order(order, "nln", p, psi0) - 2.0) < 0.15


# --- planted mutants ------------------------------------------------------------------------------

_ORIG_APPLY_R = og.OracleGPE.apply_R
_ORIG_STEP = og.OracleGPE.step_once
_ORIG_L = og.OracleGPE.apply_L


def _mut_nln_one_sided(self, psi, h, imag):
    if self.real_space == "nln":
        return self.apply_L(self.apply_N(psi, h, imag), h, imag)
    return _ORIG_APPLY_R(self, psi, h, imag)


def _mut_rkr_asymmetric(self, psi, imag):
    if self.order != "rkr":
        return _ORIG_STEP(self, psi, imag)
    psi = self.apply_R(psi, self.p.dt, imag)
    psi = self.apply_K(psi, self.p.dt, imag)
    if imag:
        psi = psi * np.sqrt(self.p.norm0 / self.norm_of(psi))
    return psi


def _mut_l_without_detuning(self, psi, h, imag):
    return og.apply2x2(og.exp2x2(self.V, 0.5 * self.omega_r, np.zeros_like(self.V), h, imag), psi)


def _pins():
    return [test_nln_real_space_split_is_locally_third_order, test_rkr_plane_wave_matrix_power,
            lambda: test_rkr_linear_ground_state_matches_eigh("nln"),
            lambda: test_second_order_in_dt_with_unequal_couplings_and_spatial_raman("rkr")]


@pytest.mark.parametrize("name,attr,fn", [("N L N one-sided", "apply_R", _mut_nln_one_sided),
                                          ("R-K-R asymmetric", "step_once", _mut_rkr_asymmetric),
                                          ("L without detuning", "apply_L", _mut_l_without_detuning)])
def test_mutant_is_caught(name, attr, fn, monkeypatch):
    monkeypatch.setattr(og.OracleGPE, attr, fn)
    failed = 0
    for pin in _pins():
        try:
            pin()
        except AssertionError:
            failed += 1
    assert failed >= 1, f"mutant '{name}' passes every pin"
