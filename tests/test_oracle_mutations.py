"""The pins must catch plausible mistakes: each mutant below plants one slip in the oracle (on the
CPU, by patching a copy of its arithmetic) and at least one quick pin check must then fail.

The checks reuse the independent expectations of test_oracle_pins.py (closed forms, expm, eigh)
at small sizes, so the whole file runs in seconds."""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import oracle.gpe as og
from oracle import OracleGPE
from workloads import Params, gaussian_state, grid_axes, thomas_fermi_state

# unpatched originals (the mutants wrap these)
_ORIG_RSH = og.OracleGPE.real_space_hamiltonian
_ORIG_ENERGY = og.OracleGPE.energy_of


def _plane(p, kx0, ky0, a_up, a_dn):
    x, y, _, _ = grid_axes(p)
    X, Y = np.meshgrid(x, y)
    ph = np.exp(1j * (kx0 * X + ky0 * Y))
    return np.stack([a_up * ph, a_dn * ph])


def check_plane_phases():
    p = Params(nx=16, ny=16, xmax=4.0, ymax=3.0, wx=0.0, wy=0.0, g_uu=1.0, g_dd=2.0, g_ud=0.5,
               k_l=1.3, delta=0.7, dt=3e-3)
    kx0, ky0 = 3 * math.pi / p.xmax, -2 * math.pi / p.ymax
    au, ad = 0.8 + 0.1j, 0.3 - 0.5j
    o = OracleGPE(p)
    o.set_psi(_plane(p, kx0, ky0, au, ad))
    o.step_real(20)
    nu, nd = abs(au) ** 2, abs(ad) ** 2
    ksq = 0.5 * (kx0 ** 2 + ky0 ** 2)
    wu = ksq + p.k_l * kx0 + 0.5 * p.delta + p.g_uu * nu + p.g_ud * nd
    wd = ksq - p.k_l * kx0 - 0.5 * p.delta + p.g_dd * nd + p.g_ud * nu
    t = 20 * p.dt
    exp = _plane(p, kx0, ky0, au * np.exp(-1j * wu * t), ad * np.exp(-1j * wd * t))
    return np.max(np.abs(o.psi - exp)) < 1e-12


def check_spinor_matrix_power(imag):
    g = 0.8
    p = Params(nx=16, ny=16, xmax=5.0, ymax=5.0, wx=0.0, wy=0.0, g_uu=g, g_dd=g, g_ud=g,
               k_l=1.1, omega=0.9, delta=0.3, dt=4e-3)
    kx0, ky0 = 2 * math.pi / p.xmax, -1 * math.pi / p.ymax
    v = np.array([0.6 + 0.2j, -0.1 + 0.4j])
    area = 4.0 * p.xmax * p.ymax
    if imag:
        v *= math.sqrt(p.norm0 / (area * np.vdot(v, v).real))
    o = OracleGPE(p)
    o.set_psi(_plane(p, kx0, ky0, v[0], v[1]))
    hk = np.array([[0.5 * (kx0 ** 2 + ky0 ** 2) + p.k_l * kx0, 0.5 * p.omega],
                   [0.5 * p.omega, 0.5 * (kx0 ** 2 + ky0 ** 2) - p.k_l * kx0]], dtype=complex)
    uk = sla.expm((-0.5 * p.dt if imag else -0.5j * p.dt) * hk)
    for _ in range(10):
        v = uk @ v
        rho = np.vdot(v, v).real
        ph = np.array([0.5 * p.delta + g * rho, -0.5 * p.delta + g * rho])
        v = (np.exp(-p.dt * ph) if imag else np.exp(-1j * p.dt * ph)) * v
        v = uk @ v
        if imag:
            v *= math.sqrt(p.norm0 / (area * np.vdot(v, v).real))
    (o.step_imag if imag else o.step_real)(10)
    return np.max(np.abs(o.psi - _plane(p, kx0, ky0, v[0], v[1]))) < 1e-12


def check_energy_closed_form():
    gu, gd, gud, om = 3.0, 5.0, 2.0, 0.8
    p = Params(nx=64, ny=64, g_uu=gu, g_dd=gd, g_ud=gud, omega=om, k_l=1.7, delta=0.6, norm0=2.5)
    x, y, _, _ = grid_axes(p)
    X, Y = np.meshgrid(x, y)
    phi = np.sqrt(p.norm0 / math.pi) * np.exp(-(X ** 2 + Y ** 2) / 2) / math.sqrt(2.0)
    o = OracleGPE(p)
    o.set_psi(np.stack([1.2 * phi, 0.4 * phi]).astype(complex) / math.sqrt(0.8))
    fu, fd = 0.5 * 1.2 ** 2 / 0.8, 0.5 * 0.4 ** 2 / 0.8
    e = (1.0 + p.norm0 * (0.5 * gu * fu * fu + 0.5 * gd * fd * fd + gud * fu * fd) / (2 * math.pi)
         + om * math.sqrt(fu * fd) + 0.5 * p.delta * (fu - fd))
    return abs(o.energy() - e) < 1e-10


def check_linear_eigh():
    from tests.test_oracle_pins import _dense_hamiltonian
    p = Params(nx=8, ny=8, xmax=5.0, ymax=5.0, wx=1.0, wy=1.3, k_l=0.9, omega=0.7,
               delta=0.25, omega_r0=0.6, omega_rw=2.0, dt=5e-3)
    w, vecs = np.linalg.eigh(_dense_hamiltonian(p))
    o = OracleGPE(p)
    N = p.nx * p.ny
    v = vecs[:, 0]
    o.set_psi(np.stack([v[:N].reshape(p.ny, p.nx), v[N:].reshape(p.ny, p.nx)]))
    if abs(o.energy() - w[0]) > 1e-11:
        return False
    o.set_psi(np.stack([v[:N].reshape(p.ny, p.nx), v[N:].reshape(p.ny, p.nx)]) + 0.05)
    o.step_imag(4000)
    return abs(o.energy() - w[0]) < 1e-6


def check_norm_and_order():
    p = Params(nx=32, ny=32, g_uu=10.0, g_dd=10.0, g_ud=10.0, k_l=2.0, omega=1.0, delta=0.2)
    psi0 = thomas_fermi_state(p, seed=4, noise=0.0)
    o = OracleGPE(p.replace(dt=4e-3))
    o.set_psi(psi0)
    n0 = o.norm()
    o.step_real(50)
    if abs(o.norm() - n0) > 1e-12 * n0:
        return False
    outs = []
    for dt in (4e-3, 2e-3, 1e-3):
        q = OracleGPE(p.replace(dt=dt))
        q.set_psi(psi0)
        q.step_real(int(round(0.1 / dt)))
        outs.append(q.get_psi())
    r = np.linalg.norm(outs[0] - outs[1]) / np.linalg.norm(outs[1] - outs[2])
    return abs(math.log2(r) - 2.0) < 0.1


def check_ho_ground_state():
    # no coupling at all: |b| = 0 at every point of both 2x2 exponentials
    p = Params(nx=32, ny=32, wx=1.0, wy=1.5, dt=1e-2)
    o = OracleGPE(p)
    o.set_psi(gaussian_state(p, sigma=1.4, x0=0.3, noise=0.0))
    o.step_imag(1500)
    return abs(o.energy() - 0.5 * (p.wx + p.wy)) < 1e-6


CHECKS = [check_ho_ground_state, check_plane_phases, lambda: check_spinor_matrix_power(False),
          lambda: check_spinor_matrix_power(True), check_energy_closed_form, check_linear_eigh,
          check_norm_and_order]


def test_unmutated_oracle_passes_every_check():
    assert all(c() for c in CHECKS)


# --- mutants -------------------------------------------------------------------------------------

def _mut_kinetic_sign(self):
    self.a_k = -self.a_k


def _mut_soc_sign(self):
    self.bz_k = -self.bz_k


def _mut_soc_factor(self):
    self.bz_k = 0.5 * self.bz_k


def _mut_raman_full_omega(self):
    self.bx_k = 2.0 * self.bx_k


def _mut_trap_factor(self):
    self.V = 2.0 * self.V


def _mut_kx_transposed(self):
    KX, KY = np.meshgrid(self.kx, self.ky)
    self.a_k = 0.5 * (KX ** 2 + KY ** 2)
    self.bz_k = self.p.k_l * KY


def _mut_omega_r_sign(self):
    self.omega_r = -self.omega_r


INIT_MUTANTS = {
    "kinetic sign": _mut_kinetic_sign,
    "spin-momentum sign": _mut_soc_sign,
    "spin-momentum factor": _mut_soc_factor,
    "uniform Raman factor 2": _mut_raman_full_omega,
    "trap factor 2": _mut_trap_factor,
    "k_x and k_y swapped in the spin-momentum term": _mut_kx_transposed,
    "spatial Raman sign": _mut_omega_r_sign,
}


def _rsh_delta_sign(self, psi):
    A, Bx, Bz = _ORIG_RSH(self, psi)
    return A, Bx, Bz - self.p.delta


def _rsh_coupling_swap(self, psi):
    p = self.p
    nu = np.abs(psi[0]) ** 2
    nd = np.abs(psi[1]) ** 2
    d_up = self.V + 0.5 * p.delta + p.g_uu * nd + p.g_ud * nu   # g_uu on the wrong density
    d_dn = self.V - 0.5 * p.delta + p.g_dd * nd + p.g_ud * nu
    return 0.5 * (d_up + d_dn), 0.5 * self.omega_r, 0.5 * (d_up - d_dn)


def _rsh_missing_cross(self, psi):
    p = self.p
    nu = np.abs(psi[0]) ** 2
    nd = np.abs(psi[1]) ** 2
    d_up = self.V + 0.5 * p.delta + p.g_uu * nu
    d_dn = self.V - 0.5 * p.delta + p.g_dd * nd
    return 0.5 * (d_up + d_dn), 0.5 * self.omega_r, 0.5 * (d_up - d_dn)


RSH_MUTANTS = {
    "detuning sign": _rsh_delta_sign,
    "g_uu applied to the down density": _rsh_coupling_swap,
    "inter-species coupling dropped": _rsh_missing_cross,
}


def _exp_real_sign_flip(a, bx, bz, h, imag):
    if imag:
        return _ORIG_EXP(a, bx, bz, h, imag)
    u = _ORIG_EXP(a, bx, bz, h, imag)
    return tuple(np.conj(x) for x in u)


def _exp_transposed(a, bx, bz, h, imag):
    u11, u12, u21, u22 = _ORIG_EXP(a, bx, bz, h, imag)
    return u11, -u12, -u21, u22


def _exp_no_sinc_limit(a, bx, bz, h, imag):
    # sin(h|b|)/|b| evaluated without its |b| -> 0 limit (0/0 where b vanishes)
    a = np.asarray(a, dtype=np.float64)
    bx = np.broadcast_to(np.asarray(bx, dtype=np.float64), a.shape)
    bz = np.broadcast_to(np.asarray(bz, dtype=np.float64), a.shape)
    bm = np.sqrt(bx * bx + bz * bz)
    with np.errstate(invalid="ignore", divide="ignore"):
        if imag:
            pref, c, s = np.exp(-h * a), np.cosh(h * bm), np.sinh(h * bm) / bm
            return (pref * (c - s * bz) + 0j, pref * (-s * bx) + 0j, pref * (-s * bx) + 0j,
                    pref * (c + s * bz) + 0j)
        pref, c, s = np.exp(-1j * h * a), np.cos(h * bm), np.sin(h * bm) / bm
        return pref * (c - 1j * s * bz), pref * (-1j * s * bx), pref * (-1j * s * bx), pref * (c + 1j * s * bz)


_ORIG_EXP = og.exp2x2
EXP_MUTANTS = {
    "real-time exponential sign": _exp_real_sign_flip,
    "off-diagonal sign of the 2x2 exponential": _exp_transposed,
    "missing |b| -> 0 limit": _exp_no_sinc_limit,
}


def _step_half_k_once(self, psi, imag):
    dt = self.p.dt
    psi = self.apply_K(psi, dt, imag)  # K(dt) R(dt) instead of K(dt/2) R(dt) K(dt/2)
    psi = self.apply_R(psi, dt, imag)
    if imag:
        psi = psi * np.sqrt(self.p.norm0 / self.norm_of(psi))
    return psi


def _step_norm_per_component(self, psi, imag):
    dt = self.p.dt
    psi = self.apply_K(psi, 0.5 * dt, imag)
    psi = self.apply_R(psi, dt, imag)
    psi = self.apply_K(psi, 0.5 * dt, imag)
    if imag:
        w = self.dx * self.dy
        for c in range(2):
            psi[c] = psi[c] * np.sqrt(0.5 * self.p.norm0 / (w * np.sum(np.abs(psi[c]) ** 2)))
    return psi


STEP_MUTANTS = {
    "first-order K R splitting": _step_half_k_once,
    "normalisation per component": _step_norm_per_component,
}


def _energy_no_half(self, psi):
    p = self.p
    q = p.replace(g_uu=2 * p.g_uu, g_dd=2 * p.g_dd)
    saved = self.p
    self.p = q
    try:
        return _ORIG_ENERGY(self, psi)
    finally:
        self.p = saved


ENERGY_MUTANTS = {"interaction energy without the 1/2": _energy_no_half}


def _detected():
    return not all(c() for c in CHECKS)


@pytest.mark.parametrize("name", sorted(INIT_MUTANTS))
def test_init_mutant_detected(name, monkeypatch):
    orig = og.OracleGPE.__init__

    def init(self, p, workers=None):
        orig(self, p, workers)
        INIT_MUTANTS[name](self)

    monkeypatch.setattr(og.OracleGPE, "__init__", init)
    assert _detected(), name


@pytest.mark.parametrize("name", sorted(RSH_MUTANTS))
def test_real_space_mutant_detected(name, monkeypatch):
    monkeypatch.setattr(og.OracleGPE, "real_space_hamiltonian", RSH_MUTANTS[name])
    assert _detected(), name


@pytest.mark.parametrize("name", sorted(EXP_MUTANTS))
def test_exponential_mutant_detected(name, monkeypatch):
    monkeypatch.setattr(og, "exp2x2", EXP_MUTANTS[name])
    assert _detected(), name


@pytest.mark.parametrize("name", sorted(STEP_MUTANTS))
def test_step_mutant_detected(name, monkeypatch):
    monkeypatch.setattr(og.OracleGPE, "step_once", STEP_MUTANTS[name])
    assert _detected(), name


@pytest.mark.parametrize("name", sorted(ENERGY_MUTANTS))
def test_energy_mutant_detected(name, monkeypatch):
    monkeypatch.setattr(og.OracleGPE, "energy_of", ENERGY_MUTANTS[name])
    assert _detected(), name
