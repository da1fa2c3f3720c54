"""Pins of the oracle's spin-Hall pieces (Sec. 6) against results fixed independently of it.

* the spatial Raman coupling as a sum of profiles along x and y: a dense Hermitian eigensolver
  on an explicitly assembled Hamiltonian (energy at the eigenvector, imaginary-time fixed point)
  and the closed-form spin rotation of a plane wave under a constant coupling;
* the phase-separation parameter: proportional densities, disjoint densities, and displaced
  Gaussians (a Gaussian overlap integral in closed form);
* the population radius: brute force over all candidate radii on a small grid, and the closed
  form of a Gaussian cloud;
* the circulation: vortices z^n of known winding, inside and outside the contour;
* the annealing update: linearity in the amplitude.
Each pin fails for a plausible slip (a transposed profile, a swapped conjugate, a lost factor).
"""
import math

import numpy as np
import pytest

from oracle import OracleGPE, phase_separation, population_radius, winding
from workloads import (Params, complex_noise, gaussian_state, grid_axes, spin_hall_params,
                       spin_hall_profile, vortex_state)


def _dense_hamiltonian(p, om):
    """H = F^-1 diag(H_K) F + diag(H_R) as a dense (2N x 2N) matrix from Eqs. (H1), (H2), (H4),
    with the spatial Raman coupling om (shape (ny, nx)) on the off-diagonal."""
    x, y, _, _ = grid_axes(p)
    nx, ny = p.nx, p.ny
    N = nx * ny
    kx = 2 * np.pi * np.fft.fftfreq(nx, d=x[1] - x[0])
    ky = 2 * np.pi * np.fft.fftfreq(ny, d=y[1] - y[0])
    F = np.kron(np.fft.fft(np.eye(ny), axis=0), np.fft.fft(np.eye(nx), axis=0))
    Finv = np.conj(F).T / N
    KX, KY = np.meshgrid(kx, ky)
    X, Y = np.meshgrid(x, y)
    a = (0.5 * (KX ** 2 + KY ** 2)).ravel()
    bz = (p.k_l * KX).ravel()
    V = (0.5 * (p.wx ** 2 * X ** 2 + p.wy ** 2 * Y ** 2)).ravel()
    H = np.zeros((2 * N, 2 * N), dtype=complex)
    H[:N, :N] = Finv @ np.diag(a + bz) @ F + np.diag(V + 0.5 * p.delta)
    H[N:, N:] = Finv @ np.diag(a - bz) @ F + np.diag(V - 0.5 * p.delta)
    H[:N, N:] = Finv @ np.diag(np.full(N, 0.5 * p.omega)) @ F + np.diag(0.5 * om.ravel())
    H[N:, :N] = H[:N, N:].conj().T
    return H


@pytest.mark.parametrize("nx,ny", [(16, 8), (12, 12)])
def test_xy_profile_linear_ground_state_matches_eigh(nx, ny):
    # distinct profiles along the two axes, on a ragged and on a square grid
    p = Params(nx=nx, ny=ny, xmax=6.0, ymax=5.0, wx=1.0, wy=1.4, k_l=0.8, omega=0.3, delta=0.2, dt=2e-3)
    x, y, _, _ = grid_axes(p)
    ox = 0.7 * np.sin(0.5 * x) + 0.2
    oy = 0.9 * np.cos(0.4 * y) * (y > -1.0)
    H = _dense_hamiltonian(p, ox[None, :] + oy[:, None])
    w, vecs = np.linalg.eigh(H)
    N = p.nx * p.ny
    o = OracleGPE(p)
    o.set_raman_profile(ox, oy)
    v = vecs[:, 0]
    o.set_psi(np.stack([v[:N].reshape(p.ny, p.nx), v[N:].reshape(p.ny, p.nx)]))
    assert abs(o.energy() - w[0]) < 1e-11
    o.set_psi(gaussian_state(p, sigma=1.5, noise=1e-2, seed=3))
    o.step_imag(15000)
    assert abs(o.energy() - w[0]) < 1e-8, (o.energy(), w[0])


def test_constant_profile_rotates_spin_in_closed_form():
    # no trap, no interactions, k_L = 0: H = k^2/2 + (c/2) sigma_x commutes piecewise, so the
    # split step is exact: psi_up = cos(c t / 2) f, psi_dn = -i sin(c t / 2) f, f a plane wave
    # with its kinetic phase.
    p = Params(nx=32, ny=16, xmax=4.0, ymax=4.0, wx=0.0, wy=0.0, dt=0.01)
    c = 1.7
    x, y, _, _ = grid_axes(p)
    o = OracleGPE(p)
    o.set_raman_profile(np.full(p.nx, c / 3.0), np.full(p.ny, 2.0 * c / 3.0))
    k0x, k0y = 3 * math.pi / p.xmax, -2 * math.pi / p.ymax
    X, Y = np.meshgrid(x, y)
    f = np.exp(1j * (k0x * X + k0y * Y))
    o.set_psi(np.stack([f, 0 * f]))
    n = 137
    o.step_real(n)
    t = n * p.dt
    ph = np.exp(-0.5j * (k0x ** 2 + k0y ** 2) * t)
    want = np.stack([math.cos(0.5 * c * t) * f * ph, -1j * math.sin(0.5 * c * t) * f * ph])
    assert np.max(np.abs(o.psi - want)) < 1e-11


def test_profile_orientation_under_transposition():
    # Omega_y(y) on a square grid equals Omega_x(x) on the transposed problem (k_L = 0, isotropic)
    p = Params(nx=32, ny=32, xmax=6.0, ymax=6.0, g_uu=5.0, g_dd=6.0, g_ud=2.0, dt=2e-3)
    x, _, _, _ = grid_axes(p)
    prof = 1.2 * np.tanh(x / 2.0) + 0.3
    psi0 = gaussian_state(p, sigma=1.3, noise=0.05, seed=9)
    a, b = OracleGPE(p), OracleGPE(p)
    a.set_raman_profile(None, prof)
    b.set_raman_profile(prof, None)
    a.set_psi(psi0)
    b.set_psi(np.transpose(psi0, (0, 2, 1)))
    a.step_imag(40)
    b.step_imag(40)
    assert np.max(np.abs(a.psi - np.transpose(b.psi, (0, 2, 1)))) < 1e-12
    assert abs(a.energy() - b.energy()) < 1e-12


def test_add_noise_is_linear_in_the_amplitude():
    p = Params(nx=16, ny=16)
    psi0 = gaussian_state(p, seed=1)
    xi = complex_noise(p, seed=4)
    a, b = OracleGPE(p), OracleGPE(p)
    a.set_psi(psi0)
    b.set_psi(psi0)
    a.add_noise(xi, 0.25)
    a.add_noise(xi, 0.5)
    b.add_noise(xi, 0.75)
    assert np.max(np.abs(a.psi - b.psi)) < 1e-15
    assert np.max(np.abs(b.psi - psi0 - 0.75 * xi)) < 1e-15
    b.add_noise(xi, 0.0)
    assert np.max(np.abs(a.psi - b.psi)) < 1e-15


# --- phase separation ----------------------------------------------------------------------------

def test_phase_separation_closed_forms():
    p = Params(nx=128, ny=128, xmax=10.0, ymax=10.0)
    x, y, _, _ = grid_axes(p)
    X, Y = np.meshgrid(x, y)
    sig = 1.1
    g = np.exp(-(X ** 2 + Y ** 2) / (2 * sig * sig))
    assert abs(phase_separation(np.stack([g, 0.3j * g]))) < 1e-14          # proportional
    left = np.where(X < 0, g, 0.0)
    right = np.where(X >= 0, g, 0.0)
    assert phase_separation(np.stack([left, right])) == 1.0                 # disjoint
    for d in (0.5, 1.0, 2.0):
        a = np.exp(-((X - d / 2) ** 2 + Y ** 2) / (2 * sig * sig))
        b = np.exp(-((X + d / 2) ** 2 + Y ** 2) / (2 * sig * sig))
        # densities exp(-|r -+ d/2|^2 / sig^2): overlap / norm = exp(-d^2 / (2 sig^2))
        want = 1.0 - math.exp(-d * d / (2 * sig * sig))
        assert abs(phase_separation(np.stack([a, b])) - want) < 1e-12


# --- population radius -----------------------------------------------------------------------------

def test_population_radius_brute_force():
    p = Params(nx=16, ny=8, xmax=3.0, ymax=2.0)
    rng = np.random.default_rng(0)
    psi = rng.standard_normal((2, 8, 16)) + 1j * rng.standard_normal((2, 8, 16))
    x, y, _, _ = grid_axes(p)
    dens = np.abs(psi[0]) ** 2 + np.abs(psi[1]) ** 2
    total = dens.sum()
    radii = sorted({math.hypot(xx, yy) for yy in y for xx in x})
    for f in (0.05, 0.3, 0.5, 0.99, 1.0):
        want = None
        for r in radii:
            inside = sum(dens[i, j] for i in range(8) for j in range(16) if x[j] ** 2 + y[i] ** 2 <= r * r + 1e-12)
            if inside >= f * total * (1 - 1e-14):
                want = r
                break
        assert abs(population_radius(psi, p.xmax, p.ymax, f) - want) < 1e-12, f


def test_population_radius_gaussian_cloud():
    # density exp(-r^2 / s^2): fraction within R is 1 - exp(-R^2 / s^2)
    p = Params(nx=512, ny=512, xmax=8.0, ymax=8.0)
    x, y, dx, _ = grid_axes(p)
    X, Y = np.meshgrid(x, y)
    s = 1.5
    g = np.exp(-(X ** 2 + Y ** 2) / (2 * s * s))
    for f in (0.5, 0.9, 0.99):
        want = s * math.sqrt(-math.log(1.0 - f))
        assert abs(population_radius(np.stack([g, g]), p.xmax, p.ymax, f) - want) < 0.5 * dx


# --- circulation ---------------------------------------------------------------------------------

@pytest.mark.parametrize("n", [-3, -1, 0, 1, 2, 5])
def test_winding_of_centred_vortices(n):
    p = Params(nx=128, ny=64, xmax=8.0, ymax=6.0)
    x, y, _, _ = grid_axes(p)
    X, Y = np.meshgrid(x, y)
    z = X + 1j * Y
    env = np.exp(-(X ** 2 + Y ** 2) / 8.0)
    v = (z ** n if n >= 0 else np.conj(z) ** (-n)) * env
    (nu, nd), (ru, rd) = winding(np.stack([v, np.conj(v)]), p.xmax, p.ymax, 3.0)
    assert (nu, nd) == (n, -n)          # counter-clockwise: x + i y winds +1
    assert abs(ru - n) < 1e-9 and abs(rd + n) < 1e-9


def test_winding_counts_only_enclosed_vortices():
    p = Params(nx=128, ny=128, xmax=8.0, ymax=8.0)
    x, y, _, _ = grid_axes(p)
    X, Y = np.meshgrid(x, y)
    z = X + 1j * Y
    inside = [(0.5 + 0.3j, 1), (-1.0 - 0.8j, 1), (0.2 - 1.5j, -1)]
    outside = [(4.5 + 0.5j, 1), (-3.9 - 3.0j, 1)]
    up = np.ones_like(z)
    for z0, s in inside + outside:
        up = up * ((z - z0) if s > 0 else np.conj(z - z0))
    (nu, _), _ = winding(np.stack([up, up]), p.xmax, p.ymax, 3.0)
    assert nu == 1
    (nu, _), _ = winding(np.stack([up, up]), p.xmax, p.ymax, 7.5)
    assert nu == 3


def test_seeded_vortex_state_winds_by_the_seed_count():
    p = spin_hall_params(n=256)
    psi = vortex_state(p, n_vortices=7, seed=3)
    r = population_radius(psi, p.xmax, p.ymax, 0.99)
    (nu, nd), _ = winding(psi, p.xmax, p.ymax, r)
    assert (nu, nd) == (7, -7)
    prof = spin_hall_profile(p)
    assert prof.shape == (p.ny,) and prof.min() == 0.0
    assert abs(prof.max() - 2.0 * p.k_l ** 2) < 1e-12          # sqrt(16) E_L at u = 4


# --- the pins above catch plausible slips (mutants planted in the oracle, on the CPU) -----------

import oracle.gpe as _og            # noqa: E402
import oracle.observables as _ob    # noqa: E402

_ORIG_ANGLE = np.angle


def _mut_profile_transposed(self, omega_x=None, omega_y=None):
    ox = np.zeros(self.nx) if omega_x is None else np.asarray(omega_x, dtype=np.float64)
    oy = np.zeros(self.ny) if omega_y is None else np.asarray(omega_y, dtype=np.float64)
    # x profile varying along rows and y profile along columns (shapes only agree on square grids)
    self.omega_r = ox[:, None] + oy[None, :] if self.nx == self.ny else ox[None, :] + oy[:, None]


def _mut_profile_half(self, omega_x=None, omega_y=None):
    ox = np.zeros(self.nx) if omega_x is None else np.asarray(omega_x, dtype=np.float64)
    oy = np.zeros(self.ny) if omega_y is None else np.asarray(omega_y, dtype=np.float64)
    self.omega_r = 0.5 * (ox[None, :] + oy[:, None])


def _mut_noise_replaces(self, xi, amplitude):
    self.psi = float(amplitude) * np.asarray(xi, dtype=np.complex128)


def _mut_sep_no_sqrt(psi):
    nu, nd = np.abs(psi[0]) ** 2, np.abs(psi[1]) ** 2
    return float(1.0 - np.sum(nu * nd) / (np.sum(nu * nu) * np.sum(nd * nd)))


def _mut_winding_conj_swapped(psi, xmax, ymax, radius):
    psi = np.asarray(psi, dtype=np.complex128)
    i, j = _ob.circle_path(psi.shape[2], psi.shape[1], xmax, ymax, radius)
    raw = [float(np.sum(np.angle(psi[c, i, j] * np.conj(np.roll(psi[c, i, j], -1))))) / (2 * math.pi)
           for c in range(2)]
    return (int(round(raw[0])), int(round(raw[1]))), tuple(raw)


def _mut_winding_unwrapped(psi, xmax, ymax, radius):
    # differences of the phases themselves, not wrapped into (-pi, pi]
    psi = np.asarray(psi, dtype=np.complex128)
    i, j = _ob.circle_path(psi.shape[2], psi.shape[1], xmax, ymax, radius)
    raw = []
    for c in range(2):
        ph = np.angle(psi[c, i, j])
        raw.append(float(np.sum(np.roll(ph, -1) - ph)) / (2 * math.pi))
    return (int(round(raw[0])), int(round(raw[1]))), tuple(raw)


def _mut_radius_not_squared(psi, xmax, ymax, fraction=0.99):
    psi = np.asarray(psi, dtype=np.complex128)
    ny, nx = psi.shape[1:]
    x, y, _, _ = _ob._grid(nx, ny, xmax, ymax)
    X, Y = np.meshgrid(x, y)
    r = np.sqrt(X * X + Y * Y).ravel()
    dens = (np.abs(psi[0]) ** 2 + np.abs(psi[1]) ** 2).ravel()
    order = np.argsort(r, kind="stable")
    cum = np.cumsum(dens[order])
    k = int(np.argmax(cum >= fraction * cum[-1]))
    return float(r[order][k] ** 2)


def _pins():
    return [lambda: test_xy_profile_linear_ground_state_matches_eigh(16, 8),
            lambda: test_xy_profile_linear_ground_state_matches_eigh(12, 12),
            test_constant_profile_rotates_spin_in_closed_form,
            test_profile_orientation_under_transposition, test_add_noise_is_linear_in_the_amplitude,
            test_phase_separation_closed_forms, test_population_radius_brute_force,
            test_population_radius_gaussian_cloud, lambda: test_winding_of_centred_vortices(2),
            test_winding_counts_only_enclosed_vortices]


MUTANTS = {
    "profile transposed": ("OracleGPE.set_raman_profile", _mut_profile_transposed),
    "profile halved": ("OracleGPE.set_raman_profile", _mut_profile_half),
    "noise replaces the state": ("OracleGPE.add_noise", _mut_noise_replaces),
    "phase separation without the square root": ("phase_separation", _mut_sep_no_sqrt),
    "winding with the conjugate on the wrong factor": ("winding", _mut_winding_conj_swapped),
    "phase increments not wrapped": ("winding", _mut_winding_unwrapped),
    "radius compared unsquared": ("population_radius", _mut_radius_not_squared),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, monkeypatch):
    target, fn = MUTANTS[name]
    if target.startswith("OracleGPE."):
        monkeypatch.setattr(_og.OracleGPE, target.split(".")[1], fn)
    else:
        monkeypatch.setitem(globals(), target, fn)
    failed = 0
    for pin in _pins():
        try:
            pin()
        except (AssertionError, ValueError, IndexError):
            failed += 1
    assert failed >= 1, f"mutant '{name}' passes every pin"
