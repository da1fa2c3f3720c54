"""Seeded synthetic workloads for the two-component quasi-2D GPE: parameters and initial states.

This module is shared by the FP64 oracle and the HIP path.  It holds no part of the split-step
method itself: it only says *what* is simulated (grid, couplings, trap, time step) and builds the
initial order parameter on the host.

Physical model (paper Sec. 3.1, Eqs. (GPEcomponent), (H1)-(H4)), dimensionless harmonic-oscillator
units (Sec. 6): hbar = m = omega_perp = 1.

Parameter meaning (the same fields, in the same order, as the C struct ``sgpe_params``):

* ``nx, ny``        -- grid points along x and y (powers of two).
* ``xmax, ymax``    -- periodic box [-xmax, xmax) x [-ymax, ymax) (Sec. 3.2), dx = 2 xmax / nx.
* ``g_uu, g_dd, g_ud`` -- mean-field couplings g_{up,up}, g_{dn,dn}, g_{up,dn} (Eq. (H3)).
* ``k_l``           -- spin-momentum coefficient k_L of Eq. (H1): the term  +k_L k_x sigma_z.
* ``omega``         -- spatially uniform Raman coupling Omega of Eq. (H4); applied in k-space.
* ``delta``         -- spatially uniform detuning delta of Eq. (H2): the term +delta/2 sigma_z.
* ``wx, wy``        -- harmonic trap V = (wx^2 x^2 + wy^2 y^2) / 2 (Eq. (H2)).
* ``omega_r0, omega_rw`` -- spatially varying Raman coupling Omega(x) = omega_r0 tanh(x / omega_rw)
  (Eq. (H4) with Omega(r)); omega_r0 = 0 disables it.  (Other profiles, such as the Sec. 6 one
  along y, are passed to the solvers as tables; see ``spin_hall_profile``.)
* ``dt``            -- time step (real time), or imaginary-time step d(tau).
* ``norm0``         -- atom number the imaginary-time state is normalised to (Sec. 3.2).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Params", "PRESETS", "preset", "grid_axes",
    "gaussian_state", "thomas_fermi_state", "initial_state", "round_to_c64", "sweep_instances",
    "SPIN_HALL_G", "SPIN_HALL_FIELD", "spin_hall_params", "spin_hall_profile", "vortex_state",
    "complex_noise",
]


@dataclasses.dataclass
class Params:
    nx: int = 64
    ny: int = 64
    xmax: float = 8.0
    ymax: float = 8.0
    g_uu: float = 0.0
    g_dd: float = 0.0
    g_ud: float = 0.0
    k_l: float = 0.0
    omega: float = 0.0
    delta: float = 0.0
    wx: float = 1.0
    wy: float = 1.0
    omega_r0: float = 0.0
    omega_rw: float = 1.0
    dt: float = 1e-3
    norm0: float = 1.0

    def replace(self, **kw) -> "Params":
        return dataclasses.replace(self, **kw)

    def as_dict(self) -> dict:
        return dataclasses.asdict(self)


# Named workloads.  Sizes, couplings and time steps follow the benchmark configurations of this
# project; where a configuration leaves a value open, the choice is written next to it.
PRESETS = {
    # Two-component 64x64 on [-8,8)^2, harmonic trap, g_uu = g_dd = 1, g_ud = 0.9, no Raman
    # coupling, no detuning.  Gaussian (sigma = 1) start plus 1e-3 seeded noise;
    # 200 imaginary-time steps at dt = 1e-3, then 200 real-time steps.
    "tiny": Params(nx=64, ny=64, g_uu=1.0, g_dd=1.0, g_ud=0.9, dt=1e-3),
    # 512x512 real time: g = 10 for all three couplings, Raman Omega = 1 with k_L = 2 in the
    # k-space 2x2 propagator, detuning delta = 0.2.  Thomas-Fermi start, 1000 steps, dt = 5e-4.
    "realtime_512": Params(nx=512, ny=512, g_uu=10.0, g_dd=10.0, g_ud=10.0, k_l=2.0,
                           omega=1.0, delta=0.2, dt=5e-4),
    # The same physics at 1024^2: the split-step throughput workload.
    "metric_1024": Params(nx=1024, ny=1024, g_uu=10.0, g_dd=10.0, g_ud=10.0, k_l=2.0,
                          omega=1.0, delta=0.2, dt=5e-4),
    # Ground-state time-to-solution: the 1024^2 physics at 256^2, imaginary-time step 1e-3.
    "ground_256": Params(nx=256, ny=256, g_uu=10.0, g_dd=10.0, g_ud=10.0, k_l=2.0,
                         omega=1.0, delta=0.2, dt=1e-3),
    # Large ground state: 2048^2 imaginary time, Omega(x) = 2 tanh(x/4) in real space, g = 50,
    # trap aspect ratio 1.5 (wx = 1, wy = 1.5); k_L = 2 and delta = 0 (not fixed by the
    # configuration); dt = 1e-3.
    "ground_2048": Params(nx=2048, ny=2048, g_uu=50.0, g_dd=50.0, g_ud=50.0, k_l=2.0,
                          wy=1.5, omega_r0=2.0, omega_rw=4.0, dt=1e-3),
}


def preset(name: str, **overrides) -> Params:
    return dataclasses.replace(PRESETS[name], **overrides)


def grid_axes(p: Params):
    """Real-space sample points x_j = -xmax + j dx, j = 0..nx-1 (endpoint excluded), same for y."""
    dx = 2.0 * p.xmax / p.nx
    dy = 2.0 * p.ymax / p.ny
    x = -p.xmax + dx * np.arange(p.nx, dtype=np.float64)
    y = -p.ymax + dy * np.arange(p.ny, dtype=np.float64)
    return x, y, dx, dy


def _add_noise_and_normalise(p: Params, psi: np.ndarray, seed: int, noise: float) -> np.ndarray:
    """psi += noise * max|psi| * (xi1 + i xi2), xi ~ N(0,1) drawn for the up component then the
    down component, row-major; then scale so that dx dy sum |psi|^2 = norm0."""
    _, _, dx, dy = grid_axes(p)
    psi = psi.astype(np.complex128, copy=True)
    if noise != 0.0:
        rng = np.random.default_rng(seed)
        amp = noise * float(np.abs(psi).max())
        for c in range(2):
            xi1 = rng.standard_normal((p.ny, p.nx))
            xi2 = rng.standard_normal((p.ny, p.nx))
            psi[c] += amp * (xi1 + 1j * xi2)
    total = dx * dy * float(np.sum(np.abs(psi) ** 2))
    psi *= math.sqrt(p.norm0 / total)
    return psi


def gaussian_state(p: Params, sigma: float = 1.0, seed: int = 0, noise: float = 1e-3,
                   x0: float = 0.0, y0: float = 0.0, weights=(1.0, 1.0)) -> np.ndarray:
    """Gaussian exp(-((x-x0)^2 + (y-y0)^2) / (2 sigma^2)) in each component (times ``weights``),
    plus seeded complex noise, normalised to norm0.  Shape (2, ny, nx), complex128."""
    x, y, _, _ = grid_axes(p)
    X, Y = np.meshgrid(x, y)
    g = np.exp(-((X - x0) ** 2 + (Y - y0) ** 2) / (2.0 * sigma * sigma))
    psi = np.stack([weights[0] * g, weights[1] * g]).astype(np.complex128)
    return _add_noise_and_normalise(p, psi, seed, noise)


def thomas_fermi_state(p: Params, seed: int = 0, noise: float = 1e-3) -> np.ndarray:
    """Thomas-Fermi profile n_s = max(mu - V, 0) / (g_ss + g_ud) per component, with
    mu = sqrt(norm0 wx wy (g_uu + g_ud) / (2 pi)) (from the integral of (mu - V)_+ over the
    plane being pi mu^2 / (wx wy)); plus seeded noise; normalised to norm0."""
    gu = p.g_uu + p.g_ud
    gd = p.g_dd + p.g_ud
    if gu <= 0.0 or gd <= 0.0:
        return gaussian_state(p, seed=seed, noise=noise)
    x, y, _, _ = grid_axes(p)
    X, Y = np.meshgrid(x, y)
    V = 0.5 * (p.wx ** 2 * X ** 2 + p.wy ** 2 * Y ** 2)
    mu = math.sqrt(p.norm0 * p.wx * p.wy * gu / (2.0 * math.pi))
    n = np.maximum(mu - V, 0.0)
    psi = np.stack([np.sqrt(n / gu), np.sqrt(n / gd)]).astype(np.complex128)
    return _add_noise_and_normalise(p, psi, seed, noise)


def round_to_c64(psi: np.ndarray) -> np.ndarray:
    """Round once to complex64 and widen back: both the oracle and the GPU start from these values."""
    return psi.astype(np.complex64).astype(np.complex128)


def initial_state(p: Params, kind: str = "tf", seed: int = 0, noise: float = 1e-3) -> np.ndarray:
    if kind == "tf":
        psi = thomas_fermi_state(p, seed=seed, noise=noise)
    elif kind == "gauss":
        psi = gaussian_state(p, seed=seed, noise=noise)
    else:
        raise ValueError(f"unknown initial state kind {kind!r}")
    return round_to_c64(psi)


def sweep_instances(seed: int = 0, sizes=(128, 256, 512), per_size: int = 32) -> list:
    """A batched parameter sweep: per_size instances of each grid size (n x n on [-8, 8)^2,
    isotropic trap), in that order.  Per instance, drawn from default_rng(seed) in the order
    (g, Omega, delta): one interaction strength g ~ U[1, 100] for all three couplings, a uniform
    Raman coupling Omega ~ U[0, 3] (k-space), a detuning delta ~ U[-0.5, 0.5]; k_L = 2 and
    imaginary-time step 1e-3 for all."""
    rng = np.random.default_rng(seed)
    out = []
    for n in sizes:
        for _ in range(per_size):
            g = float(rng.uniform(1.0, 100.0))
            om = float(rng.uniform(0.0, 3.0))
            de = float(rng.uniform(-0.5, 0.5))
            out.append(Params(nx=n, ny=n, g_uu=g, g_dd=g, g_ud=g, k_l=2.0, omega=om, delta=de, dt=1e-3))
    return out


# --- Spin-Hall ground states (Sec. 6) ---------------------------------------------------------
# Readings of what Sec. 6 leaves open:
# * g: 10^4 atoms of 87Rb (a_s = 100 Bohr radii; the species is not named) in a trap with
#   omega_z / omega_perp = 2000 / 50, so a_z = a_0 / sqrt(40) and g = sqrt(8 pi) N a_s / a_z
#   = 1.10e3 in units of hbar omega_perp a_0^2 with the state normalised to one.
# * The Raman profile of Eq. (Omega) is applied along y through the coordinate
#   u = clamp(2 + y / ell, 0, 4): the double-well minima move from +-k_L at u = 0 to 0 at u = 4,
#   the gauge potential A*(u) = k_L (1 - u / 4) is linear there, and ell = k_L / (4 |B*|) gives
#   the printed field |B*| = 0.369 hbar / (q a_0^2).  k_L = 3 (ell = 2.03): the linear strip
#   |y| <= 2 ell spans three quarters of the cloud's diameter, while the dressed-state potential
#   -Omega^2 / (16 E_L) that a varying Omega brings with it (depth E_L = 4.5 over the strip) moves
#   the cloud by about 0.6 a_0.  A wider strip needs a larger k_L and a deeper potential, which
#   pulls the cloud out of the field (k_L = 5); y in units of a_0 (k_L = 1.476) leaves a 4 a_0
#   strip with hardly any vortices.
# * Box [-16, 16)^2 (dx = 1/32 at 1024^2, several points per healing length); uniform Omega = 0,
#   delta = 0, isotropic trap; imaginary-time step 1e-3.
SPIN_HALL_G = 1.10e3
SPIN_HALL_FIELD = 0.369


def spin_hall_params(n: int = 1024, ratio: float = 0.1, g: float = SPIN_HALL_G, k_l: float = 3.0,
                     xmax: float = 16.0, dt: float = 1e-3) -> Params:
    """The spin-Hall system of Sec. 6: g_uu = g_dd = g, g_ud = ratio * g, spin-momentum k_L, no
    uniform Raman coupling (the coupling is the spatial profile of ``spin_hall_profile``)."""
    return Params(nx=n, ny=n, xmax=xmax, ymax=xmax, g_uu=g, g_dd=g, g_ud=ratio * g, k_l=k_l,
                  omega=0.0, delta=0.0, wx=1.0, wy=1.0, omega_r0=0.0, omega_rw=1.0, dt=dt, norm0=1.0)


def spin_hall_profile(p: Params, field: float = SPIN_HALL_FIELD) -> np.ndarray:
    """Omega(y_i), length ny: Eq. (Omega), hbar Omega / E_L = sqrt(8 u - u^2) with E_L = k_L^2 / 2,
    u = clamp(2 + y / ell, 0, 4), ell = k_L / (4 field)."""
    _, y, _, _ = grid_axes(p)
    ell = p.k_l / (4.0 * field)
    u = np.clip(2.0 + y / ell, 0.0, 4.0)
    e_l = 0.5 * p.k_l * p.k_l
    return e_l * np.sqrt(np.maximum(8.0 * u - u * u, 0.0))


def vortex_state(p: Params, n_vortices: int = 50, seed: int = 0, spread: float = 0.8,
                 core: float | None = None) -> np.ndarray:
    """Thomas-Fermi amplitudes (no noise) with n_vortices singly quantised vortices imprinted in
    each component (Sec. 6): positions uniform in the disc of radius spread * R_TF about the
    centre, drawn from default_rng(seed) for the up component (radius, then angle, per vortex) and
    then the down one; winding +1 in the up component and -1 in the down one; each vortex
    multiplies by (z - z_k) / sqrt(|z - z_k|^2 + core^2), z = x +- i y (default core: the healing
    length 1 / sqrt(2 mu)).  Normalised to norm0, rounded to complex64."""
    base = thomas_fermi_state(p, seed=0, noise=0.0)
    gu = p.g_uu + p.g_ud
    mu = math.sqrt(p.norm0 * p.wx * p.wy * gu / (2.0 * math.pi))
    r_tf = math.sqrt(2.0 * mu) / max(p.wx, p.wy)
    if core is None:
        core = 1.0 / math.sqrt(2.0 * mu)
    x, y, dx, dy = grid_axes(p)
    X, Y = np.meshgrid(x, y)
    rng = np.random.default_rng(seed)
    psi = base.copy()
    for c, sign in ((0, 1.0), (1, -1.0)):
        for _ in range(n_vortices):
            r = spread * r_tf * math.sqrt(float(rng.uniform()))
            a = 2.0 * math.pi * float(rng.uniform())
            zx, zy = X - r * math.cos(a), Y - r * math.sin(a)
            psi[c] *= (zx + 1j * sign * zy) / np.sqrt(zx * zx + zy * zy + core * core)
    total = dx * dy * float(np.sum(np.abs(psi) ** 2))
    psi *= math.sqrt(p.norm0 / total)
    return round_to_c64(psi)


def complex_noise(p: Params, seed: int) -> np.ndarray:
    """Complex Gaussian field of shape (2, ny, nx): real and imaginary parts ~ N(0, 1), drawn from
    default_rng(seed) as one (2, ny, nx, 2) array."""
    a = np.random.default_rng(seed).standard_normal((2, p.ny, p.nx, 2))
    return a[..., 0] + 1j * a[..., 1]
