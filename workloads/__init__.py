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
  (Eq. (H4) with Omega(r)); omega_r0 = 0 disables it.
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
