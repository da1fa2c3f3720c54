"""FP64 CPU oracle of the time-splitting spectral (TSSP) propagation of the two-component GPE.

TEST INFRASTRUCTURE ONLY.  This module exists so that tests, the smoke check and the CPU
baseline leg of the benchmark can check the HIP path against a plain, slow, obviously correct
implementation.  The product path never imports, links or calls it.

What is computed (Smith, Cooke & LeBlanc, "GPU-accelerated solutions of the nonlinear
Schroedinger equation for simulating 2D spinor BECs"):

* Model -- Sec. 3.1, Eq. (GPEcomponent) with the four Hamiltonian pieces Eqs. (H1)-(H4):
  kinetic plus spin-momentum term, trap plus detuning, mean-field interaction, Raman coupling.
* Grids -- Sec. 3.2: nx x ny points on the periodic box [-xmax, xmax) x [-ymax, ymax); the
  momentum grid spans +-pi/dx with spacing pi/xmax.
* Propagators -- Sec. 3.2, Eq. (TEOp): each piece is applied through the exponential of its
  Hamiltonian times the time step; real time, or imaginary time (dt -> -i dtau).
* Splitting -- Sec. 3.2: Strang splitting of the k-space and real-space pieces; one step is
  K(dt/2) R(dt) K(dt/2), where K is the k-space 2x2 propagator reached through a 2D FFT and R the
  real-space 2x2 exponential of trap, detuning, mean-field and spatial Raman terms.  Variants
  (``set_splitting``): the other Strang ordering R(dt/2) K(dt) R(dt/2); and R itself split to
  second order (Sec. 3.2 asks for it because the real-space pieces need not commute) as
  N(h/2) L(h) N(h/2), N the mean-field phase with the densities of its input, L the exponential
  of the linear real-space terms.
* Normalisation -- Sec. 3.2: in imaginary time the order parameter is rescaled to the atom number
  after every step.

Readings where the paper is silent or inconsistent (each one is exercised by a pinned test):

1. Sign of time evolution: i d/dt psi = H psi, U = exp(-i H dt) in real time and exp(-H dtau) in
   imaginary time.  (Eq. (GPEcomponent)/(TEOp) print the opposite real-time sign; the imaginary-time
   operator is the same either way.)
2. Kinetic term: +|k|^2/2 (Eq. (H1) prints -k^2/2, which cannot give a ground state).
3. Spin-momentum term: +k_L k_x sigma_z, so the up component's minimum sits at k_x = -k_L and the
   down component's at +k_L (the text of Sec. 3.1 and Sec. 6).
4. A spatially uniform Raman coupling Omega is part of the k-space 2x2 propagator; a spatially
   varying Omega(x, y) and the detuning delta are part of the real-space exponential.
5. The real-space exponential freezes the densities at the start of the sub-step and
   exponentiates the full 2x2 real-space Hamiltonian in closed form.
6. Normalisation is of the total (both components) to norm0, after each full imaginary step.
7. Energy per particle: the standard Gross-Pitaevskii functional (not printed in the paper),
   with one half on the interaction terms, of the state rescaled to norm0 -- the quadratic terms
   divided by the norm N, the quartic (interaction) terms by N^2 / norm0.  For a state of norm
   norm0 this is the plain functional over norm0; for others it does not depend on the norm, so a
   small norm error of a complex64 state does not enter the energy at first order.

Everything here is complex128 / float64 and uses NumPy/SciPy only.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

__all__ = ["OracleGPE", "exp2x2", "apply2x2"]


def exp2x2(a, bx, bz, h, imag):
    """Closed-form exponential of the Hermitian 2x2 matrix H = a*1 + bx*sigma_x + bz*sigma_z.

    Real time returns exp(-i h H); imaginary time returns exp(-h H).  a, bx, bz are real arrays of
    one shape; the result is the four entries (u11, u12, u21, u22) of that shape.  With
    |b| = sqrt(bx^2 + bz^2) and b.sigma = [[bz, bx], [bx, -bz]]:

      exp(-i h H) = e^{-i h a} [cos(h|b|) 1 - i sin(h|b|)/|b| b.sigma]
      exp(-h H)   = e^{-h a}   [cosh(h|b|) 1 - sinh(h|b|)/|b| b.sigma]

    with sin(h|b|)/|b| -> h and sinh(h|b|)/|b| -> h as |b| -> 0.
    """
    a = np.asarray(a, dtype=np.float64)
    bx = np.broadcast_to(np.asarray(bx, dtype=np.float64), a.shape)
    bz = np.broadcast_to(np.asarray(bz, dtype=np.float64), a.shape)
    bm = np.sqrt(bx * bx + bz * bz)
    safe = np.where(bm > 0.0, bm, 1.0)
    if imag:
        pref = np.exp(-h * a)
        c = np.cosh(h * bm)
        s = np.where(bm > 0.0, np.sinh(h * bm) / safe, h)
        u11 = pref * (c - s * bz)
        u22 = pref * (c + s * bz)
        u12 = pref * (-s * bx)
        return (u11.astype(np.complex128), u12.astype(np.complex128),
                u12.astype(np.complex128), u22.astype(np.complex128))
    pref = np.exp(-1j * h * a)
    c = np.cos(h * bm)
    s = np.where(bm > 0.0, np.sin(h * bm) / safe, h)
    u11 = pref * (c - 1j * s * bz)
    u22 = pref * (c + 1j * s * bz)
    u12 = pref * (-1j * s * bx)
    return u11, u12, u12.copy(), u22


def apply2x2(u, psi):
    """psi' = U psi for a field of 2x2 matrices U (entries broadcast over the grid)."""
    u11, u12, u21, u22 = u
    return np.stack([u11 * psi[0] + u12 * psi[1], u21 * psi[0] + u22 * psi[1]])


class OracleGPE:
    """Literal TSSP integrator.  State: complex128 array of shape (2, ny, nx), component 0 = up.

    ``p`` is any object with the fields of ``workloads.Params``.
    """

    def __init__(self, p, workers: int | None = None):
        self.p = p
        self.workers = workers
        nx, ny = int(p.nx), int(p.ny)
        self.nx, self.ny = nx, ny
        # Sec. 3.2: real grid on (-xmax, xmax) with spacing dx; momentum spacing pi/xmax.
        self.dx = 2.0 * p.xmax / nx
        self.dy = 2.0 * p.ymax / ny
        self.x = -p.xmax + self.dx * np.arange(nx)
        self.y = -p.ymax + self.dy * np.arange(ny)
        self.kx = 2.0 * np.pi * np.fft.fftfreq(nx, d=self.dx)
        self.ky = 2.0 * np.pi * np.fft.fftfreq(ny, d=self.dy)
        X, Y = np.meshgrid(self.x, self.y)
        KX, KY = np.meshgrid(self.kx, self.ky)
        # Eq. (H2): trap.
        self.V = 0.5 * (p.wx ** 2 * X ** 2 + p.wy ** 2 * Y ** 2)
        # Eq. (H4) with a spatially varying coupling Omega(x).
        if p.omega_r0 != 0.0:
            self.omega_r = p.omega_r0 * np.tanh(X / p.omega_rw)
        else:
            self.omega_r = np.zeros_like(X)
        # Eq. (H1) (+ uniform Eq. (H4)): H_K(k) = a 1 + bx sigma_x + bz sigma_z.
        self.a_k = 0.5 * (KX ** 2 + KY ** 2)
        self.bz_k = p.k_l * KX
        self.bx_k = np.full_like(KX, 0.5 * p.omega)
        self.psi = np.zeros((2, ny, nx), dtype=np.complex128)
        self._uk_cache = {}
        self.order = "krk"          # or "rkr"
        self.real_space = "frozen"  # or "nln"

    def set_splitting(self, order="krk", real_space="frozen"):
        """Strang ordering of a step ("krk": K(dt/2) R(dt) K(dt/2); "rkr": R(dt/2) K(dt) R(dt/2)) and
        the form of R ("frozen": one closed-form exponential of H_R with the densities of its input;
        "nln": N(h/2) L(h) N(h/2))."""
        if order not in ("krk", "rkr") or real_space not in ("frozen", "nln"):
            raise ValueError("unknown splitting")
        self.order, self.real_space = order, real_space

    # -- state ------------------------------------------------------------------------------
    def set_psi(self, psi):
        psi = np.asarray(psi)
        if psi.shape != (2, self.ny, self.nx):
            raise ValueError(f"psi must have shape (2, {self.ny}, {self.nx}), got {psi.shape}")
        if not np.all(np.isfinite(psi)):
            raise ValueError("psi contains non-finite values")
        self.psi = psi.astype(np.complex128, copy=True)

    def get_psi(self):
        return self.psi.copy()

    def set_raman_profile(self, omega_x=None, omega_y=None):
        """Spatially varying Raman coupling of Eq. (H4) as a sum of profiles along the two axes,
        Omega(x, y) = Omega_x(x_j) + Omega_y(y_i) (Sec. 6 imposes one along y, Eq. (Omega)).  None
        stands for a zero profile.  Replaces the tanh profile of the parameters."""
        ox = np.zeros(self.nx) if omega_x is None else np.asarray(omega_x, dtype=np.float64)
        oy = np.zeros(self.ny) if omega_y is None else np.asarray(omega_y, dtype=np.float64)
        if ox.shape != (self.nx,) or oy.shape != (self.ny,):
            raise ValueError("profile lengths must be nx and ny")
        self.omega_r = ox[np.newaxis, :] + oy[:, np.newaxis]

    def add_noise(self, xi, amplitude):
        """Annealing update of Sec. 6: the state plus `amplitude` times the given noise field
        (drawn by the caller), with no renormalisation."""
        xi = np.asarray(xi, dtype=np.complex128)
        if xi.shape != self.psi.shape:
            raise ValueError("noise must have the state's shape")
        self.psi = self.psi + float(amplitude) * xi

    # -- sub-steps --------------------------------------------------------------------------
    def _fft2(self, f):
        return sfft.fft2(f, axes=(-2, -1), workers=self.workers)

    def _ifft2(self, f):
        return sfft.ifft2(f, axes=(-2, -1), workers=self.workers)

    def kinetic_propagator(self, h, imag):
        key = (float(h), bool(imag))
        if key not in self._uk_cache:
            self._uk_cache[key] = exp2x2(self.a_k, self.bx_k, self.bz_k, h, imag)
        return self._uk_cache[key]

    def apply_K(self, psi, h, imag):
        """K(h): FFT to momentum space, where Eq. (H1) is diagonal in k (Sec. 3.2), apply the
        2x2 exponential of H_K(k) at every k, transform back."""
        psik = self._fft2(psi)
        psik = apply2x2(self.kinetic_propagator(h, imag), psik)
        return self._ifft2(psik)

    def real_space_hamiltonian(self, psi):
        """Entries (A, Bx, Bz) of H_R = A 1 + Bx sigma_x + Bz sigma_z at every point: Eqs. (H2),
        (H3), (H4) with the densities of ``psi``."""
        p = self.p
        nu = np.abs(psi[0]) ** 2
        nd = np.abs(psi[1]) ** 2
        d_up = self.V + 0.5 * p.delta + p.g_uu * nu + p.g_ud * nd
        d_dn = self.V - 0.5 * p.delta + p.g_dd * nd + p.g_ud * nu
        return 0.5 * (d_up + d_dn), 0.5 * self.omega_r, 0.5 * (d_up - d_dn)

    def apply_R(self, psi, h, imag):
        """R(h): densities frozen at entry, then the closed-form 2x2 exponential per point; or,
        with the "nln" split, N(h/2) L(h) N(h/2)."""
        if self.real_space == "nln":
            psi = self.apply_N(psi, 0.5 * h, imag)
            psi = self.apply_L(psi, h, imag)
            return self.apply_N(psi, 0.5 * h, imag)
        A, Bx, Bz = self.real_space_hamiltonian(psi)
        return apply2x2(exp2x2(A, Bx, Bz, h, imag), psi)

    def apply_N(self, psi, h, imag):
        """Mean-field part of Eq. (H3) alone: a diagonal phase (or decay) per component with the
        densities of the input."""
        p = self.p
        nu = np.abs(psi[0]) ** 2
        nd = np.abs(psi[1]) ** 2
        d_up = p.g_uu * nu + p.g_ud * nd
        d_dn = p.g_dd * nd + p.g_ud * nu
        f = (lambda d: np.exp(-h * d)) if imag else (lambda d: np.exp(-1j * h * d))
        return np.stack([f(d_up) * psi[0], f(d_dn) * psi[1]])

    def apply_L(self, psi, h, imag):
        """Linear real-space part: trap and detuning (Eq. (H2)) and spatial Raman coupling (Eq. (H4))
        as one closed-form 2x2 exponential per point."""
        return apply2x2(exp2x2(self.V, 0.5 * self.omega_r, np.full_like(self.V, 0.5 * self.p.delta), h, imag),
                        psi)

    def step_once(self, psi, imag):
        dt = self.p.dt
        if self.order == "rkr":
            psi = self.apply_R(psi, 0.5 * dt, imag)
            psi = self.apply_K(psi, dt, imag)
            psi = self.apply_R(psi, 0.5 * dt, imag)
        else:
            psi = self.apply_K(psi, 0.5 * dt, imag)
            psi = self.apply_R(psi, dt, imag)
            psi = self.apply_K(psi, 0.5 * dt, imag)
        if imag:
            psi = psi * np.sqrt(self.p.norm0 / self.norm_of(psi))
        return psi

    # -- public steps -----------------------------------------------------------------------
    def step_real(self, n):
        for _ in range(int(n)):
            self.psi = self.step_once(self.psi, imag=False)

    def step_imag(self, n):
        for _ in range(int(n)):
            self.psi = self.step_once(self.psi, imag=True)

    # -- observables ------------------------------------------------------------------------
    def norm_of(self, psi):
        """N[psi] = dx dy sum over both components and all points of |psi|^2."""
        return float(self.dx * self.dy * np.sum(np.abs(psi) ** 2))

    def norm(self):
        return self.norm_of(self.psi)

    def energy_of(self, psi):
        """Energy per particle of the Gross-Pitaevskii functional at the state rescaled to norm0:

        E = (1/N) { (dx dy / N_pts) sum_k psik^dag H_K(k) psik
                    + dx dy sum_r [ V (n_u + n_d) + delta/2 (n_u - n_d) + Omega(r) Re(psi_u^* psi_d) ] }
          + (norm0/N^2) dx dy sum_r [ g_uu n_u^2 / 2 + g_dd n_d^2 / 2 + g_ud n_u n_d ]
        with psik the unnormalised 2D DFT of each component and N the norm of psi.
        """
        p = self.p
        w = self.dx * self.dy
        npts = self.nx * self.ny
        pk = self._fft2(psi)
        pu2 = np.abs(pk[0]) ** 2
        pd2 = np.abs(pk[1]) ** 2
        cross_k = np.real(np.conj(pk[0]) * pk[1])
        e_k = np.sum(self.a_k * (pu2 + pd2) + self.bz_k * (pu2 - pd2) + 2.0 * self.bx_k * cross_k)
        nu = np.abs(psi[0]) ** 2
        nd = np.abs(psi[1]) ** 2
        cross_r = np.real(np.conj(psi[0]) * psi[1])
        e_lin = np.sum(self.V * (nu + nd) + 0.5 * p.delta * (nu - nd) + self.omega_r * cross_r)
        e_int = np.sum(0.5 * p.g_uu * nu * nu + 0.5 * p.g_dd * nd * nd + p.g_ud * nu * nd)
        nrm = self.norm_of(psi)
        return (w / npts * float(e_k) + w * float(e_lin)) / nrm + w * float(e_int) * p.norm0 / (nrm * nrm)

    def energy(self):
        return self.energy_of(self.psi)
