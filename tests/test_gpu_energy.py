"""The energy and norm kernels against the FP64 oracle's definitions (Eqs. (H1)-(H4), the state
rescaled to norm0), at every line length the library accepts along each axis, in both precisions,
with and without a spatial Raman coupling, one context at a time and batched.  Both sides evaluate
the same rounded state in fp64, so they agree to far below the solver's parity bars: the bound here
is 1e-11 (relative), a transform or term error of any instantiation shows at 1e-6 or more."""
import os

import numpy as np
import pytest

from oracle import OracleGPE
from workloads import Params, gaussian_state, round_to_c64

pytestmark = pytest.mark.gpu

WORKERS = max(1, min(16, len(os.sched_getaffinity(0))))
# every power of two from 16 to 4096 as a row length and as a column length, 65 536 points each
SHAPES = [(1 << k, 1 << (16 - k)) for k in range(4, 13)]


@pytest.fixture(scope="module")
def sgpe():
    import paper_2010_15069_amd as m
    if m.device_count() <= 0:
        pytest.skip("no HIP device")
    return m


def _params(nx, ny, spatial):
    return Params(nx=nx, ny=ny, xmax=7.0, ymax=9.0, g_uu=5.0, g_dd=2.0, g_ud=3.0, k_l=1.1, omega=0.8,
                  delta=-0.3, wx=1.2, wy=0.9, omega_r0=1.5 if spatial else 0.0, omega_rw=3.0)


def _state(p, seed):
    rng = np.random.default_rng(seed)
    shape = (2, p.ny, p.nx)
    return gaussian_state(p, sigma=2.0, noise=0.0) * (1.0 + 0.2 * (rng.standard_normal(shape)
                                                                   + 1j * rng.standard_normal(shape)))


@pytest.mark.parametrize("precision", ["c64", "c128"])
@pytest.mark.parametrize("spatial", [False, True])
def test_every_line_length(sgpe, precision, spatial):
    for i, (nx, ny) in enumerate(SHAPES):
        p = _params(nx, ny, spatial)
        psi = _state(p, i)
        if precision == "c64":
            psi = round_to_c64(psi)
        print(f"case: {nx}x{ny} {precision} spatial={spatial}", flush=True)
        o = OracleGPE(p, workers=WORKERS)
        o.set_psi(psi)
        s = sgpe.Solver(p, precision=precision).set_psi(psi)
        e, eo = s.energy(), o.energy()
        assert abs(e - eo) <= 1e-11 * abs(eo), (nx, ny, e, eo)
        assert abs(s.norm() - o.norm()) <= 1e-12 * o.norm(), (nx, ny)
        s.close()


def test_batched_energies_every_line_length(sgpe):
    ps = [_params(nx, ny, False) for nx, ny in SHAPES]
    states = [round_to_c64(_state(p, 100 + i)) for i, p in enumerate(ps)]
    b = sgpe.Batch(ps)
    for i, psi in enumerate(states):
        b.set_psi(i, psi)
    e = b.energies()
    for i, (p, psi) in enumerate(zip(ps, states)):
        o = OracleGPE(p, workers=WORKERS)
        o.set_psi(psi)
        eo = o.energy()
        assert abs(e[i] - eo) <= 1e-11 * abs(eo), (p.nx, p.ny, e[i], eo)
    b.close()
