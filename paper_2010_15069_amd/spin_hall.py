"""Spin-Hall ground states of a two-component BEC (Sec. 6), on the split-step solver.

One trial (Sec. 6):
  1. the spin-Hall system (``workloads.spin_hall_params``): g_uu = g_dd = g, g_ud = ratio * g,
     spin-momentum k_L, and the Raman coupling profile Omega(y) of Eq. (Omega) in the real-space
     exponential (``sgpe_set_raman_profile``);
  2. a Thomas-Fermi start with 50 seeded vortices per component of opposite winding;
  3. segment one: imaginary-time steps with a Gaussian-noise anneal every ``anneal_every`` steps
     (``sgpe_add_noise``), the amplitude falling linearly from ``anneal_amp`` times the initial
     peak amplitude to zero over the segment (reading: the schedule is not printed);
  4. segment two: imaginary-time steps without noise;
  5. observables of the relaxed state: energy per particle, the phase-separation parameter s and
     the winding numbers of both components along the circle that holds 99 % of the atoms.
The noise fields are drawn on the host from a seeded generator and passed in.

    python -m paper_2010_15069_amd.spin_hall [--n 1024] [--ratios 0,0.1,...] [--trials 1]
prints one JSON line per trial.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from paper_2010_15069_amd.solver import Solver  # noqa: E402
from workloads import complex_noise, spin_hall_params, spin_hall_profile, vortex_state  # noqa: E402

SEGMENTS = (60000, 60000)


def anneal_schedule(segment: int, anneal_every: int, amp0: float):
    """[(steps before the anneal, amplitude)] for segment one: an anneal after every
    `anneal_every` steps, the amplitude amp0 (1 - k / K) for the k-th of K anneals (k = 1..K;
    the last one, zero, is skipped), then the remaining steps with no anneal (amplitude 0)."""
    k_total = segment // anneal_every
    out = [(anneal_every, amp0 * (1.0 - k / k_total)) for k in range(1, k_total + 1)]
    rest = segment - k_total * anneal_every
    if rest:
        out.append((rest, 0.0))
    return out


def real_space_split(p) -> str:
    """The real-space split that keeps the step second order (Sec. 3.2 asks for a second-order
    split of the real-space pieces).  With a spatial Raman coupling the densities change within the
    real-space sub-step, and one exponential with the densities frozen at its start is the exact
    sub-flow only if the mean field is a multiple of the total density (g_uu = g_dd = g_ud), which
    the coupling conserves.  Otherwise the split N(h/2) L(h) N(h/2) is needed."""
    return "frozen" if p.g_uu == p.g_dd == p.g_ud else "nln"


def run_trial(ratio: float = 0.1, seed: int = 0, n: int = 1024, segments=SEGMENTS, anneal_every: int = 2000,
              anneal_amp: float = 0.05, n_vortices: int = 50, log=None, return_psi: bool = False,
              real_space: str = "auto", **system) -> dict:
    """One trial; `system` overrides fields of ``workloads.spin_hall_params`` (g, k_l, xmax, dt).
    real_space: "frozen", "nln", or "auto" (``real_space_split``)."""
    p = spin_hall_params(n=n, ratio=ratio, **system)
    if real_space == "auto":
        real_space = real_space_split(p)
    psi0 = vortex_state(p, n_vortices=n_vortices, seed=seed)
    amp0 = anneal_amp * float(np.abs(psi0).max())
    t0 = time.perf_counter()
    with Solver(p) as s:
        s.set_splitting("krk", real_space)
        s.set_raman_profile(omega_y=spin_hall_profile(p))
        s.set_psi(psi0)
        done = 0
        for k, (steps, amp) in enumerate(anneal_schedule(segments[0], anneal_every, amp0)):
            s.step_imag(steps)
            done += steps
            if amp > 0.0:
                s.add_noise(complex_noise(p, seed=[seed, k]), amp)
            if log and (k + 1) % 10 == 0:
                log(f"  ratio {ratio}: {done} annealed steps ({time.perf_counter() - t0:.1f} s)")
        s.step_imag(segments[1])
        e = s.energy()
        t_steps = time.perf_counter() - t0
        sep = s.phase_separation()
        r99 = s.population_radius(0.99)
        n_up, n_dn, raw_up, raw_dn = s.winding(r99)
        psi = s.get_psi() if return_psi else None
    out = {"ratio": ratio, "seed": seed, "n": n, "steps": int(sum(segments)), "real_space": real_space, "energy": e,
            "phase_separation": sep, "radius_99": r99, "winding_up": n_up, "winding_down": n_dn,
            "winding_raw": [raw_up, raw_dn], "seconds": t_steps}
    if return_psi:
        out["psi"] = psi
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--ratios", default="0,0.1,0.2,0.3,0.4,0.5,0.6,0.7,0.8,0.9,1.0")
    ap.add_argument("--trials", type=int, default=1)
    ap.add_argument("--segment", type=int, default=SEGMENTS[0])
    args = ap.parse_args()
    for r in [float(v) for v in args.ratios.split(",")]:
        for t in range(args.trials):
            res = run_trial(ratio=r, seed=t, n=args.n, segments=(args.segment, args.segment),
                            log=lambda m: print(m, flush=True))
            print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
