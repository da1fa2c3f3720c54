"""Writes ground_energy.json: the FP64 oracle's converged imaginary-time energy for the
ground-state time-to-solution workload (workloads preset "ground_256", Thomas-Fermi start, seed 0).

Calls only the oracle.  Stops when the energy changes by less than 1e-13 relative over 1000 steps;
with the observed geometric convergence the remaining error is then below ~3e-13.

    python tests/golden/make_ground_energy.py [workers]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import OracleGPE  # noqa: E402
from workloads import initial_state, preset  # noqa: E402


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else os.cpu_count()
    name = "ground_256"
    p = preset(name)
    o = OracleGPE(p, workers=workers)
    o.set_psi(initial_state(p, "tf", seed=0))
    t0 = time.time()
    e_prev, steps, trace = o.energy(), 0, []
    while True:
        o.step_imag(1000)
        steps += 1000
        e = o.energy()
        rel = abs(e - e_prev) / abs(e)
        trace.append([steps, e])
        print(f"{steps:7d} steps  E = {e:.15f}  |dE|/E over 1000 steps = {rel:.2e}  "
              f"({time.time() - t0:.0f} s)", flush=True)
        e_prev = e
        if rel < 1e-13 or steps >= 400000:
            break
    out = {
        "workload": name,
        "params": p.as_dict(),
        "initial_state": "thomas_fermi_state(seed=0, noise=1e-3) rounded once to complex64",
        "energy": e,
        "steps": steps,
        "converged_rel_change_per_1000_steps": rel,
        "trace_every_1000_steps": trace[-20:],
        "note": "FP64 oracle (oracle/gpe.py) imaginary-time relaxation; written by "
                "tests/golden/make_ground_energy.py",
    }
    with open(os.path.join(ROOT, "tests", "golden", "ground_energy.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
