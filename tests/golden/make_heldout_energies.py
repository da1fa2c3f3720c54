"""Writes heldout_energies.json: the FP64 oracle's converged imaginary-time energies for the held-out
parameter sets of the learned-start workload (``workloads.sweep_instances(seed=2, sizes=(256,),
per_size=8)``: 256^2, g ~ U[1, 100] for all couplings, uniform Omega ~ U[0, 3], delta ~ U[-0.5, 0.5],
k_L = 2, dt = 1e-3), each from its Thomas-Fermi start (seed 10000 + index).

Calls only the oracle.  Each set runs until its energy changes by less than 1e-11 relative over
1000 steps (at most 300 000 steps).  The energy approaches the fixed point geometrically; from the
last two changes d1, d2 over 1000 steps the remaining distance is about d2 r / (1 - r), r = d2 / d1,
and that estimate is stored next to each energy.

    python tests/golden/make_heldout_energies.py [index ...]   # all sets if none given; one process each
"""
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
OUT = os.path.join(ROOT, "tests", "golden", "heldout_energies.json")
N_SETS = 8


def converge(index):
    from oracle import OracleGPE
    from workloads import initial_state, sweep_instances
    p = sweep_instances(seed=2, sizes=(256,), per_size=N_SETS)[index]
    o = OracleGPE(p, workers=1)
    o.set_psi(initial_state(p, "tf", seed=10000 + index))
    t0 = time.time()
    e_prev, d_prev, steps = o.energy(), None, 0
    while True:
        o.step_imag(1000)
        steps += 1000
        e = o.energy()
        d = abs(e - e_prev)
        rel = d / abs(e)
        if steps % 10000 == 0:
            print(f"set {index}: {steps} steps, E = {e:.15f}, |dE|/E per 1000 steps {rel:.2e} "
                  f"({time.time() - t0:.0f} s)", flush=True)
        if rel < 1e-11 or steps >= 300000:
            break
        e_prev, d_prev = e, d
    r = d / d_prev if d_prev else 0.0
    tail = d * r / (1.0 - r) if 0.0 < r < 1.0 else float("nan")
    return {"index": index, "params": p.as_dict(), "energy": e, "steps": steps,
            "rel_change_per_1000_steps": rel, "ratio_of_changes": r,
            "estimated_remaining_rel": tail / abs(e)}


def main():
    args = sys.argv[1:]
    if args and args[0] == "--one":
        print("RESULT " + json.dumps(converge(int(args[1]))), flush=True)
        return
    idx = [int(a) for a in args] or list(range(N_SETS))
    procs = [subprocess.Popen([sys.executable, __file__, "--one", str(i)], stdout=subprocess.PIPE, text=True)
             for i in idx]
    results = []
    for pr in procs:
        for line in pr.stdout:
            if line.startswith("RESULT "):
                results.append(json.loads(line[7:]))
            else:
                print(line, end="", flush=True)
        pr.wait()
    results.sort(key=lambda r: r["index"])
    out = {
        "workload": "learned-start held-out sets: sweep_instances(seed=2, sizes=(256,), per_size=8)",
        "initial_state": "thomas_fermi_state(seed=10000 + index, noise=1e-3) rounded once to complex64",
        "sets": results,
        "note": "FP64 oracle (oracle/gpe.py) imaginary-time relaxation; written by "
                "tests/golden/make_heldout_energies.py",
    }
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
