"""Train the learned initial state (paper_2010_15069_amd.surrogate) and measure what it buys.

    python -m paper_2010_15069_amd.train_surrogate [--train 4096] [--heldout 256] [--out PATH]

1. Parameter sets: the sweep ranges (g ~ U[1,100] for all couplings, uniform Raman Omega ~ U[0,3],
   delta ~ U[-0.5,0.5], k_L = 2, isotropic trap, 256^2, imaginary-time dt = 1e-3); training sets
   from seed 1, held-out sets from seed 2.
2. Training targets: each set relaxed by the plain solver from its Thomas-Fermi start (batched,
   all sets in one batch), `--relax` steps.
3. The FNO trained on (parameters -> relaxed state), phase-invariant infidelity loss.
4. Held-out evaluation, both arms stepped in batches with an energy check every 50 steps: steps
   until |E - E_ref| <= 1e-6 |E_ref| from the plain Thomas-Fermi start and from the predicted
   start.  E_ref per set is the lower of the two arms' energies after `--ref-steps` steps.
Prints progress lines and one JSON summary line; writes the weights (safetensors).
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
import torch  # noqa: E402

from paper_2010_15069_amd import Batch, surrogate  # noqa: E402
from workloads import initial_state, sweep_instances  # noqa: E402

WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "fno_256.safetensors")


def log(msg):
    print(msg, flush=True)


def relax(params, starts, steps, chunk=1000):
    """Plain imaginary-time relaxation of all sets in one batch; returns the relaxed states."""
    b = Batch(params)
    for i, s in enumerate(starts):
        b.set_psi(i, s)
    done, t0 = 0, time.perf_counter()
    while done < steps:
        n = min(chunk, steps - done)
        b.step_imag(n).synchronize()
        done += n
        log(f"  relaxed {done}/{steps} steps ({time.perf_counter() - t0:.0f} s)")
    out = [b.get_psi(i).astype(np.complex64) for i in range(len(params))]
    b.close()
    return out


def steps_to_tolerance(params, starts, ref_steps, every=50, tol=1e-6):
    """Energies of all sets every `every` steps up to ref_steps; returns (trace[k][i], final energies)."""
    b = Batch(params)
    for i, s in enumerate(starts):
        b.set_psi(i, s)
    trace = []
    t0 = time.perf_counter()
    for k in range(ref_steps // every):
        b.step_imag(every)
        trace.append(b.energies())
        if (k + 1) % 100 == 0:
            log(f"  {(k + 1) * every}/{ref_steps} steps ({time.perf_counter() - t0:.0f} s)")
    b.close()
    return np.array(trace)


def first_within(trace, e_ref, every, tol=1e-6):
    """Per set: steps at the first check with |E - E_ref| <= tol |E_ref| (None if never)."""
    out = []
    for i in range(trace.shape[1]):
        ok = np.nonzero(np.abs(trace[:, i] - e_ref[i]) <= tol * abs(e_ref[i]))[0]
        out.append(int((ok[0] + 1) * every) if len(ok) else None)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=4096)
    ap.add_argument("--heldout", type=int, default=256)
    ap.add_argument("--relax", type=int, default=40000, help="plain steps for the training targets")
    ap.add_argument("--ref-steps", type=int, default=60000, help="steps of the held-out arms")
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--out", default=WEIGHTS)
    args = ap.parse_args()
    dev = torch.device("cuda")
    t_all = time.perf_counter()

    train_p = sweep_instances(seed=1, sizes=(256,), per_size=args.train)
    held_p = sweep_instances(seed=2, sizes=(256,), per_size=args.heldout)
    log(f"training targets: {len(train_p)} sets, {args.relax} plain steps each")
    starts = [initial_state(p, "tf", seed=i) for i, p in enumerate(train_p)]
    targets = relax(train_p, starts, args.relax)
    del starts

    log("training the FNO")
    torch.manual_seed(0)
    model = surrogate.FNO2d().to(dev)
    x = surrogate.encode(train_p, dev)
    y = surrogate.to_channels(targets, dev)
    del targets
    hist = surrogate.train(model, x, y, epochs=args.epochs, log=log)
    del x, y
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    surrogate.save(model, args.out)
    log(f"weights -> {args.out}")

    log(f"held-out evaluation: {len(held_p)} sets, {args.ref_steps} steps per arm")
    plain = [initial_state(p, "tf", seed=10000 + i) for i, p in enumerate(held_p)]
    model.eval()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    learned = surrogate.predict(model, held_p, dev)
    torch.cuda.synchronize()
    t_inf = (time.perf_counter() - t0) / len(held_p)
    every = 50
    tr_plain = steps_to_tolerance(held_p, plain, args.ref_steps, every)
    tr_learn = steps_to_tolerance(held_p, learned, args.ref_steps, every)
    e_ref = np.minimum(tr_plain[-1], tr_learn[-1])
    sp = first_within(tr_plain, e_ref, every)
    sl = first_within(tr_learn, e_ref, every)
    pairs = [(a, b) for a, b in zip(sp, sl) if a is not None and b is not None]
    res = {
        "train_sets": len(train_p), "heldout_sets": len(held_p), "relax_steps": args.relax,
        "epochs": args.epochs, "final_train_infidelity": hist[-1],
        "plain_reached": sum(s is not None for s in sp), "learned_reached": sum(s is not None for s in sl),
        "plain_steps_median": float(np.median([a for a, _ in pairs])) if pairs else None,
        "learned_steps_median": float(np.median([b for _, b in pairs])) if pairs else None,
        "plain_steps_mean": float(np.mean([a for a, _ in pairs])) if pairs else None,
        "learned_steps_mean": float(np.mean([b for _, b in pairs])) if pairs else None,
        "learned_faster_fraction": float(np.mean([b < a for a, b in pairs])) if pairs else None,
        "inference_s_per_set": t_inf, "total_s": time.perf_counter() - t_all,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
