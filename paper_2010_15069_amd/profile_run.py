"""A fixed run of the split-step solver for profilers: `steps` steps of a named workload at a given
precision after a warm-up, timed with HIP events, one JSON line out.

    python -m paper_2010_15069_amd.profile_run [--workload metric_1024] [--precision c64|c128]
                                               [--steps 200] [--warmup 20] [--real]

Under rocprofv3 it gives a kernel trace or counter pass of exactly these kernels, with no other
work in the process.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="metric_1024")
    ap.add_argument("--precision", default="c64", choices=["c64", "c128"])
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--real", action="store_true", help="real-time steps (default: imaginary time, dt = 1e-3)")
    args = ap.parse_args()

    import torch

    from paper_2010_15069_amd import Solver
    from workloads import initial_state, preset

    p = preset(args.workload)
    if not args.real:
        p = p.replace(dt=1e-3)
    stream = torch.cuda.current_stream()
    s = Solver(p, stream=stream.cuda_stream, precision=args.precision).set_psi(initial_state(p, "tf", seed=0))
    step = s.step_real if args.real else s.step_imag
    step(args.warmup)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    print(json.dumps({"workload": args.workload, "precision": args.precision, "real": args.real,
                      "steps": args.steps, "ms": ms, "steps_per_s": args.steps / (ms * 1e-3),
                      "energy": s.energy()}), flush=True)


if __name__ == "__main__":
    main()
