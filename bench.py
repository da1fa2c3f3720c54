"""Split-step throughput of the two-component GPE solver on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Workload: 1024 x 1024 grid, two components, complex64 state resident in HBM; g_uu = g_dd = g_ud
= 10, k_L = 2, uniform Raman Omega = 1, detuning 0.2, harmonic trap, Thomas-Fermi start (seed 0).
A step is one imaginary-time Strang step K(dt/2) R(dt) K(dt/2) with renormalisation (every stage of
the hot path), dt = 1e-3; real-time steps (dt = 5e-4) are reported beside it.  K steps are timed
in batches of 100 (one step_imag(100) call each) with HIP events; value = K / total time.

Prints one JSON line.  Also reports: the dominant kernel's HBM roofline fraction (algorithmic bytes
over its mean launch time in the real schedule, from HIP events on the solver's stream);
the same physics at 512^2 and 2048^2; the ground-state time-to-solution (wall time until the
energy is within 1e-6 of the FP64 oracle's converged value, 256^2), from the Thomas-Fermi start
and from the learned (neural-operator) start; the learned start against the plain one on held-out
parameter sets; the batched parameter sweep (96 instances of three sizes, one graph-captured call);
one spin-Hall trial (Sec. 6, 2 x 60000 steps at 1024^2); and the FP64 oracle's throughput on a
bounded sample of the 1024^2 workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E peak
BYTES_PER_POINT_PASS = 32      # one pass reads and writes both complex64 components
BYTES_PER_POINT_STEP = 64      # two passes per step
IMAG_DT = 1e-3                 # imaginary-time step of the throughput workload

# The paper's own timings for this path (Sec. 5, Fig. 2 and Fig. 3; hardware of Table 1; Sec. 6),
# quoted as context: complex128 PyTorch/cuFFT on 2015-2018 NVIDIA GPUs, not a target.
PAPER_CONTEXT = {
    "precision": "complex128 (PyTorch tensors, cuFFT)",
    "step_time_fit": "GPU step time ~ theta N + offset with theta = 9.7(1)e-8 s per grid point "
                     "(Fig. 2); about 0.10 s per step at N = 1024^2",
    "cpu_exponent": "CPU step time ~ N^kappa, kappa = 1.03(3) (Fig. 2)",
    "max_speedup_gpu_vs_cpu": [6.3, 36, 85],
    "break_even": "GPU and CPU step times equal near N = 2^12 grid points",
    "spin_hall_trial": "about 45 minutes per trial (1024^2 x 2, 2 x 60000 imaginary-time steps) on the "
                       "Titan V, about a day estimated on the i9-9900K (Sec. 6)",
    "hardware": {"GeForce MX150": "384 cores, 2 GB, 48.06 GB/s",
                 "GeForce GTX 980 Ti": "2816 cores, 6 GB, 336.6 GB/s",
                 "Titan V": "5120 cores, 12 GB, 651.3 GB/s",
                 "CPUs": "i5-7200U, FX-6300, i9-9900K"},
}


_T0 = time.perf_counter()


def progress(msg):
    """One line per finished leg on stderr (the JSON line stays alone on stdout)."""
    print(f"bench: {msg} ({time.perf_counter() - _T0:.0f} s)", file=sys.stderr, flush=True)


def median_mad(xs):
    import numpy as np
    a = np.asarray(xs, dtype=float)
    med = float(np.median(a))
    return med, float(np.median(np.abs(a - med)))


def _traffic_record(kernel_name, workload, schedule):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken on the
    current step kernels (matched by the kernel-source hash) with the same launch schedule; else
    None."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
        from paper_2010_15069_amd.build import kernel_hash
        if (rec.get("kernel_hash") != kernel_hash() or rec.get("workload") != workload
                or rec.get("schedule") != schedule):
            return None
        return rec.get("kernels", {}).get(kernel_name)
    except Exception:
        return None


def _oracle_rate(p, psi0, seconds, workers):
    from oracle import OracleGPE
    o = OracleGPE(p, workers=workers)
    o.set_psi(psi0)
    o.step_imag(1)  # warm-up (plans, caches)
    n, t0 = 0, time.perf_counter()
    while True:
        o.step_imag(1)
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            return n, el


def cpu_baseline(p, psi0, seconds, single_seconds):
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    n, el = _oracle_rate(p, psi0, seconds, cores)
    n1, el1 = _oracle_rate(p, psi0, single_seconds, 1)
    return {"value": n / el, "unit": "split-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} imaginary-time steps of the 1024^2 x 2 workload in complex128 "
                      f"({el:.1f} s, scipy.fft workers={cores})",
            "single_thread": {"value": n1 / el1, "unit": "split-steps/s", "cores": 1,
                              "sample": f"{n1} steps ({el1:.1f} s, workers=1)"}}


def other_grids(torch, stream, timed, p, steps=500, warmup=50):
    """The same physics at 512^2 and 2048^2: imaginary-time split-steps/s (dt = 1e-3) and the
    HBM roofline fraction on B_alg."""
    from paper_2010_15069_amd import Solver
    from workloads import initial_state
    res = {}
    for n in (512, 2048):
        q = p.replace(nx=n, ny=n, dt=IMAG_DT)
        s = Solver(q, stream=stream.cuda_stream)
        s.set_psi(initial_state(q, "tf", seed=0))
        s.step_imag(warmup)
        total_ms, per = timed(s.step_imag, steps, 100)
        v = steps / (total_ms * 1e-3)
        res[f"{n}x{n}"] = {"split_steps_per_s": v, "step_ms_median": median_mad(per)[0],
                           "hbm_roofline_frac": BYTES_PER_POINT_STEP * n * n * v / (HBM_PEAK_GBS * 1e9)}
        s.close()
    return res


def batched_sweep(torch, stream, steps=500, tune_steps=5):
    """The batched parameter sweep: 96 instances (32 each of 128^2, 256^2, 512^2; g, Omega,
    delta drawn from seed 0), 500 imaginary-time steps of all of them in one call.  The per-class
    schedules come from the library's autotuner; the first call captures the graph, the timed
    call replays it.  Reported: instance-steps/s, and the roofline fraction on B_alg summed over
    the instances; the same call with direct launches beside it."""
    from paper_2010_15069_amd import Batch
    from workloads import initial_state, sweep_instances
    ps = sweep_instances(seed=0)
    b = Batch(ps, stream=stream.cuda_stream)
    for i, p in enumerate(ps):
        b.set_psi(i, initial_state(p, "tf", seed=i))
    t0 = time.perf_counter()
    tuned_ms = b.autotune(tune_steps)
    tune_s = time.perf_counter() - t0
    schedules = {f"{nx}x{ny}": b.get_schedule(k) for k, (nx, ny, _) in enumerate(b.classes())}

    def timed_call():
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        b.step_imag(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3

    t_capture = timed_call()             # captures and runs the graph
    t_graph = timed_call()               # replays it
    b.use_graph(False)
    t_direct = timed_call()
    pts = sum(p.nx * p.ny for p in ps)
    e = [b.energy(i) for i in (0, 32, 64)]
    # persistent mode: one cooperative launch for every steady-state step of every instance
    for i, p in enumerate(ps):
        b.set_psi(i, initial_state(p, "tf", seed=i))
    b.use_graph(True)
    b.use_persistent(True)
    tp_first = timed_call()
    tp = timed_call()
    b.use_graph(False)
    tp_direct = timed_call()
    e_p = [b.energy(i) for i in (0, 32, 64)]
    b.close()
    best = min(t_graph, tp, tp_direct)
    return {"workload": "96 instances: 32 x 128^2, 32 x 256^2, 32 x 512^2, g ~ U[1,100], Omega ~ U[0,3], "
                        "delta ~ U[-0.5,0.5] (seed 0), k_L = 2, imaginary time dt = 1e-3, Thomas-Fermi starts",
            "steps": steps, "seconds_graph": t_graph, "seconds_direct": t_direct,
            "seconds_first_call_with_capture": t_capture,
            "instance_steps_per_s": len(ps) * steps / best,
            "hbm_roofline_frac": BYTES_PER_POINT_STEP * pts * steps / best / (HBM_PEAK_GBS * 1e9),
            "per_class_launches": {"instance_steps_per_s": len(ps) * steps / t_graph, "seconds_graph": t_graph,
                                   "seconds_direct": t_direct, "autotune_seconds": tune_s, "schedules": schedules,
                                   "tuned_ms_per_step_per_class": tuned_ms, "energies_sample": e},
            "persistent": {"instance_steps_per_s": len(ps) * steps / min(tp, tp_direct),
                           "seconds_graph_replay": tp, "seconds_direct": tp_direct,
                           "seconds_first_call": tp_first, "energies_sample": e_p,
                           "note": "one cooperative launch for steps 1..n-1 of all 96 instances; the call's "
                                   "first and last passes per class"}}


def ground_state_time(torch, stream, check_every=50, max_steps=200000):
    """Wall time from set_psi (Thomas-Fermi start) until the energy is within 1e-6 (relative) of
    the FP64 oracle's converged imaginary-time energy for the same workload and time step
    (tests/golden/ground_energy.json): one sgpe_relax_imag call with that target, the energy
    checked every `check_every` steps (the checks run behind the steps, and are timed)."""
    from paper_2010_15069_amd import Solver
    from workloads import initial_state, preset
    ref = json.load(open(os.path.join(ROOT, "tests", "golden", "ground_energy.json")))
    name = ref["workload"]
    p = preset(name)
    psi0 = initial_state(p, "tf", seed=0)
    e_ref = float(ref["energy"])
    s = Solver(p, stream=stream.cuda_stream)
    s.set_psi(psi0)                      # warm-up of the code paths, then the timed run
    s.relax_imag(check_every=check_every, max_steps=2 * check_every, rule="delta", tol=0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.set_psi(psi0)
    r = s.relax_imag(check_every=check_every, max_steps=max_steps, target=e_ref, tol=1e-6)
    el = time.perf_counter() - t0
    s.close()
    return {"workload": f"{name}: {p.nx}x{p.ny} x 2 components, g=10 (all), k_L=2, Omega=1, "
                        f"delta=0.2, harmonic trap, imaginary-time dt={p.dt}, Thomas-Fermi start",
            "time_to_1e-6_s": el, "steps": r["steps"], "steps_taken": r["steps_taken"],
            "energy": r["energy"], "energy_ref": e_ref, "rel_error": abs(r["energy"] - e_ref) / abs(e_ref),
            "check_every": check_every, "reached": r["met"],
            "driver": "sgpe_relax_imag: energy checks queued behind the steps (the state ends at most two "
                      "chunks past the stopping check; those steps are timed too)"}


def _load_surrogate(torch):
    """The learned-start model (weights shipped with the package), warmed up once."""
    from paper_2010_15069_amd import surrogate
    from paper_2010_15069_amd.train_surrogate import WEIGHTS
    from workloads import sweep_instances
    if not os.path.exists(WEIGHTS):
        return None
    model = surrogate.load(WEIGHTS, "cuda")
    # warm-up at the batch sizes used below (library plans and kernel choices are per shape)
    for count in (1, 64):
        qs = sweep_instances(seed=3, sizes=(256,), per_size=count)
        surrogate.predict(model, qs, "cuda")
        surrogate.predict_device(model, qs, "cuda")
    torch.cuda.synchronize()
    return model


def ground_2048_convergence(torch, stream, every=10, tol=1e-9, max_steps=150000):
    """The large ground state at full size: 2048^2, Omega(x) = 2 tanh(x/4) in the real-space
    exponential, g = 50, trap aspect 1.5, Thomas-Fermi start; imaginary-time steps until the first
    check (every `every` steps) with |E_n - E_{n-every}| < tol |E_n|, in one sgpe_relax_imag call.
    Also reported: the step at which the energy first came within 1e-6 of the final one (read off
    the same checks), with its wall time pro rata."""
    from paper_2010_15069_amd import Solver
    from workloads import initial_state, preset
    p = preset("ground_2048")
    psi0 = initial_state(p, "tf", seed=0)
    s = Solver(p, stream=stream.cuda_stream)
    s.set_psi(psi0)
    s.relax_imag(check_every=every, max_steps=2 * every, rule="delta", tol=0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.set_psi(psi0)
    r = s.relax_imag(check_every=every, max_steps=max_steps, rule="delta", tol=tol, record_energies=True)
    el = time.perf_counter() - t0
    s.close()
    es = r["energies"]
    trace = [(k * every, None, float(e)) for k, e in enumerate(es)]
    e_fin = float(es[-1])
    hit = next((st for st, _, e in trace if abs(e - e_fin) <= 1e-6 * abs(e_fin)), None)
    print(f"ground_2048: {r['steps']} steps, E = {e_fin!r} ({el:.1f} s)", file=sys.stderr, flush=True)
    return {"workload": "ground_2048: 2048x2048 x 2, Omega(x) = 2 tanh(x/4) (real space), g = 50 (all), "
                        "k_L = 2, wx = 1, wy = 1.5, imaginary-time dt = 1e-3, Thomas-Fermi start",
            "stop_rule": f"|E_n - E_(n-{every})| < {tol:g} |E_n|, checked every {every} steps (checks timed)",
            "converged": r["met"], "steps": r["steps"], "steps_taken": r["steps_taken"], "seconds": el,
            "energy": e_fin, "steps_to_1e-6_of_final": hit,
            "seconds_to_1e-6_of_final_pro_rata": None if hit is None else el * hit / max(1, r["steps_taken"]),
            "fixed_point_estimate": _aitken_estimate(trace)}


def _aitken_estimate(trace, spacing=5000):
    """Distance of the last energy from the imaginary-time fixed point, estimated from the energy
    trace alone: with E_n - E_inf ~ A r^n (one slowest mode), Aitken's delta-squared over three checks
    `spacing` steps apart gives E_inf.  Reported for the last triple, with the first step whose
    estimated distance was below 1e-6 |E| (None if none)."""
    by_step = {st: e for st, _, e in trace}
    marks = [st for st in sorted(by_step) if st % spacing == 0]
    first, last = None, None
    for i in range(2, len(marks)):
        e0, e1, e2 = by_step[marks[i - 2]], by_step[marks[i - 1]], by_step[marks[i]]
        d1, d2 = e1 - e0, e2 - e1
        if d2 == d1 or d1 == 0.0:
            continue
        e_inf = e2 - d2 * d2 / (d2 - d1)
        dist = abs(e2 - e_inf) / abs(e_inf)
        last = {"steps": marks[i], "energy_inf": e_inf, "distance_rel": dist, "ratio_per_spacing": d2 / d1}
        if first is None and dist < 1e-6:
            first = marks[i]
    return {"method": f"Aitken delta^2 over energies {spacing} steps apart", "last": last,
            "steps_to_estimated_1e-6": first}


def ground_state_learned(torch, stream, model, check_every=50, max_steps=200000):
    """The ground-state time-to-solution of the same workload from the learned start: the timed
    region holds the input encoding, the network's forward pass, the state handed to the solver on
    the device (sgpe_set_psi_device) and the checked steps (one sgpe_relax_imag call, check 0 being
    the predicted state itself)."""
    from paper_2010_15069_amd import Solver, surrogate
    from workloads import initial_state, preset
    ref = json.load(open(os.path.join(ROOT, "tests", "golden", "ground_energy.json")))
    p = preset(ref["workload"])
    e_ref = float(ref["energy"])
    s = Solver(p, stream=stream.cuda_stream)
    s.set_psi(initial_state(p, "tf", seed=0))      # warm-up of the code paths, then the timed run
    s.relax_imag(check_every=check_every, max_steps=2 * check_every, rule="delta", tol=0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    psi0 = surrogate.predict_device(model, [p], "cuda")[0]     # stays on the device
    t_inf = time.perf_counter() - t0
    s.set_psi_device(psi0)
    r = s.relax_imag(check_every=check_every, max_steps=max_steps, target=e_ref, tol=1e-6)
    el = time.perf_counter() - t0
    s.close()
    return {"time_to_1e-6_s": el, "inference_s": t_inf, "steps": r["steps"], "steps_taken": r["steps_taken"],
            "energy": r["energy"], "rel_error": abs(r["energy"] - e_ref) / abs(e_ref), "reached": r["met"]}


def learned_start_sweep(torch, stream, model, n_sets=64, steps=60000, check_every=50):
    """Held-out parameter sets (seed 2 of the sweep distribution at 256^2), each relaxed from the
    plain Thomas-Fermi start and from the learned start, all sets of one arm in one batch, the
    energy of every set checked every 50 steps (sgpe_batch_energies: one launch per kernel for the
    whole batch).  E_ref per set: the lower of the two arms' final energies.
    Reported per arm: steps and batch wall time until each set is within 1e-6 (medians)."""
    import numpy as np
    from paper_2010_15069_amd import Batch, surrogate
    from workloads import initial_state, sweep_instances
    ps = sweep_instances(seed=2, sizes=(256,), per_size=n_sets)

    def arm(starts_fn, on_device=False):
        b = Batch(ps, stream=stream.cuda_stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i, psi in enumerate(starts_fn()):
            if on_device:
                b.set_psi_device(i, psi)
            else:
                b.set_psi(i, psi)
        trace, clock = [], []
        for _ in range(steps // check_every):
            b.step_imag(check_every)
            trace.append(b.energies())
            clock.append(time.perf_counter() - t0)
        b.close()
        return np.array(trace), np.array(clock)

    tr_p, ck_p = arm(lambda: [initial_state(p, "tf", seed=10000 + i) for i, p in enumerate(ps)])
    tr_l, ck_l = arm(lambda: surrogate.predict_device(model, ps, "cuda"), on_device=True)
    e_ref = np.minimum(tr_p[-1], tr_l[-1])

    def first(trace, clock):
        st, sec = [], []
        for i in range(len(ps)):
            ok = np.nonzero(np.abs(trace[:, i] - e_ref[i]) <= 1e-6 * abs(e_ref[i]))[0]
            if len(ok):
                st.append((ok[0] + 1) * check_every)
                sec.append(float(clock[ok[0]]))
        return st, sec

    sp, tp = first(tr_p, ck_p)
    sl, tl = first(tr_l, ck_l)
    med = lambda v: float(np.median(v)) if v else None  # noqa: E731
    # the first held-out sets against the FP64 oracle's converged energies
    oracle_check = None
    gpath = os.path.join(ROOT, "tests", "golden", "heldout_energies.json")
    if os.path.exists(gpath):
        gold = json.load(open(gpath))["sets"]
        k = min(len(gold), len(ps))
        eo = np.array([g["energy"] for g in gold[:k]])
        oracle_check = {"sets": k,
                        "max_rel_error_plain_final": float(np.max(np.abs(tr_p[-1, :k] - eo) / np.abs(eo))),
                        "max_rel_error_learned_final": float(np.max(np.abs(tr_l[-1, :k] - eo) / np.abs(eo))),
                        "max_rel_error_e_ref": float(np.max(np.abs(e_ref[:k] - eo) / np.abs(eo)))}
    return {"workload": f"{n_sets} held-out sets (seed 2): 256^2, g ~ U[1,100] (all couplings), Omega ~ U[0,3], "
                        f"delta ~ U[-0.5,0.5], k_L = 2, dt = 1e-3; one batch per arm; energy every {check_every} steps",
            "max_steps": steps,
            "e_ref": "per set, the lower of the two arms' final energies (the plain solver judges)",
            "plain": {"reached": len(sp), "steps_median": med(sp), "batch_seconds_median": med(tp)},
            "learned": {"reached": len(sl), "steps_median": med(sl), "batch_seconds_median": med(tl)},
            "oracle_check": oracle_check}


def splitting_variants(torch, stream, timed, p, p_imag, psi0, steps=600, warmup=30):
    """Throughput of the splitting variants on the headline workload (1024^2): K-R-K with the
    N L N real-space split, R-K-R, R-K-R with N L N; imaginary and real time."""
    from paper_2010_15069_amd import Solver
    out = {}
    for order, rs in (("krk", "nln"), ("rkr", "frozen"), ("rkr", "nln")):
        res = {}
        for kind, pp in (("imag", p_imag), ("real", p)):
            s = Solver(pp, stream=stream.cuda_stream).set_splitting(order, rs).set_psi(psi0)
            step = s.step_imag if kind == "imag" else s.step_real
            step(warmup)
            total_ms, _ = timed(step, steps, 100)
            res[kind] = steps / (total_ms * 1e-3)
            s.close()
        out[f"{order}+{rs}"] = {"split_steps_per_s_imag": res["imag"], "split_steps_per_s_real": res["real"]}
    return out


def complex128_rates(torch, stream, timed, p, p_imag, psi0, steps=300, warmup=20):
    """Throughput of the complex128 instantiation on the headline workload (1024^2)."""
    from paper_2010_15069_amd import Solver
    res = {}
    for kind, pp in (("imag", p_imag), ("real", p)):
        s = Solver(pp, stream=stream.cuda_stream, precision="c128").set_psi(psi0)
        step = s.step_imag if kind == "imag" else s.step_real
        step(warmup)
        total_ms, _ = timed(step, steps, 100)
        res[f"split_steps_per_s_{kind}"] = steps / (total_ms * 1e-3)
        s.close()
    res["hbm_roofline_frac_imag"] = 128 * p.nx * p.ny * res["split_steps_per_s_imag"] / (HBM_PEAK_GBS * 1e9)
    res["note"] = "complex128 state: 32 B per point per sweep, 128 B per point per step"
    return res


def spin_hall_trial(torch):
    """One spin-Hall trial (Sec. 6) at 1024^2: vortex-seeded start, 60000 annealed and 60000
    plain imaginary-time steps with the Raman profile Omega(y), then the observables."""
    from paper_2010_15069_amd.spin_hall import run_trial
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = run_trial(ratio=0.1, seed=0, n=1024)
    res["wall_seconds"] = time.perf_counter() - t0
    res["steps_per_s"] = res["steps"] / res["seconds"]
    res["workload"] = ("spin-Hall trial: 1024^2 x 2, g = 1100, g_ud / g = 0.1, k_L = 3, Omega(y) of Eq. (Omega), "
                       "50 seeded vortices per component, 2 x 60000 imaginary-time steps (dt = 1e-3), "
                       "30 noise anneals in the first segment")
    return res


def roofline_references(torch, n, steady_step_ms, dominant_gbps):
    """Measured references for the roofline on this device: a plain device copy of 256 MiB (torch
    copy_, the best of five), and the arithmetic-free copy with a step's data movement at n x n
    (sgpe_probe_exchange: the row partition, then the column partition, plain stores, 4-column
    tiles; mean of 50 rounds)."""
    from paper_2010_15069_amd import probe_exchange
    a = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream()
    best = None
    for _ in range(6):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        b.copy_(a)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    copy_gbps = 2 * a.numel() * 4 / (best * 1e-3) / 1e9
    del a, b
    _, _, round_ms = probe_exchange(n, n, 1, 1, 4, write_through=False, wave_local=False, reps=50)
    return {"plain_copy_GBps": copy_gbps,
            "dominant_pass_frac_of_plain_copy": dominant_gbps / copy_gbps,
            "exchange_copy_step_us": 1e3 * round_ms,
            "exchange_copy_frac_of_peak": BYTES_PER_POINT_STEP * n * n / (round_ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
            "steady_step_over_exchange_copy": steady_step_ms / round_ms,
            "method": "plain copy: torch copy_ of 256 MiB, best of 6 (read + written bytes); exchange copy: "
                      "sgpe_probe_exchange at the headline size, 64 B per point per round"}


def exchange_floor():
    """The arithmetic-free copy with the two passes' data movement, per layout and tile: mean
    microseconds per launch of each partition (events between launches), per row + column round
    back to back, and the bandwidth of a round on the algorithmic bytes (32 B per point per launch).
    Tiles as the step kernels' lanes hold them (a lane pair per point), and wave-local (a wave per
    row or column, both components per lane)."""
    from paper_2010_15069_amd import probe_exchange
    out = []
    for n in (256, 512, 1024, 2048):
        configs = []
        for L, rt, ct in [(1, 1, 2), (1, 1, 4), (1, 1, 8), (2, 2, 2), (2, 2, 4), (4, 4, 1), (4, 4, 2),
                          (8, 8, 1)]:
            if 2 * rt * (n // 16) > 1024 or 2 * ct * (n // 16) > 1024:
                continue
            configs.append((L, rt, ct, False))
        if n >= 512:   # a wave per line needs 512..2048 points
            for L, rt, ct in [(1, 1, 1), (1, 2, 4), (1, 4, 4), (4, 1, 1), (4, 4, 4), (8, 1, 1), (8, 2, 2), (8, 4, 4)]:
                configs.append((L, rt, ct, True))
        for L, rt, ct, wl in configs:
            for wt in (True, False):
                r, c, pr = probe_exchange(n, n, L, rt, ct, wt, wl, reps=40)
                rec = {"n": n, "layout_rows": L, "row_tile": rt, "col_tile": ct, "wave_local": wl,
                       "write_through": wt, "row_us": round(1e3 * r, 3), "col_us": round(1e3 * c, 3),
                       "round_us": round(1e3 * pr, 3), "round_GBps": round(2 * 32.0 * n * n / (pr * 1e-3) / 1e9, 1)}
                out.append(rec)
                print(json.dumps(rec), flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--batch", type=int, default=100)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu-single-seconds", type=float, default=8.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ground", action="store_true", help="skip the ground-state time-to-solution")
    ap.add_argument("--no-other-grids", action="store_true", help="skip the 512^2 and 2048^2 lines")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched parameter sweep")
    ap.add_argument("--no-spin-hall", action="store_true", help="skip the spin-Hall trial")
    ap.add_argument("--ground-2048", type=int, default=60000, metavar="MAX_STEPS",
                    help="the 2048^2 ground state to |dE|/E < 1e-9 per 10 steps, at most MAX_STEPS (0: skip)")
    ap.add_argument("--workload", default="metric_1024")
    ap.add_argument("--heldout-sets", type=int, default=256,
                    help="held-out parameter sets of the learned-start comparison (256 in the workload)")
    ap.add_argument("--exchange-floor", action="store_true",
                    help="only measure the arithmetic-free copy with a step's data movement "
                         "(sgpe_probe_exchange) over layouts and tiles at 512^2-2048^2, print JSON, exit")
    ap.add_argument("--copy-reference", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (calibrates the HBM "
                         "byte counters of a profiler run) and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this solver runs one instance on one GPU; --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.exchange_floor:
        exchange_floor()
        return

    if args.copy_reference:
        n = args.copy_reference * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_reference_bytes_read": 4 * n, "copy_reference_bytes_written": 4 * n,
                          "launches": 5}))
        return

    from paper_2010_15069_amd import Solver
    from workloads import initial_state, preset

    p = preset(args.workload)                 # real time: dt = 5e-4
    p_imag = p.replace(dt=IMAG_DT)            # imaginary time: dt = 1e-3
    psi0 = initial_state(p, "tf", seed=0)     # the start does not depend on dt
    npts = p.nx * p.ny
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    s = Solver(p_imag, stream=stream.cuda_stream)
    s.set_psi(psi0)
    s_real = Solver(p, stream=stream.cuda_stream)

    def timed(step, k, batch):
        sizes = [min(batch, k - i) for i in range(0, k, batch)]
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(len(sizes) + 1)]
        torch.cuda.synchronize()
        evs[0].record(stream)
        for i, b in enumerate(sizes):
            step(b)
            evs[i + 1].record(stream)
        torch.cuda.synchronize()
        per = [evs[i].elapsed_time(evs[i + 1]) / b for i, b in enumerate(sizes)]
        total_ms = evs[0].elapsed_time(evs[-1])
        return total_ms, per

    # imaginary time (headline)
    s.step_imag(args.warmup)
    total_ms, per = timed(s.step_imag, args.steps, args.batch)
    med, mad = median_mad(per)
    value = args.steps / (total_ms * 1e-3)
    e_final = s.energy()

    progress("imaginary-time 1024^2 timed")
    # real time, same workload
    s_real.set_psi(psi0)
    s_real.step_real(args.warmup)
    total_r, per_r = timed(s_real.step_real, args.steps, args.batch)
    med_r, mad_r = median_mad(per_r)
    s_real.close()

    # Dominant kernel's launch duration in the real (alternating) schedule.  The steady-state step
    # time is the difference of two timed calls (one HIP event pair each, on the solver's stream),
    # step_imag(n + 1000) and step_imag(n), over 1000: the call boundary's sweeps (the first x
    # transform and half K, the last inverse x transform) cancel.  HIP events around every launch
    # of 200 further steps split that time between the two passes (the events' own overhead is
    # the same for both launches, so only their ratio is used).
    s.set_psi(psi0)
    s.step_imag(20)
    t_short, _ = timed(s.step_imag, 200, 200)
    t_long, _ = timed(s.step_imag, 1200, 1200)
    steady_ms = (t_long - t_short) / 1000.0
    ev_row, ev_col = s.profile_steps(200, imag=True)
    row_ms = steady_ms * ev_row / (ev_row + ev_col)
    col_ms = steady_ms * ev_col / (ev_row + ev_col)
    dom_name, dom_ms = ("col_pass", col_ms) if col_ms >= row_ms else ("row_pass", row_ms)
    alg_bytes = BYTES_PER_POINT_PASS * npts
    achieved = alg_bytes / (dom_ms * 1e-3) / 1e9
    traffic = _traffic_record(dom_name, args.workload, s.get_schedule())

    out = {
        "metric": "split-steps/s at 1024^2x2 c64 (%HBM roofline); ground-state time-to-1e-6 E",
        "value": value,
        "unit": "split-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "seed": 0,
        "device": torch.cuda.get_device_name(0),
        "rocm": getattr(torch.version, "hip", None),
        "config": {
            "workload": f"{args.workload}: {p.nx}x{p.ny} grid x 2 components, complex64 state, "
                        f"imaginary-time Strang split steps with renormalisation, g=10 (all), k_L=2, "
                        f"Omega=1 (k-space), delta=0.2, harmonic trap, Thomas-Fermi start",
            "grid": [p.ny, p.nx], "components": 2, "dt": p_imag.dt, "dt_real": p.dt,
            "batch": args.batch,
        },
        # one batch (K <= batch): a single timed call, whose time includes the call's start and end
        # after and before a synchronisation (it continues the warm-up's schedule: 2K sweeps for K
        # steps); no spread to report
        "step_ms_median": med, "step_ms_mad": mad if len(per) > 1 else None,
        "timed_calls": len(per),
        "note": f"the timed region is {len(per)} step_imag call(s) of at most {args.batch} steps, after the "
                f"untimed warm-up call; consecutive calls continue one fused schedule: each call leaves its "
                f"last half-step (K(dt/2) and the inverse x transform) to the next call, whose first sweep "
                f"merges it with its own first K(dt/2), so the timed calls run 2 sweeps per step; the first "
                f"timed sweep completes the warm-up's pending half-step, and the one the last timed call "
                f"leaves is completed after the timed region (by the energy read)",
        "hbm_roofline_frac_step": BYTES_PER_POINT_STEP * npts * value / (HBM_PEAK_GBS * 1e9),
        # the same rate priced at one sweep per step (32 B per point: each value read and written
        # once), the floor no two-pass 2-D transform reaches; reported beside the two-sweep figure
        "hbm_roofline_frac_step_one_sweep": BYTES_PER_POINT_STEP // 2 * npts * value / (HBM_PEAK_GBS * 1e9),
        "steady_state": {"step_ms": steady_ms, "split_steps_per_s": 1e3 / steady_ms,
                         "hbm_roofline_frac_step": BYTES_PER_POINT_STEP * npts / (steady_ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
                         "method": "(time of step_imag(1200) - time of step_imag(200)) / 1000, one event pair each"},
        "real_time": {"value": args.steps / (total_r * 1e-3), "unit": "split-steps/s",
                      "step_ms_median": med_r, "step_ms_mad": mad_r if len(per_r) > 1 else None},
        "kernels_ms": {"row_pass": row_ms, "col_pass": col_ms,
                       "per_launch_events": {"row_pass": ev_row, "col_pass": ev_col},
                       "method": "steady-state step time split between the passes in the ratio of "
                                 "per-launch HIP event durations"},
        "paper_context": PAPER_CONTEXT,
        "energy_after_timed_steps": e_final,
        "roofline": {"bound": "hbm", "kernel": dom_name, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic["bytes_per_launch"] if traffic else None,
                     "traffic_detail": traffic, "alg_bytes_per_launch": alg_bytes,
                     "launch_ms": dom_ms},
    }
    s.close()
    out["roofline_references"] = roofline_references(torch, p.nx, steady_ms, achieved)
    progress("real-time 1024^2 and per-pass timing")
    if not args.no_other_grids:
        out["other_grids"] = other_grids(torch, stream, timed, p)
        out["splitting_variants"] = splitting_variants(torch, stream, timed, p, p_imag, psi0)
        out["complex128"] = complex128_rates(torch, stream, timed, p, p_imag, psi0)
        progress("other grids, splitting variants, complex128")
    if not args.no_ground:
        out["ground_state"] = ground_state_time(torch, stream)
        progress("ground state 256^2")
        if args.ground_2048:
            out["ground_2048"] = ground_2048_convergence(torch, stream, max_steps=args.ground_2048)
            progress("ground state 2048^2")
        model = _load_surrogate(torch)
        if model is not None:
            out["ground_state"]["learned_start"] = ground_state_learned(torch, stream, model)
            if not args.no_batch:
                out["learned_start_sweep"] = learned_start_sweep(torch, stream, model, n_sets=args.heldout_sets)
            del model
            progress("learned start")
    if not args.no_batch:
        out["batched_sweep"] = batched_sweep(torch, stream)
        progress("batched sweep")
    if not args.no_spin_hall:
        out["spin_hall_trial"] = spin_hall_trial(torch)
        progress("spin-Hall trial")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, psi0, args.cpu_seconds, args.cpu_single_seconds)
        progress("oracle CPU baseline")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
