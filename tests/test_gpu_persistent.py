"""The persistent batch mode (one cooperative launch for every steady-state step of every instance)
against single contexts and against the per-class launches, through the C ABI: every instance
bit-identical to a single context with the persistent kernel's schedule (8 points per lane, 1024 / n
rows or columns per workgroup), in real and imaginary time, with and without graph capture, over
call lengths 1, 2 and longer; the 96-instance sweep equal to the per-class launches; one instance
against the FP64 oracle; the error paths; and a forced barrier give-up (a lowered poll bound, set
from the host) reported by the batch's synchronize with every kernel leaving normally."""
import os
import subprocess
import sys

import numpy as np
import pytest

from oracle import OracleGPE
from workloads import Params, initial_state, sweep_instances

pytestmark = pytest.mark.gpu

WORKERS = max(1, min(16, len(os.sched_getaffinity(0))))
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def api():
    from paper_2010_15069_amd import Batch, SgpeError, Solver, device_count
    if device_count() <= 0:
        pytest.skip("no HIP device")
    return Batch, Solver, SgpeError


def _single_schedule(n):
    return dict(row_points=8, col_points=8, row_tile=1024 // n, col_tile=1024 // n, row_iters=1, col_iters=1)


CALLS = [("imag", 37), ("imag", 1), ("imag", 2), ("real", 23), ("real", 1), ("imag", 5)]


@pytest.mark.parametrize("graph", [True, False])
def test_bitwise_equal_to_single_contexts(api, graph):
    Batch, Solver, _ = api
    ps = sweep_instances(seed=5, sizes=(128, 256, 512), per_size=2)
    starts = [initial_state(p, "tf", seed=100 + i) for i, p in enumerate(ps)]
    b = Batch(ps)
    for i, s0 in enumerate(starts):
        b.set_psi(i, s0)
    b.use_graph(graph)
    b.use_persistent(True)
    print(f"case: 6 instances (128^2, 256^2, 512^2), persistent, graph={graph}", flush=True)
    for kind, n in CALLS:
        getattr(b, f"step_{kind}")(n)
    b.synchronize()
    for i, p in enumerate(ps):
        s = Solver(p).set_schedule(**_single_schedule(p.nx)).set_psi(starts[i])
        for kind, n in CALLS:
            # the batch completes every call; a single context leaves a call's last half-step for
            # its next call of the same kind unless something reads the state in between
            getattr(s, f"step_{kind}")(n)
            s.synchronize()
        assert np.array_equal(b.get_psi(i), s.get_psi()), f"instance {i} ({p.nx}^2)"
        s.close()
    b.close()


def test_sweep_equal_to_per_class_launches(api):
    Batch, _, _ = api
    ps = sweep_instances(seed=0)
    starts = [initial_state(p, "tf", seed=i) for i, p in enumerate(ps)]
    a = Batch(ps)
    c = Batch(ps)
    for i, s0 in enumerate(starts):
        a.set_psi(i, s0)
        c.set_psi(i, s0)
    a.use_persistent(True)
    c.use_persistent(True)
    c.use_persistent(False)      # same schedules, per-class launches
    print("case: 96-instance sweep, 60 imaginary steps, persistent vs per-class", flush=True)
    a.step_imag(60)
    c.step_imag(60)
    for i in range(len(ps)):
        assert np.array_equal(a.get_psi(i), c.get_psi(i)), i
    a.close()
    c.close()


def test_one_instance_against_the_oracle(api):
    Batch, _, _ = api
    p = sweep_instances(seed=7, sizes=(128,), per_size=1)[0]
    psi0 = initial_state(p, "tf", seed=3)
    b = Batch([p, p.replace(g_uu=2.0 * p.g_uu, g_dd=2.0 * p.g_dd, g_ud=2.0 * p.g_ud)])
    b.set_psi(0, psi0)
    b.set_psi(1, psi0)
    b.use_persistent(True)
    b.step_imag(300)
    o = OracleGPE(p, workers=WORKERS)
    o.set_psi(psi0)
    o.step_imag(300)
    g = b.get_psi(0)
    err = float(np.linalg.norm(g - o.psi) / np.linalg.norm(o.psi))
    assert err <= 1e-5, err
    assert abs(b.energy(0) - o.energy()) <= 1e-6 * abs(o.energy())


def test_error_paths(api):
    Batch, _, SgpeError = api
    with pytest.raises(SgpeError, match="SGPE_EINVAL"):
        Batch([Params(nx=64, ny=64)]).use_persistent(True)              # size not supported
    with pytest.raises(SgpeError, match="SGPE_EINVAL"):
        Batch([Params(nx=256, ny=128)]).use_persistent(True)            # not square
    with pytest.raises(SgpeError, match="SGPE_EINVAL"):
        Batch([Params(nx=128, ny=128, omega_r0=1.0)]).use_persistent(True)   # spatial Raman coupling
    b = Batch([Params(nx=128, ny=128)])
    b.use_persistent(True)
    with pytest.raises(SgpeError, match="SGPE_ESTATE"):
        b.set_schedule(0, col_tile=4)
    with pytest.raises(SgpeError, match="SGPE_ESTATE"):
        b.autotune(2)
    b.use_persistent(False)
    b.set_schedule(0, None)


FORCED_GIVE_UP = r"""
import numpy as np
from paper_2010_15069_amd import Batch, SgpeError
from workloads import initial_state, sweep_instances
ps = sweep_instances(seed=5, sizes=(128, 256), per_size=2)
b = Batch(ps)
for i, p in enumerate(ps):
    b.set_psi(i, initial_state(p, "tf", seed=i))
b.use_graph(False)
b.use_persistent(True)                 # the lowered poll bound is read here
try:
    b.step_imag(5)
    b.synchronize()
    print("NO-ERROR")
except SgpeError as e:
    print("GAVE-UP", e.status, str(e))
"""


def test_forced_barrier_give_up_is_reported(api):
    # a poll bound of 0 makes the first barrier give up; run in a child process so that the
    # lowered bound stays there
    env = dict(os.environ, SGPE_PERSIST_SPIN_LIMIT="0", PYTHONPATH=ROOT, AMD_LOG_LEVEL="1")
    print("case: persistent batch with the barrier poll bound at 0 (child process)", flush=True)
    out = subprocess.run([sys.executable, "-c", FORCED_GIVE_UP], env=env, cwd=ROOT, stdout=subprocess.PIPE,
                         stderr=subprocess.STDOUT, text=True, timeout=120)
    assert out.returncode == 0, out.stdout
    assert "GAVE-UP 3" in out.stdout, out.stdout        # SGPE_EDEVICE
