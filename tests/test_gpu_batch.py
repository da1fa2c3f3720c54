"""GPU: batched parameter sweeps (many instances, mixed grid shapes, one launch per class and
pass) against single contexts with the same schedule (bit-identical) and against the FP64
oracle; graph capture and replay; the autotuner."""
import os

import numpy as np
import pytest

from oracle import OracleGPE
from workloads import Params, gaussian_state, initial_state, preset, sweep_instances

pytestmark = pytest.mark.gpu

WORKERS = max(1, min(16, len(os.sched_getaffinity(0))))


@pytest.fixture(scope="module")
def sgpe():
    import paper_2010_15069_amd as m
    if m.device_count() <= 0:
        pytest.skip("no HIP device")
    return m


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def mixed_params():
    base = dict(xmax=8.0, ymax=6.0, wx=1.0, wy=1.3, dt=1e-3)
    return [
        Params(nx=64, ny=64, g_uu=3.0, g_dd=2.0, g_ud=1.0, k_l=1.0, omega=0.5, delta=0.1, **base),
        Params(nx=64, ny=64, g_uu=9.0, g_dd=9.0, g_ud=9.0, k_l=2.0, omega=1.5, delta=-0.3, **base),
        Params(nx=128, ny=64, g_uu=5.0, g_dd=4.0, g_ud=4.5, k_l=0.5, omega=0.0, delta=0.2, **base),
        Params(nx=64, ny=64, g_uu=1.0, g_dd=1.0, g_ud=0.5, k_l=0.0, omega=2.0, delta=0.0, **base),
        Params(nx=32, ny=256, g_uu=2.0, g_dd=2.5, g_ud=1.0, k_l=1.5, omega=0.7, delta=0.4,
               omega_r0=1.0, omega_rw=2.0, **base),
        Params(nx=128, ny=64, g_uu=7.0, g_dd=7.0, g_ud=3.0, k_l=2.0, omega=1.0, delta=-0.1, **base),
    ]


def states(params, seed=0):
    return [gaussian_state(p, sigma=1.3, seed=seed + i, noise=1e-2).astype(np.complex64).astype(complex)
            for i, p in enumerate(params)]


def test_batch_classes_and_bitwise_equality_with_single_contexts(sgpe):
    ps = mixed_params()
    psi0 = states(ps)
    b = sgpe.Batch(ps)
    assert len(b) == len(ps)
    cls = b.classes()
    assert sorted((nx, ny) for nx, ny, _ in cls) == sorted({(64, 64), (128, 64), (32, 256)})
    for i, psi in enumerate(psi0):
        b.set_psi(i, psi)
    b.step_imag(7).step_real(5)
    for i, p in enumerate(ps):
        s = sgpe.Solver(p)
        s.set_schedule(b.get_schedule(b.instance_class(i)))
        s.set_psi(psi0[i]).step_imag(7).step_real(5)
        assert np.array_equal(b.get_psi(i), s.get_psi()), i
        assert b.energy(i) == s.energy() and b.norm(i) == s.norm(), i
        s.close()
    b.close()


def test_batch_graph_replays_match_direct_launches(sgpe):
    ps = mixed_params()
    psi0 = states(ps, seed=10)
    g, d = sgpe.Batch(ps).use_graph(True), sgpe.Batch(ps).use_graph(False)
    for i, psi in enumerate(psi0):
        g.set_psi(i, psi)
        d.set_psi(i, psi)
    for rep in range(3):
        # the same captured graph replayed, with eager work and synchronisation in between
        g.step_imag(6)
        d.step_imag(6)
        for i in range(len(ps)):
            assert np.array_equal(g.get_psi(i), d.get_psi(i)), (rep, i)
        g.step_real(4)
        d.step_real(4)
        e = [g.energy(i) for i in range(len(ps))]
        assert e == [d.energy(i) for i in range(len(ps))], rep
    g.close()
    d.close()


def test_batch_autotune_keeps_state_and_agrees_with_set_schedule(sgpe):
    ps = mixed_params()
    psi0 = states(ps, seed=20)
    a, b = sgpe.Batch(ps), sgpe.Batch(ps)
    for i, psi in enumerate(psi0):
        a.set_psi(i, psi)
        b.set_psi(i, psi)
    before = [a.get_psi(i) for i in range(len(ps))]
    ms = a.autotune(3)
    assert len(ms) == len(a.classes()) and all(m > 0 for m in ms)
    for i in range(len(ps)):
        assert np.array_equal(a.get_psi(i), before[i]), i
    for k in range(len(a.classes())):
        b.set_schedule(k, a.get_schedule(k))
    a.step_real(6).step_imag(4)
    b.step_real(6).step_imag(4)
    for i in range(len(ps)):
        assert np.array_equal(a.get_psi(i), b.get_psi(i)), i
    a.close()
    b.close()


def test_batch_sweep_instances_against_oracle(sgpe):
    # the sweep workload's parameter draws, one instance per size, against the FP64 oracle
    ps = sweep_instances(seed=3, sizes=(128, 256, 512), per_size=2)
    psi0 = [initial_state(p, "tf", seed=i) for i, p in enumerate(ps)]
    b = sgpe.Batch(ps)
    for i, psi in enumerate(psi0):
        b.set_psi(i, psi)
    b.step_imag(20)
    for i in (0, 3, 5):
        o = OracleGPE(ps[i], workers=WORKERS)
        o.set_psi(psi0[i])
        o.step_imag(20)
        assert rel_l2(b.get_psi(i), o.psi) <= 1e-5, i
        eo = o.energy()
        assert abs(b.energy(i) - eo) <= 1e-6 * abs(eo), i
    b.close()


def test_batch_energies_at_once_match_one_by_one(sgpe):
    # every class (square and ragged grids, a spatial Raman coupling) in one launch per kernel
    ps = mixed_params()
    print("case: mixed batch of 6, energies() vs energy(i)", flush=True)
    b = sgpe.Batch(ps)
    with pytest.raises(sgpe.SgpeError, match="SGPE_ESTATE"):
        b.energies()            # no state yet
    for i, psi in enumerate(states(ps)):
        b.set_psi(i, psi)
    for n in (0, 15):
        if n:
            b.step_imag(n)
        e_all = b.energies()
        e_one = np.array([b.energy(i) for i in range(len(ps))])
        np.testing.assert_allclose(e_all, e_one, rtol=1e-13, atol=0)
    # the sweep workload's sizes, against the oracle
    qs = sweep_instances(seed=4, sizes=(128, 256), per_size=3)
    q0 = [initial_state(p, "tf", seed=i) for i, p in enumerate(qs)]
    c = sgpe.Batch(qs)
    for i, psi in enumerate(q0):
        c.set_psi(i, psi)
    e = c.energies()
    for i in (0, 4):
        o = OracleGPE(qs[i], workers=WORKERS)
        o.set_psi(q0[i])
        eo = o.energy()
        assert abs(e[i] - eo) <= 1e-6 * abs(eo), i
    # a non-finite instance: every value is written, the call reports it
    bad = q0[1] * 1e20
    c.set_psi(1, bad)
    c.step_imag(2)
    with pytest.raises(sgpe.SgpeError, match="SGPE_ENONFINITE"):
        c.energies()
    b.close()
    c.close()


def test_batch_errors(sgpe):
    ps = mixed_params()[:2]
    b = sgpe.Batch(ps)
    with pytest.raises(sgpe.SgpeError):
        b.step_imag(1)          # no state yet
    for i in range(2):
        b.set_psi(i, states(ps)[i])
    with pytest.raises(sgpe.SgpeError):
        b.energy(5)             # index out of range
    with pytest.raises(sgpe.SgpeError):
        b.set_schedule(0, row_iters=2)   # batched launches take one tile per workgroup
    b.close()


def test_workgroup_placement_follows_dispatch_order(sgpe):
    # The batched and persistent launches keep an instance's workgroups on one XCD by relying on
    # the dispatcher's order: workgroup L of a launch (x fastest) runs on XCD (s + L) mod 8, where s
    # is where the dispatcher's rotation stood when the launch began.  Results never depend on it,
    # only the locality does.  The probe reads each workgroup's hardware XCC_ID.
    from paper_2010_15069_amd import probe_placement
    for gx, gy, threads in [(1024, 1, 256), (64, 32, 256), (7, 32, 128), (768, 1, 256), (13, 1, 64)]:
        xcd = probe_placement(gx, gy, threads).ravel()
        print(f"case: placement {gx}x{gy}x{threads}: first 16 {xcd[:16].tolist()}", flush=True)
        assert xcd.max() < 8
        shift = (xcd.astype(np.int64) - np.arange(gx * gy)) % 8
        assert np.all(shift == shift[0]), np.unique(shift)
