"""Consecutive step calls continue one fused schedule (the last half-step of a call waits for the
next call of the same kind, or for whatever reads the state next): calls of n1 and n2 steps are
bit-identical to one call of n1 + n2, every reader sees the completed state, and a context on a
caller's state buffer completes every call."""
import numpy as np
import pytest

from workloads import initial_state, preset

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2010_15069_amd as m
    if m.device_count() <= 0 or not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch, m


@pytest.mark.parametrize("precision", ["c64", "c128"])
@pytest.mark.parametrize("kind", ["imag", "real"])
def test_split_calls_equal_one_call(env, kind, precision):
    torch, m = env
    p = preset("ground_256", nx=128, ny=128)
    psi = initial_state(p, "tf", seed=5)
    print(f"case: 128^2 {precision} {kind}, 7 + 13 + 1 steps vs 21", flush=True)
    a = m.Solver(p, precision=precision).set_psi(psi)
    b = m.Solver(p, precision=precision).set_psi(psi)
    step_a = a.step_imag if kind == "imag" else a.step_real
    step_b = b.step_imag if kind == "imag" else b.step_real
    step_a(7)
    step_a(0)
    step_a(13)
    step_a(1)
    step_b(21)
    assert np.array_equal(a.get_psi(), b.get_psi())
    assert a.energy() == b.energy() and a.norm() == b.norm()


def test_readers_and_kind_changes_complete_the_step(env):
    # a reader, or a step of the other kind, completes the pending half-step exactly as the end of
    # a call would: the same results as explicit reads (get_psi) at the same points
    torch, m = env
    p = preset("ground_256", nx=128, ny=64)
    psi = initial_state(p, "tf", seed=6)
    a = m.Solver(p).set_psi(psi)
    a.step_imag(5)
    e5 = a.energy()
    a.step_imag(5)
    a.step_real(3)
    n = a.norm()
    a.step_real(2)
    b = m.Solver(p).set_psi(psi)
    b.step_imag(5)
    b.get_psi()
    b.step_imag(5)
    b.get_psi()
    b.step_real(3)
    b.get_psi()
    b.step_real(2)
    assert np.array_equal(a.get_psi(), b.get_psi())
    c = m.Solver(p).set_psi(psi).step_imag(5)
    assert c.energy() == e5
    d = m.Solver(p).set_psi(psi).step_imag(5)
    d.get_psi()
    d.step_imag(5).step_real(3)
    assert d.norm() == n
    # a schedule change completes the pending half-step under the schedule it began with
    e = m.Solver(p).set_psi(psi).step_imag(4)
    e.set_col_tile(1)
    f = m.Solver(p).set_psi(psi).step_imag(4)
    f.get_psi()
    f.set_col_tile(1)
    e.step_imag(3)
    f.step_imag(3)
    assert np.array_equal(e.get_psi(), f.get_psi())


def test_caller_state_buffer_holds_the_completed_state(env):
    torch, m = env
    p = preset("tiny")
    psi = initial_state(p, "gauss", seed=2)
    buf = torch.zeros((p.ny, p.nx, 4), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    s = m.Solver(p, psi_dev=buf.data_ptr()).set_psi(psi)
    s.step_imag(6)
    s.synchronize()
    g = s.get_psi()
    direct = buf.cpu().numpy().astype(np.float64)
    assert np.array_equal(direct[..., 0] + 1j * direct[..., 1], g[0])
    assert np.array_equal(direct[..., 2] + 1j * direct[..., 3], g[1])
    # every call completed: the same as a context of its own read between the two calls
    s.step_imag(6)
    s2 = m.Solver(p).set_psi(psi).step_imag(6)
    s2.get_psi()
    s2.step_imag(6)
    assert np.array_equal(s.get_psi(), s2.get_psi())
