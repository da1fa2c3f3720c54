"""sgpe_set_psi_device: a state handed over in device memory, in the context's own layout, against
the same values through sgpe_set_psi (bit-identical states), its non-finite check, and the learned
start's device-side prediction against the host one."""
import ctypes

import numpy as np
import pytest

from workloads import initial_state, preset, sweep_instances

pytestmark = pytest.mark.gpu

SGPE_EINVAL, SGPE_ENONFINITE = 1, 4


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2010_15069_amd as m
    if m.device_count() <= 0 or not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch, m


def _layout(psi, dtype, torch):
    """(2, ny, nx) complex -> (ny, nx, 4) of (re_up, im_up, re_dn, im_dn) on the device."""
    a = np.stack([psi[0].real, psi[0].imag, psi[1].real, psi[1].imag], axis=-1).astype(dtype)
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_equals_host_set_psi(env, precision):
    torch, m = env
    p = preset("ground_256", nx=128, ny=64)
    psi = initial_state(p, "tf", seed=3)
    dtype = np.float32 if precision == "c64" else np.float64
    if precision == "c64":
        psi = psi.astype(np.complex64).astype(np.complex128)
    print(f"case: 128x64 {precision} set_psi_device vs set_psi", flush=True)
    a = m.Solver(p, precision=precision).set_psi(psi)
    b = m.Solver(p, precision=precision).set_psi_device(_layout(psi, dtype, torch))
    assert np.array_equal(a.get_psi(), b.get_psi())
    a.step_imag(20)
    b.step_imag(20)
    assert np.array_equal(a.get_psi(), b.get_psi()) and a.energy() == b.energy()


def test_nonfinite_and_misaligned_are_rejected(env):
    torch, m = env
    p = preset("tiny")
    psi = initial_state(p, "gauss", seed=1).astype(np.complex64).astype(np.complex128)
    s = m.Solver(p).set_psi(psi)
    before = s.get_psi()
    t = _layout(psi, np.float32, torch)
    t[5, 7, 2] = float("nan")
    torch.cuda.synchronize()
    assert s._lib.sgpe_set_psi_device(s._ctx, ctypes.c_void_p(t.data_ptr())) == SGPE_ENONFINITE
    assert np.array_equal(s.get_psi(), before)                     # unchanged
    big = torch.zeros(4 * p.nx * p.ny + 2, dtype=torch.float32, device="cuda")
    assert s._lib.sgpe_set_psi_device(s._ctx, ctypes.c_void_p(big.data_ptr() + 8)) == SGPE_EINVAL
    with pytest.raises(ValueError):
        s.set_psi_device(t.double())                               # wrong dtype for complex64


def test_batch_and_learned_start_on_the_device(env):
    torch, m = env
    from paper_2010_15069_amd import surrogate
    from paper_2010_15069_amd.train_surrogate import WEIGHTS
    model = surrogate.load(WEIGHTS, "cuda")
    ps = sweep_instances(seed=2, sizes=(256,), per_size=3)
    host = surrogate.predict(model, ps, "cuda")
    dev = surrogate.predict_device(model, ps, "cuda")
    b = m.Batch(ps)
    for i in range(len(ps)):
        b.set_psi_device(i, dev[i])
        g = b.get_psi(i)
        # the same prediction, normalised in fp32 (device) or fp64 then rounded (host)
        assert np.linalg.norm(g - host[i]) <= 1e-6 * np.linalg.norm(host[i]), i
        assert abs(b.norm(i) - ps[i].norm0) <= 1e-5 * ps[i].norm0
    c = m.Batch(ps)
    for i in range(len(ps)):
        c.set_psi(i, b.get_psi(i))
    b.step_imag(30)
    c.step_imag(30)
    for i in range(len(ps)):
        assert np.array_equal(b.get_psi(i), c.get_psi(i)), i
