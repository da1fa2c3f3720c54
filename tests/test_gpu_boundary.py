"""GPU checks of the boundary's error contract: a non-finite imaginary-time norm (the
renormalisation of Sec. 3.2 divides by it) is latched in the context and reported by the next
synchronising call; set_psi clears it.  The states here are finite complex64 values whose squares
overflow fp32: a data-level overflow, with every kernel running to its normal end."""
import ctypes

import numpy as np
import pytest

from workloads import initial_state, preset

pytestmark = pytest.mark.gpu

SGPE_OK, SGPE_ENONFINITE = 0, 4


@pytest.fixture(scope="module")
def lib():
    from paper_2010_15069_amd import _lib, device_count
    if device_count() <= 0:
        pytest.skip("no HIP device")
    return _lib.lib()


def test_overflowing_norm_is_latched_by_synchronize(lib):
    from paper_2010_15069_amd import Solver
    p = preset("tiny")
    good = initial_state(p, "gauss", seed=0)
    s = Solver(p)
    print("case: tiny 64^2, |psi| ~ 1e20 then step_imag(2)", flush=True)
    s.set_psi(good * 1e20)          # finite in fp32; |psi|^2 ~ 1e40 is not
    assert lib.sgpe_step_imag(s._ctx, 2) == SGPE_OK   # asynchronous: nothing reported yet
    assert lib.sgpe_synchronize(s._ctx) == SGPE_ENONFINITE
    assert lib.sgpe_synchronize(s._ctx) == SGPE_ENONFINITE   # stays latched
    d = ctypes.c_double()
    assert lib.sgpe_norm(s._ctx, ctypes.byref(d)) == SGPE_ENONFINITE
    # a fresh state clears the latch; ordinary steps then report success
    s.set_psi(good)
    assert lib.sgpe_synchronize(s._ctx) == SGPE_OK
    assert lib.sgpe_step_imag(s._ctx, 5) == SGPE_OK
    assert lib.sgpe_synchronize(s._ctx) == SGPE_OK
    assert abs(s.norm() - p.norm0) < 1e-6


def test_zero_state_norm_is_latched(lib):
    from paper_2010_15069_amd import Solver
    p = preset("tiny")
    s = Solver(p)
    print("case: tiny 64^2, zero state then step_imag(3)", flush=True)
    s.set_psi(np.zeros((2, p.ny, p.nx), dtype=np.complex128))
    assert lib.sgpe_step_imag(s._ctx, 3) == SGPE_OK
    assert lib.sgpe_synchronize(s._ctx) == SGPE_ENONFINITE


def test_real_time_steps_do_not_latch(lib):
    # real time has no renormalisation; a finite ordinary run reports success
    from paper_2010_15069_amd import Solver
    p = preset("tiny")
    s = Solver(p).set_psi(initial_state(p, "gauss", seed=1))
    assert lib.sgpe_step_real(s._ctx, 10) == SGPE_OK
    assert lib.sgpe_synchronize(s._ctx) == SGPE_OK


def test_batch_reports_a_nonfinite_instance(lib):
    from paper_2010_15069_amd import Batch
    ps = [preset("tiny"), preset("tiny", g_uu=2.0, g_dd=2.0, g_ud=1.8)]
    b = Batch(ps)
    b.set_psi(0, initial_state(ps[0], "gauss", seed=0))
    b.set_psi(1, initial_state(ps[1], "gauss", seed=1) * 1e20)
    print("case: batch of two 64^2 instances, the second overflowing", flush=True)
    assert lib.sgpe_batch_step_imag(b._b, 2) == SGPE_OK
    assert lib.sgpe_batch_synchronize(b._b) == SGPE_ENONFINITE
    b.set_psi(1, initial_state(ps[1], "gauss", seed=1))
    assert lib.sgpe_batch_step_imag(b._b, 2) == SGPE_OK
    assert lib.sgpe_batch_synchronize(b._b) == SGPE_OK
