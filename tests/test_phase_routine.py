"""The real-space exponential's phase routines, built for the host from the kernels' own header and
checked against fp64 sine and cosine (no GPU needed).

The real-time exponential of Eqs. (H2)-(H4) multiplies each component by exp(-i phi) (diagonal
case) or by cos(theta) 1 - i sin(theta)/theta (hB . sigma) (full 2x2 case).  The kernels form
(cos(phi) - 1, sin(phi), sin(phi)/phi) with relative accuracy for small angles: a short Taylor form
for |phi| <= pi/4 and a Cody-Waite reduction by pi/2 beyond.  Checked here:

* the general routine against fp64 over [-20, 20] rad (every quadrant, and k = rint(2 phi / pi)
  a nonzero multiple of 4, where sin(r)/r of the reduced angle is not sin(phi)/phi);
* relative accuracy of cos(phi) - 1 and sin(phi) for small angles;
* the general routine returns the short routine's bits for |phi| <= pi/4, so a wave's choice of
  routine does not change results.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "phase_routine_host.hip")
CSRC = os.path.join(ROOT, "paper_2010_15069_amd", "csrc")
HIPCC = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")


@pytest.fixture(scope="module")
def routine(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("phase") / "phase_routine")
    cmd = [HIPCC, "-O2", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature",
           "-Xclang", "-packed-fp32-ops", "-I", CSRC, "-I", os.path.join(ROOT, "include"), SRC, "-o", out]
    proc = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert proc.returncode == 0, proc.stdout

    def run(phis):
        phis = np.asarray(phis, dtype=np.float32)
        text = "\n".join(float(p).hex() for p in phis) + "\n"
        res = subprocess.run([out], input=text, stdout=subprocess.PIPE, text=True, check=True)
        rows = [[float.fromhex(v) for v in line.split()] for line in res.stdout.splitlines()]
        a = np.array(rows, dtype=np.float64)
        assert a.shape == (len(phis), 7)
        assert np.array_equal(a[:, 0], phis.astype(np.float64))
        return a
    return run


def exact(phi):
    phi = np.asarray(phi, dtype=np.float64)
    s = np.sin(phi)
    cm1 = -2.0 * np.sin(0.5 * phi) ** 2
    sinc = np.where(phi == 0.0, 1.0, s / np.where(phi == 0.0, 1.0, phi))
    return cm1, s, sinc


def test_general_routine_over_minus20_to_20(routine):
    phis = np.linspace(-20.0, 20.0, 80001, dtype=np.float32)
    # the quadrant edges and whole turns, and a float either side of each
    k = np.arange(-13, 14)
    edges = np.concatenate([k * np.pi / 2, k * np.pi / 2 + np.pi / 4]).astype(np.float32)
    edges = np.concatenate([edges, np.nextafter(edges, np.float32(np.inf)),
                            np.nextafter(edges, np.float32(-np.inf))])
    phis = np.concatenate([phis, edges[np.abs(edges) <= 20.0]])
    a = routine(phis)
    cm1, s, sinc = exact(a[:, 0])
    # fp32 result of magnitude <= 2: a few units in the last place of 1
    assert np.max(np.abs(a[:, 1] - cm1)) < 5e-7
    assert np.max(np.abs(a[:, 2] - s)) < 5e-7
    big = np.abs(a[:, 0]) > 0.5
    assert np.max(np.abs(a[big, 3] - sinc[big]) * np.abs(a[big, 0])) < 5e-7
    small = ~big
    assert np.max(np.abs(a[small, 3] - sinc[small])) < 3e-7


def test_whole_turns_give_sinc_of_phi(routine):
    # k = rint(2 phi / pi) a nonzero multiple of 4: sin(phi)/phi is close to zero at phi = 2 pi,
    # not sin(r)/r = 1 of the reduced angle
    phis = np.array([2 * np.pi, -2 * np.pi, 4 * np.pi, 5.6, -5.6, 6.0, 13.0, -13.0], dtype=np.float32)
    a = routine(phis)
    _, _, sinc = exact(a[:, 0])
    assert np.max(np.abs(a[:, 3] - sinc)) < 1e-7
    assert abs(a[0, 3]) < 1e-7


def test_small_angles_relative_accuracy(routine):
    mags = np.float32(np.pi / 4) * np.logspace(-12, 0, 4001, dtype=np.float64).astype(np.float32)
    phis = np.concatenate([mags, -mags])
    a = routine(phis)
    cm1, s, _ = exact(a[:, 0])
    eps = np.float64(np.finfo(np.float32).eps)
    for col in (1, 4):   # general and short routine
        assert np.max(np.abs(a[:, col] - cm1) / np.abs(cm1)) < 8 * eps
    for col in (2, 5):
        assert np.max(np.abs(a[:, col] - s) / np.abs(s)) < 4 * eps


def test_general_matches_short_routine_bits_below_pi_over_4(routine):
    phis = np.linspace(-np.pi / 4, np.pi / 4, 20001, dtype=np.float32)
    phis = phis[np.abs(phis) <= np.float32(0.785398163)]
    a = routine(phis)
    assert np.array_equal(a[:, 1:4], a[:, 4:7])
