"""Host-side helpers of bench.py on synthetic inputs."""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import bench  # noqa: E402


def test_aitken_recovers_a_geometric_approach():
    # E_n = E_inf + A r^(n / 5000): the estimate recovers E_inf and the remaining distance
    e_inf, a, r = -1.25, 0.02, 0.5
    trace = [(n, 0.0, e_inf + a * r ** (n / 5000)) for n in range(10, 150001, 10)]
    est = bench._aitken_estimate(trace)
    last = est["last"]
    assert abs(last["energy_inf"] - e_inf) < 1e-12
    assert abs(last["distance_rel"] - a * r ** 30 / abs(e_inf)) < 1e-12
    assert abs(last["ratio_per_spacing"] - r) < 1e-9
    # the first 5000-step mark whose estimated distance is below 1e-6 |E|
    k = next(k for k in range(3, 31) if a * r ** k / abs(e_inf) < 1e-6)
    assert est["steps_to_estimated_1e-6"] == 5000 * k


def test_median_mad():
    med, mad = bench.median_mad([1.0, 2.0, 3.0, 4.0, 100.0])
    assert med == 3.0 and mad == 1.0
