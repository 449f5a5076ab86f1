"""Host logic of bench.py that decides reported figures: the stationarity
criterion of the wall-seconds-to-stationary leg."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def _reps(powers, states):
    return [dict(p_port=p, x=np.array([x, 0.5 * x])) for p, x in zip(powers, states)]


def test_stationary_index_first_period_of_a_stable_window():
    r = _reps([50, 70, 59, 60, 60.2, 59.9] + [60] * 10, [1, 1.2, 1.05, 1.0, 1.001, 0.999] + [1.0] * 10)
    assert bench.stationary_index(r, 60.0) == 3


def test_stationary_index_ignores_a_single_passing_period():
    # period 2 passes both tests, period 3 leaves the band again
    r = _reps([50, 70, 60, 66, 60] + [60] * 10, [1, 1.2, 1.0, 1.1, 1.0] + [1.0] * 10)
    assert bench.stationary_index(r, 60.0) == 4


def test_stationary_index_needs_a_whole_window():
    assert bench.stationary_index(_reps([60] * 9, [1.0] * 9), 60.0) is None
    assert bench.stationary_index(_reps([60] * 10, [1.0] * 10), 60.0) == 0
    # a drift of 0.2 % per period leaves the 1 % band within the window
    assert bench.stationary_index(_reps([60] * 12, [1.0 + 0.002 * k for k in range(12)]), 60.0) is None


def test_feature_scale_treats_constant_columns_as_unit_scale():
    # a constant column whose numerical std is one ulp, a varying one, an exact zero column
    a = np.column_stack([np.full(240, 2.666447368421053), np.linspace(0.0, 3.0, 240), np.zeros(240)])
    s = bench.feature_scale(a)
    assert s[0] == 1.0 and s[2] == 1.0
    assert abs(s[1] - np.std(np.linspace(0.0, 3.0, 240))) < 1e-15
