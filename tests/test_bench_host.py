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


def _reps_x(powers, mags):
    """Reports whose state x = (I_f, I_1, V_1): turn magnitudes as given."""
    return [dict(p_port=p, x=np.array([1.0, m, 2.0 * m], complex)) for p, m in zip(powers, mags)]


def test_stationary_q27_compares_window_means_with_the_preceding_window():
    # a settled run: power in the band and magnitudes flat from period 3
    r = _reps_x([50, 55, 58] + [60] * 30, [1.5, 1.4, 1.3] + [1.0] * 30)
    # window 10: the preceding window [i-10, i) must be settled too, so the
    # first index is 13 (its preceding window starts at 3)
    assert bench.stationary_q27(r, 60.0, window=10) == 13


def test_stationary_q27_rejects_a_drift_above_one_percent_per_window():
    # magnitudes grow 0.2 % per period: window means move 2 % per window
    r = _reps_x([60] * 40, [1.0 + 0.002 * k for k in range(40)])
    assert bench.stationary_q27(r, 60.0, window=10) is None
    # 0.05 % per period: 0.5 % per window passes from the first possible index
    r = _reps_x([60] * 40, [1.0 + 0.0005 * k for k in range(40)])
    assert bench.stationary_q27(r, 60.0, window=10) == 10


def test_stationary_q27_needs_the_power_band_over_the_whole_window():
    r = _reps_x([60] * 15 + [61] + [60] * 24, [1.0] * 40)
    # period 15 is 1.7 % off: windows containing it fail
    assert bench.stationary_q27(r, 60.0, window=10) == 16


def test_settled_index_needs_the_band_to_the_end():
    r = _reps_x([50, 58, 60.5, 59.5, 60.2] + [60] * 10, [1.0] * 15)
    assert bench.settled_index(r, 60.0) == 2
    # a late excursion moves the settling period past it
    r = _reps_x([60] * 5 + [61] + [60] * 12, [1.0] * 18)
    assert bench.settled_index(r, 60.0) == 6
    # in band only over the last 9 periods: too short to count
    r = _reps_x([50] * 6 + [60] * 9, [1.0] * 15)
    assert bench.settled_index(r, 60.0) is None
