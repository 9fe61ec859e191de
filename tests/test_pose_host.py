"""Host logic of the learned-pose driver (paper_2508_04929_amd/pose.py)
without a GPU: the fallback threshold calibrated on validation particles."""
import numpy as np
import pytest


def test_fallback_threshold_calibration():
    """The smallest set of lowest-fit particles whose grid-search errors
    bring the mean within the margin; the threshold separates exactly that
    set; no fallback when the learned mean already qualifies; everything
    when nothing short of the grid search does; undefined fits first."""
    from paper_2508_04929_amd.pose import calibrate_threshold
    z = np.array([0.9, 0.1, 0.5, 0.8, np.nan, 0.3])
    e_l = np.array([2.0, 90.0, 3.0, 2.0, 120.0, 40.0])
    e_g = np.array([2.0, 5.0, 3.0, 2.0, 6.0, 4.0])
    # grid mean 3.667; learned mean 42.83; replacing nan (k=1) -> 23.83,
    # then z=0.1 (k=2) -> 9.67, then z=0.3 (k=3) -> 3.67 <= 3.667 + 0.5
    tau, frac = calibrate_threshold(z, e_l, e_g, 0.5)
    assert frac == pytest.approx(3 / 6)
    assert 0.3 < tau < 0.5
    fb = ~(z >= tau)
    assert fb.tolist() == [False, True, False, False, True, True]
    tau0, frac0 = calibrate_threshold(z, e_g, e_g, 0.5)
    assert frac0 == 0.0 and not np.any(np.nan_to_num(z, nan=1.0) < tau0)
    tau1, frac1 = calibrate_threshold(z, e_l, e_g, -10.0)
    assert frac1 == 1.0 and tau1 == float("inf")
