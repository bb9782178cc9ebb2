"""Pins of the accuracy metrics of the experiments module (host arithmetic,
no GPU): bad-pixel rates and mean relative error counted by hand."""
from __future__ import annotations

import numpy as np
import pytest

from lfsynth.rig import line_rig


def test_bad_pixels_counted_by_hand():
    from paper_1812_06856_amd.experiments import depth_errors

    gt = np.array([[2.0, 2.0, 4.0, 0.0]])
    # focal * baseline = 20: disparity 10 at depth 2, 5 at depth 4
    d = np.array([[2.0, 20 / 10.8, 20 / 5.4, 3.0]])   # errors 0, 0.8, 0.4 px; the last pixel has no ground truth
    e = depth_errors(d, gt, focal=100.0, baseline=0.2)
    assert e["pixels"] == 3
    assert e["bad_1"] == 0.0
    assert e["bad_0.5"] == pytest.approx(1 / 3)
    assert e["mare"] == pytest.approx((0.0 + abs(20 / 10.8 - 2) / 2 + abs(20 / 5.4 - 4) / 4) / 3)
    # a missing estimate is bad at every threshold
    d2 = d.copy()
    d2[0, 0] = 0.0
    e2 = depth_errors(d2, gt, focal=100.0, baseline=0.2)
    assert e2["bad_1"] == pytest.approx(1 / 3) and e2["missing"] == pytest.approx(1 / 3)


def test_nearest_baseline_and_frame_difference():
    from paper_1812_06856_amd.experiments import frame_difference, nearest_baseline

    views = line_rig(4, 0.25, 100.0, 8, 8)
    assert nearest_baseline(views, 0) == pytest.approx(0.25)
    assert nearest_baseline(views, 2) == pytest.approx(0.25)
    a = np.array([[2.0, 4.0, 0.0, 5.0]])
    b = np.array([[2.0, 5.0, 3.0, 5.0]])
    static = np.array([[True, True, True, False]])
    assert frame_difference(a, b, static) == pytest.approx((0.0 + 0.2) / 2)
    assert frame_difference(a, a, static) == 0.0
