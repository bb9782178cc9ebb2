"""The accuracy experiments (Fig. 5 / Fig. 6 analogues and the temporal
metric) run end to end on the GPU on small rigs; the values they report
keep the properties that hold at any size."""
from __future__ import annotations

import numpy as np
import pytest

from lfsynth import config1, configs, tiny_custom

pytestmark = pytest.mark.gpu


def test_refinement_history_scores_every_stage():
    from paper_1812_06856_amd import experiments

    hist = experiments.solve_with_history(config1(), 3)
    assert [h["iteration"] for h in hist] == [0, 1, 2, 3]
    for h in hist:
        assert 0.0 <= h["bad_1"] <= h["bad_0.5"] <= 1.0 and h["stage_ms"] > 0
    assert all(b["total_ms"] > a["total_ms"] for a, b in zip(hist, hist[1:]))
    print("bad pixels (1 px) after the sweep %.4f, after 3 iterations %.4f; mean relative error %.4g -> %.4g" % (
        hist[0]["bad_1"], hist[-1]["bad_1"], hist[0]["mare"], hist[-1]["mare"]))
    # the tiny scene's sweep is already fine (0.12 px of disparity per level), so no ordering is asserted


def test_sensitivity_runner_small():
    from paper_1812_06856_amd import experiments

    def make(sp):
        g = max(2, int(round(160 / np.sqrt(sp))))
        return tiny_custom(160, 120, g, max(2, int(round(g * 0.75))), seed=5, levels=24, iterations=2)

    out = experiments.sensitivity(make, sp_sizes=(64, 144), kernel_steps=(2, 5), kernel_radii=(3, 0), iterations=2)
    assert len(out["vs_iterations"]) == 9
    assert [r["superpixel_px"] for r in out["vs_superpixel_size"]] == [64, 144]
    assert len(out["energy_terms"]) == 5
    for group in ("vs_superpixel_size", "vs_kernel_step", "vs_kernel_radius", "energy_terms"):
        for r in out[group]:
            assert 0.0 <= r["bad_1"] <= 1.0 and r["total_ms"] > 0


def test_temporal_metric_is_zero_for_a_still_scene():
    """A still scene (no motion): every frame's cold solve is identical, so its
    flicker is exactly 0; the serving form reports finite values."""
    from paper_1812_06856_amd import experiments

    seq = configs.tiny_sequence(seed=71, vmax=0.0)
    out = experiments.temporal_consistency(seq, 3)
    assert out["cold"]["flicker"] == [0.0, 0.0]
    assert all(s == 1.0 for s in out["static_frac"])
    assert all(np.isfinite(x) for x in out["warm"]["flicker"])
    moving = experiments.temporal_consistency(configs.tiny_sequence(seed=72), 3)
    assert all(0.0 <= s < 1.0 for s in moving["static_frac"])
    print("moving scene flicker: cold %.3g, warm %.3g" % (moving["cold"]["mean_flicker"], moving["warm"]["mean_flicker"]))
