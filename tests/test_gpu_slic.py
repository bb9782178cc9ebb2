"""GPU SLIC (slf_segment) against the oracle's SLIC: the labels are integer
decisions taken in FP32 from exactly represented inputs in the same order of
operations on both sides, so they must be identical on every pixel."""
from __future__ import annotations

import numpy as np
import pytest

from lfsynth import config1, tiny_custom
from lfsynth.configs import config2
from oracle import oracle

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _ctx_with_images(rig):
    from paper_1812_06856_amd import slf

    ctx = slf.Context(0)
    vs = rig.views
    ctx.set_cameras([(v.W, v.H) for v in vs], [v.K for v in vs], [v.R for v in vs], [v.t for v in vs])
    for i, v in enumerate(vs):
        ctx.set_image(i, v.rgb)
    return ctx


def _compare(rig, gw, gh, iterations, compactness, views=None, what=""):
    ctx = _ctx_with_images(rig)
    views = range(rig.n_views) if views is None else views
    for v in views:
        ctx.segment(v, gw, gh, iterations, compactness)
        got = ctx.get_labels(v)
        exp = oracle.slic(rig.views[v].rgb, gw, gh, iterations, compactness)
        bad = np.argwhere(got != exp)
        _say("%s view %d %dx%d grid %dx%d m=%g: %d labels, %d pixels differ" % (
            what, v, rig.views[v].W, rig.views[v].H, gw, gh, compactness, len(np.unique(exp)), len(bad)))
        assert len(bad) == 0, bad[:10]
    return ctx


def test_segment_tiny_views_match_oracle():
    _compare(config1().rig, 20, 15, 10, 20.0, what="tiny")


@pytest.mark.parametrize("W, H, gw, gh, m, iters", [(161, 117, 19, 13, 20.0, 10), (97, 61, 9, 7, 0.0, 4),
                                                     (200, 80, 17, 6, 40.0, 1), (64, 64, 1, 1, 10.0, 3)])
def test_segment_ragged_and_degenerate_grids_match_oracle(W, H, gw, gh, m, iters):
    rig = tiny_custom(W, H, max(1, gw), max(1, gh), seed=9, labels="grid").rig
    _compare(rig, gw, gh, iters, m, views=[0, 2], what="ragged")


def test_segment_fullsize_views_match_oracle():
    w = config2(labels="grid")
    _compare(w.rig, 103, 58, 10, 20.0, views=[0, 5], what="full HD")


def test_segmented_labels_drive_the_path_like_host_labels():
    """A rig whose labels come from slf_segment gives the same sweep and
    refinement, bit for bit, as the same labels given with slf_set_labels."""
    from paper_1812_06856_amd import slf

    w = config1()
    p = slf.params_from(w.params)
    a = _ctx_with_images(w.rig)
    a.set_params(p)
    b = _ctx_with_images(w.rig)
    b.set_params(p)
    for v in range(w.rig.n_views):
        a.segment(v, 20, 15, 10, 20.0)
        b.set_labels(v, oracle.slic(w.rig.views[v].rgb, 20, 15, 10, 20.0), 20, 15)
    for c in (a, b):
        c.sweep()
        c.propagate(1, 2)
    for v in range(w.rig.n_views):
        for x, y in zip(a.get_planes(v), b.get_planes(v)):
            assert np.array_equal(x.view(np.uint32) if x.dtype == np.float32 else x,
                                  y.view(np.uint32) if y.dtype == np.float32 else y)
        assert np.array_equal(a.get_depth(v), b.get_depth(v))


def test_segment_error_paths():
    from paper_1812_06856_amd import slf

    w = config1()
    ctx = slf.Context(0)
    vs = w.rig.views
    ctx.set_cameras([(v.W, v.H) for v in vs], [v.K for v in vs], [v.R for v in vs], [v.t for v in vs])
    with pytest.raises(slf.SlfError) as e:
        ctx.segment(0, 20, 15)          # no image yet
    assert e.value.status == slf.SLF_ESTATE
    with pytest.raises(slf.SlfError) as e:
        ctx.get_labels(0)
    assert e.value.status == slf.SLF_ESTATE
    ctx.set_image(0, vs[0].rgb)
    for bad in [(0, 15, 10, 20.0), (161, 15, 10, 20.0), (20, 121, 10, 20.0), (20, 15, 0, 20.0),
                (20, 15, 10, -1.0), (20, 15, 10, float("nan"))]:
        with pytest.raises(slf.SlfError) as e:
            ctx.segment(0, *bad)
        assert e.value.status == slf.SLF_EINVAL, bad
    with pytest.raises(slf.SlfError) as e:
        ctx.segment(7, 20, 15)
    assert e.value.status == slf.SLF_EINVAL
