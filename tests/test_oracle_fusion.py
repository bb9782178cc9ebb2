"""Pins of the oracle's stability-based depth fusion (Sec. III-D; two passes per
reference view, Sec. III-E).

Pass 1 projects every other view's depth map into the reference viewport
(nearest pixel, closest point kept); pass 2 scores each candidate by the
candidates that agree with it minus those that do not and keeps the closest
candidate with non-negative stability.  The expected values here are counted
by hand (vote lists), follow from rectified geometry with integer disparities
(exact), or come from ray-plane intersections computed with numpy from the
camera definition (never from the oracle's projection).
"""
from __future__ import annotations

import math

import numpy as np
import pytest

from lfsynth.rig import arc_rig, grid_rig, line_rig
from oracle.oracle import FusionCams, fuse_vote


# ---------------------------------------------------------------- pass 2 on hand-made candidate lists

@pytest.mark.parametrize("cands, tau, winner, stab", [
    # a lone outlier is rejected; the three agreeing candidates have 2 - 1 = 1
    ([5.0, 5.01, 5.02, 2.0], 0.01, 0, [1, 1, 1, -3]),
    # the near pair is outvoted (1 - 3 = -2), the far triple is kept (2 - 2 = 0)
    ([6.0, 6.0, 6.0, 3.0, 3.0], 0.01, 0, [0, 0, 0, -2, -2]),
    ([3.0, 3.0, 6.0, 6.0, 6.0], 0.01, 2, [-2, -2, 0, 0, 0]),
    # three near, two far: the closest with stability >= 0 wins (2 - 2 = 0)
    ([6.0, 6.0, 3.0, 3.0, 3.0], 0.01, 2, [-2, -2, 0, 0, 0]),
    # equal depths: the smaller index
    ([4.0, 4.0], 0.01, 0, [1, 1]),
    # zeros are no candidates and neither vote nor win
    ([0.0, 4.0, 0.0], 0.01, 1, [0, 0, 0]),
    ([0.0, 0.0], 0.01, -1, [0, 0]),
    # one candidate: stability 0, kept
    ([7.5], 0.01, 0, [0]),
    # the bound is inclusive and relative to the candidate being scored
    ([1.0, 1.5], 0.5, 0, [1, 1]),
    ([1.0, 1.5], 0.25, -1, [-1, -1]),
    ([1.0, 1.5], 0.4, 1, [-1, 1]),
])
def test_votes_counted_by_hand(cands, tau, winner, stab):
    b, s = fuse_vote(cands, tau)
    assert b == winner
    assert s.tolist() == stab


def test_vote_tolerance_is_taken_against_the_scored_candidate():
    """1.0, 1.0099, 1.0201 at tau = 0.01: the middle one agrees with both ends
    only from their side (0.0102 <= 0.010201 from 1.0201, but 0.0102 > 0.010099
    from 1.0099), so every stability is 0 and the closest, 1.0, wins."""
    b, s = fuse_vote([1.0201, 1.0099, 1.0], 0.01)
    assert s.tolist() == [0, 0, 0]
    assert b == 2


# ---------------------------------------------------------------- pass 1 on rectified rigs

def _rectified(n, W=40, H=12, f=100.0, baseline=0.1):
    return line_rig(n, baseline, f, W, H)


@pytest.mark.parametrize("ref", [0, 1, 3])
def test_fronto_parallel_plane_shifts_by_integer_disparity(ref):
    """Cameras on the x axis with equal intrinsics, a plane at depth 2.5: view
    i's pixel (u, v) lands on (u + f (b_i - b_ref) / z, v) = (u + 4 (i - ref),
    v) of the reference with depth exactly 2.5.  So the reference pixel u holds
    a candidate of view i iff 0 <= u - 4 (i - ref) < W, every candidate equals
    2.5 and agrees with every other: stability = count - 1 and the fused depth
    is unchanged."""
    n, W, H = 4, 40, 12
    views = _rectified(n, W, H)
    cams = FusionCams(views)
    depths = [np.full((H, W), 2.5, np.float32) for _ in range(n)]
    u = np.arange(W)
    for i in range(n):
        if i == ref:
            continue
        cand = cams.project(depths, ref, i)
        covered = (u - 4 * (i - ref) >= 0) & (u - 4 * (i - ref) < W)
        exp = np.where(covered, np.float32(2.5), np.float32(0.0))
        assert np.array_equal(cand, np.broadcast_to(exp, (H, W)))
    fused, win, stab, nc = cams.fuse(depths, ref, 0.01)
    cnt = sum(((u - 4 * (i - ref) >= 0) & (u - 4 * (i - ref) < W)).astype(int) for i in range(n))
    assert np.array_equal(nc, np.broadcast_to(cnt, (H, W)))
    assert np.array_equal(stab, nc - 1)
    assert np.all(fused == np.float32(2.5))
    # the winner is the smallest view index holding a candidate
    first = np.array([min(i for i in range(n) if 0 <= x - 4 * (i - ref) < W) for x in u])
    assert np.array_equal(win, np.broadcast_to(first, (H, W)))


def test_depth_test_keeps_the_closest_point():
    """f b = 20 between views 0 and 1 (b = 0.2): view 1's pixel 0 at depth 2
    and pixel 5 at depth 4 both land on reference column 10 (disparities 10
    and 5); the candidate there is 2.  A lone point at depth 4 elsewhere lands
    5 columns on."""
    W, H = 30, 3
    views = line_rig(2, 0.2, 100.0, W, H)
    cams = FusionCams(views)
    d1 = np.zeros((H, W), np.float32)
    d1[1, 0] = 2.0
    d1[1, 5] = 4.0
    d1[2, 12] = 4.0
    cand = cams.project([np.zeros((H, W), np.float32), d1], 0, 1)
    exp = np.zeros((H, W), np.float32)
    exp[1, 10] = 2.0
    exp[2, 17] = 4.0
    assert np.array_equal(cand, exp)
    # and in the other direction the shift is negative
    d0 = np.zeros((H, W), np.float32)
    d0[0, 20] = 4.0
    cand = cams.project([d0, np.zeros((H, W), np.float32)], 1, 0)
    exp = np.zeros((H, W), np.float32)
    exp[0, 15] = 4.0
    assert np.array_equal(cand, exp)


def test_vertical_baseline_shifts_rows():
    """A 2 x 1 grid rig (cameras stacked along y): the shift is along rows, with
    the sign of the camera offset; an exchange of u and v or of the pose signs
    fails here."""
    W, H = 16, 30
    views = grid_rig(2, 1, 0.1, 100.0, W, H)
    cams = FusionCams(views)
    d = [np.full((H, W), 2.5, np.float32) for _ in range(2)]
    cand = cams.project(d, 0, 1)          # view 1 sits 0.1 below view 0 (y down): v -> v + 4
    vv = np.arange(H)[:, None]
    exp = np.where((vv - 4 >= 0), np.float32(2.5), np.float32(0.0))
    assert np.array_equal(cand, np.broadcast_to(exp, (H, W)))


def test_points_behind_the_reference_or_outside_are_dropped():
    """A point behind the reference camera or projecting outside its image
    gives no candidate; depths <= 0, NaN and inf are no points."""
    W, H = 20, 10
    views = line_rig(2, 5.0, 100.0, W, H)       # baseline 5 at depth 2.5: disparity 200 px, all outside
    cams = FusionCams(views)
    d = [np.full((H, W), 2.5, np.float32), np.full((H, W), 2.5, np.float32)]
    assert not cams.project(d, 0, 1).any()
    views = line_rig(2, 0.1, 100.0, W, H)
    cams = FusionCams(views)
    d1 = np.full((H, W), 2.5, np.float32)
    d1[:, :5] = [-1.0, 0.0, np.nan, np.inf, -np.inf]
    cand = cams.project([np.zeros((H, W), np.float32), d1], 0, 1)
    assert not cand[:, 4:9].any()            # columns 0..4 of view 1 land on 4..8
    assert np.all(cand[:, 9:] == np.float32(2.5))
    # a camera looking away: the rotated view sees the points behind it
    R = np.diag([-1.0, 1.0, -1.0])
    views[1].R, views[1].t = R, np.zeros(3)
    cams = FusionCams(views)
    assert not cams.project([np.full((H, W), 2.5, np.float32)] * 2, 1, 0).any()


# ---------------------------------------------------------------- pass 1 on a toed-in rig against ray-plane geometry

def _plane_depth(view, n, delta):
    """Depth map of the world plane n . X = delta seen by `view`, by intersecting
    each pixel ray C + lam R^T K^-1 (u, v, 1) (camera z of the ray point is lam)."""
    H, W = view.H, view.W
    u, v = np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64))
    rays_c = np.linalg.solve(view.K, np.stack([u.ravel(), v.ravel(), np.ones(u.size)]))
    rays_w = view.R.T @ rays_c
    C = -view.R.T @ view.t
    lam = (delta - n @ C) / (n @ rays_w)
    return lam.reshape(H, W)


@pytest.mark.parametrize("ref", [0, 2])
def test_toed_in_rig_candidates_lie_on_the_plane(ref):
    """An arc of 4 toed-in cameras and one slanted world plane.  A candidate of
    view i at reference pixel p is the camera-r depth of a point of the plane
    whose projection rounds to p, so it differs from the plane's depth along
    p's own ray by at most the depth gradient over half a pixel diagonal; the
    reference's plane depth comes from a ray-plane intersection.  Most pixels
    are covered, and a transposed rotation or a wrong pose sign is off by far
    more than the bound."""
    W, H = 64, 48
    views = arc_rig(4, 5.0, 1.5, 60.0, W, H)
    n = np.array([0.2, -0.15, -1.0])
    n /= np.linalg.norm(n)
    delta = float(n @ np.array([0.0, 0.0, 4.0]))
    depths = [_plane_depth(v, n, delta).astype(np.float32) for v in views]
    assert all(np.all(d > 0) for d in depths)
    Dr = depths[ref].astype(np.float64)
    gy, gx = np.gradient(Dr)
    bound = (np.abs(gx) + np.abs(gy)) * 0.5 * 1.05 + 1e-5 * Dr
    cams = FusionCams(views)
    for i in range(4):
        if i == ref:
            continue
        cand = cams.project(depths, ref, i).astype(np.float64)
        hit = cand > 0
        assert hit.mean() > 0.6
        err = np.abs(cand - Dr)[hit]
        assert np.all(err <= bound[hit]), (err.max(), bound[hit].max())
    fused, win, stab, nc = cams.fuse(depths, ref, 0.01)
    assert np.all(nc >= 1)
    # every candidate agrees at tau = 1 %: stability = count - 1, fused = a candidate <= own depth
    assert np.array_equal(stab, nc - 1)
    assert np.all(fused <= depths[ref])
    assert np.all(np.abs(fused.astype(np.float64) - Dr) <= bound)


def test_outliers_are_removed_by_the_vote():
    """Five rectified views of a plane at depth 2.5.  A block of the
    reference's own depth map set to 1.25 (a near outlier) is outvoted by the
    four other views and replaced by 2.5; a block of one source view set to
    1.0 lands elsewhere and is outvoted where it lands.  Where only the
    reference sees the scene its depth is kept."""
    n, W, H = 5, 60, 10
    views = _rectified(n, W, H)
    cams = FusionCams(views)
    d = [np.full((H, W), 2.5, np.float32) for _ in range(n)]
    ref = 2
    d[ref][3:6, 28:32] = 1.25
    d[0][:, 30:34] = 1.0           # disparity 10 per spacing at z = 1: lands on 30 + 10 * (0 - 2) = 10..13
    fused, win, stab, nc = cams.fuse(d, ref, 0.01)
    # the block: views 0, 1, 3, 4 agree (3 - 1 = 2); the winner is view 0's candidate
    assert np.all(fused[3:6, 28:32] == np.float32(2.5))
    assert np.all(stab[3:6, 28:32] == 2) and np.all(win[3:6, 28:32] == 0)
    # view 0's near block lands on columns 10..13 (z = 1: 10 px per spacing), where it is closer
    # than view 0's own points at 2.5 and is kept by the depth test, then outvoted
    assert np.all(win[:, 10:14] == 1) and np.all(stab[:, 10:14] == 2)
    assert np.all(fused == np.float32(2.5))


def test_disagreeing_pair_without_majority_has_no_depth():
    """Two views of which each sees a different depth at a pixel: each
    candidate has stability -1, so the pixel gets no depth (0)."""
    W, H = 8, 2
    views = line_rig(2, 0.1, 100.0, W, H)
    cams = FusionCams(views)
    d0 = np.full((H, W), 2.5, np.float32)
    d1 = np.zeros((H, W), np.float32)
    d1[0, 0] = 5.0          # disparity 2 at z = 5: lands on reference column 2 (view 1 sits at +0.1: u -> u + 2)
    fused, win, stab, nc = cams.fuse([d0, d1], 0, 0.01)
    assert nc[0, 2] == 2 and fused[0, 2] == 0.0 and win[0, 2] == -1
    assert fused[1, 2] == np.float32(2.5) and stab[1, 2] == 0


def test_third_view_siding_with_the_farther_depth_decides():
    """Three views; at reference column 6 the reference sees 2.5 and views 1
    and 2 see 5.0 (disparities 2 and 4 at z = 5): the closer candidate has
    stability -2, the farther ones 0, so the farther depth is kept (view 1's
    candidate, the smaller index)."""
    W, H = 10, 1
    views = line_rig(3, 0.1, 100.0, W, H)
    cams = FusionCams(views)
    d0 = np.full((H, W), 2.5, np.float32)
    d1 = np.zeros((H, W), np.float32)
    d2 = np.zeros((H, W), np.float32)
    d1[0, 4] = 5.0
    d2[0, 2] = 5.0
    fused, win, stab, nc = cams.fuse([d0, d1, d2], 0, 0.01)
    assert nc[0, 6] == 3 and fused[0, 6] == np.float32(5.0) and win[0, 6] == 1 and stab[0, 6] == 0
    assert np.all(np.delete(fused[0], 6) == np.float32(2.5))
