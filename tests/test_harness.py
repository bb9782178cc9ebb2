"""Self-tests of the seeded input generators (no method arithmetic involved)."""
from __future__ import annotations

import hashlib

import numpy as np

from lfsynth import config1, tiny_custom, random_planes
from lfsynth.rig import arc_rig, grid_rig, line_rig


def _digest(w):
    h = hashlib.sha256()
    for v in w.rig.views:
        h.update(v.rgb.tobytes())
        h.update(v.labels.tobytes())
        h.update(v.gt_depth.tobytes())
    return h.hexdigest()


def test_generation_is_reproducible():
    assert _digest(config1()) == _digest(config1())
    assert _digest(config1(seed=1)) != _digest(config1(seed=9))


def test_background_depth_matches_its_plane():
    w = config1()
    for v in w.rig.views:
        bg = v.gt_plane == 0
        assert bg.any()
        assert np.allclose(v.gt_depth[bg], 8.0, rtol=1e-12)
        assert np.all(v.gt_depth[~bg] < 8.0 + 1e-9)
        assert np.all(v.gt_depth[v.gt_plane >= 0] >= 2.0 - 1e-9)


def test_rect_depth_is_ray_plane_intersection():
    w = config1()
    scene = w.rig.scene
    for v in w.rig.views:
        C = v.centre
        Kinv = np.linalg.inv(v.K)
        for j in range(1, scene["rects"].shape[0]):
            ys, xs = np.nonzero(v.gt_plane == j)
            if len(xs) == 0:
                continue
            row = scene["rects"][j]
            P0, n = row[0:3], row[9:12]
            rays_c = Kinv @ np.stack([xs, ys, np.ones_like(xs)])
            rays_w = v.R.T @ rays_c
            th = (n @ (P0 - C)) / (n @ rays_w)
            assert np.allclose(v.gt_depth[ys, xs], th, rtol=1e-10)


def test_slic_labels_keep_seed_grid_ids():
    w = config1()
    for v in w.rig.views:
        assert v.labels.min() >= 0 and v.labels.max() < v.gw * v.gh
        sx, sy = v.W / v.gw, v.H / v.gh
        for k in np.unique(v.labels):
            ys, xs = np.nonzero(v.labels == k)
            gx, gy = k % v.gw, k // v.gw
            assert abs(xs.mean() - (gx + 0.5) * sx) < 1.5 * sx
            assert abs(ys.mean() - (gy + 0.5) * sy) < 1.5 * sy


def test_slic_components_are_connected():
    w = tiny_custom(61, 47, 7, 5, seed=3)
    for v in w.rig.views:
        lab = v.labels
        for k in np.unique(lab):
            m = lab == k
            seen = np.zeros_like(m)
            ys, xs = np.nonzero(m)
            stack = [(ys[0], xs[0])]
            seen[ys[0], xs[0]] = True
            while stack:
                y, x = stack.pop()
                for dy, dx in ((0, 1), (0, -1), (1, 0), (-1, 0)):
                    yy, xx = y + dy, x + dx
                    if 0 <= yy < lab.shape[0] and 0 <= xx < lab.shape[1] and m[yy, xx] and not seen[yy, xx]:
                        seen[yy, xx] = True
                        stack.append((yy, xx))
            assert seen.sum() == m.sum()


def test_arc_rig_cameras_look_at_the_arc_centre():
    views = arc_rig(8, 5.0, 1.5, 2400.0, 1920, 1080)
    cs = np.stack([v.centre for v in views])
    assert np.allclose(np.linalg.norm(cs - [0, 0, 5.0], axis=1), 5.0)
    assert np.isclose(np.linalg.norm(cs[0] - cs[-1]), 1.5)
    for v in views:
        d = v.R @ (np.array([0, 0, 5.0]) - v.centre)
        assert np.allclose(d[:2], 0, atol=1e-12) and d[2] > 0
        assert np.allclose(v.R @ v.R.T, np.eye(3), atol=1e-14)


def test_grid_and_line_rigs():
    g = grid_rig(4, 4, 0.05, 1600.0, 1280, 720)
    cs = np.stack([v.centre for v in g])
    assert cs.shape == (16, 3) and np.allclose(cs[:, 2], 0)
    assert np.isclose(cs[:, 0].max() - cs[:, 0].min(), 0.15)
    l = line_rig(3, 0.1, 200.0, 160, 120)
    assert np.allclose([v.centre[0] for v in l], [-0.1, 0, 0.1])


def test_random_planes_face_the_camera():
    rng = np.random.default_rng(0)
    P = random_planes(rng, 20, 15, 2.0, 8.0)
    assert P.shape == (300, 4)
    assert np.all((P[:, 0] >= 2.0 - 1e-12) & (P[:, 0] <= 8.0 + 1e-12))
    assert np.allclose(np.linalg.norm(P[:, 1:], axis=1), 1.0)
    assert np.all(P[:, 3] >= np.cos(np.radians(40)) - 1e-12)
