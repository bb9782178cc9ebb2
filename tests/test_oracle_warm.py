"""Pins of the oracle's serving warm start: each cell keeps its previous 3D
plane, read at its new centroid; fallbacks for cells without one."""
from __future__ import annotations

import numpy as np
import pytest

from oracle.oracle import Oracle, warm_start_planes

F, W, H = 200.0, 160, 120
K = np.array([[F, 0, (W - 1) / 2], [0, F, (H - 1) / 2], [0, 0, 1.0]])
KINV = np.linalg.inv(K)


def _unit(v):
    v = np.asarray(v, np.float64)
    return v / np.linalg.norm(v)


def _basis(n):
    a = np.array([1.0, 0, 0]) if abs(n[0]) < 0.9 else np.array([0, 1.0, 0])
    u = _unit(np.cross(n, a))
    return u, np.cross(n, u)


def test_warm_start_depth_is_where_the_new_ray_meets_the_previous_plane():
    rng = np.random.default_rng(5)
    S = 40
    A = np.zeros((S, 4))
    cen0 = rng.uniform([10, 10], [W - 10, H - 10], size=(S, 2))
    cen1 = cen0 + rng.uniform(-6, 6, size=(S, 2))
    for g in range(S):
        n = _unit([rng.uniform(-0.4, 0.4), rng.uniform(-0.4, 0.4), -1.0])
        n = -n if n @ (KINV @ [cen0[g, 0], cen0[g, 1], 1]) < 0 else n
        A[g] = [rng.uniform(2.5, 7.5), *n]
    area = np.full(S, 50)
    out = warm_start_planes(np.repeat(KINV[None], S, 0), cen0, area, A, cen1, area, 2.0, 8.0)
    for g in range(S):
        n = A[g, 1:]
        P0 = A[g, 0] * (KINV @ [cen0[g, 0], cen0[g, 1], 1.0])  # the previous centroid's 3D point
        u, v = _basis(n)
        ray = KINV @ [cen1[g, 0], cen1[g, 1], 1.0]
        lam, a, b = np.linalg.solve(np.stack([ray, -u, -v], 1), P0)  # lam ray = P0 + a u + b v
        assert out[g, 0] == pytest.approx(lam, rel=1e-12)
        assert np.array_equal(out[g, 1:], n)


def test_fronto_parallel_planes_keep_their_depth():
    rng = np.random.default_rng(6)
    S = 25
    A = np.zeros((S, 4))
    A[:, 0] = rng.uniform(2, 8, S)
    A[:, 3] = 1.0
    cen0 = rng.uniform(0, 120, size=(S, 2))
    cen1 = rng.uniform(0, 120, size=(S, 2))
    area = np.ones(S, int)
    out = warm_start_planes(np.repeat(KINV[None], S, 0), cen0, area, A, cen1, area, 2.0, 8.0)
    assert np.array_equal(out, A)


def test_fallbacks_and_empty_cells():
    d_fb = 2.0 / (1 / 2.0 + 1 / 8.0)  # 3.2
    Kinv = np.repeat(KINV[None], 4, 0)
    A = np.array([[4.0, 0, 0, 1.0],   # empty before -> fallback
                  [4.0, 0, 0, 1.0],   # empty now -> zeros
                  [4.0, *_unit([0.999, 0, 0.045])],  # nearly edge-on: behind the camera at the new centroid
                  [0.0, 0, 0, 0]])    # no previous plane -> fallback
    cen0 = np.array([[80.0, 60], [80, 60], [80.0, 60], [80, 60]])
    cen1 = np.array([[80.0, 60], [80, 60], [20.0, 60], [80, 60]])
    area0 = np.array([0, 10, 10, 10])
    area1 = np.array([10, 0, 10, 10])
    r0 = KINV @ [80.0, 60, 1]
    r1 = KINV @ [20.0, 60, 1]
    n2 = A[2, 1:]
    assert n2 @ r0 > 0 and (A[2, 0] * (n2 @ r0)) / (n2 @ r1) < 0  # the case really has no positive depth
    out = warm_start_planes(Kinv, cen0, area0, A, cen1, area1, 2.0, 8.0)
    assert np.array_equal(out[0], [d_fb, 0, 0, 1])
    assert np.array_equal(out[1], [0, 0, 0, 0])
    assert np.array_equal(out[2], [d_fb, 0, 0, 1])
    assert np.array_equal(out[3], [d_fb, 0, 0, 1])


def test_oracle_warm_start_on_two_frames_keeps_every_cell_on_its_plane():
    from lfsynth import configs, states

    seq = configs.tiny_sequence(seed=21)
    r0, r1 = seq.frame(0), seq.frame(1)
    o0 = Oracle(r0, seq.params)
    o1 = Oracle(r1, seq.params)
    rng = np.random.default_rng(3)
    A = np.concatenate([states.random_planes(rng, v.gw, v.gh, 2.0, 8.0, max_tilt_deg=30) for v in r0.views])
    area0, cen0, _ = o0.sp_stats()
    area1, cen1, _ = o1.sp_stats()
    A[area0 == 0] = 0
    out = o1.warm_start(o0, A)
    assert not np.array_equal(cen0[area1 > 0], cen1[area1 > 0])  # the frames differ
    kept = 0
    for v in range(o1.V):
        Kinv = np.linalg.inv(np.asarray(r1.views[v].K, np.float64))
        for g in range(int(o1.sp_off[v]), int(o1.sp_off[v + 1])):
            if area1[g] == 0:
                assert not out[g].any()
                continue
            if area0[g] == 0 or not np.array_equal(out[g, 1:], A[g, 1:]):
                assert np.array_equal(out[g], [3.2, 0, 0, 1])
                continue
            kept += 1
            n = A[g, 1:]
            X0 = A[g, 0] * (Kinv @ [cen0[g, 0], cen0[g, 1], 1])
            X1 = out[g, 0] * (Kinv @ [cen1[g, 0], cen1[g, 1], 1])
            assert n @ X1 == pytest.approx(n @ X0, rel=1e-12)
    assert kept > 0.9 * int((area1 > 0).sum())
