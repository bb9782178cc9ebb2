"""Named synthetic workloads.

1  tiny:      3 cameras on a line (baseline 0.1), f = 200, 160x120, background +
              3 tilted rectangles, SLIC grid 20x15, 64 levels on [2, 8], 3 iterations.
2  full HD:   8 toed-in cameras on an arc (radius 5, chord 1.5), f = 2400,
              1920x1080, background + 20 rectangles of which 6 low-texture,
              grid 103x58, 256 levels on [1.9, 8.6] (camera z of the scene spans 2.0-8.56 on the arc), 8 iterations.
3  precision: 4x4 planar grid (spacing 0.05), f = 1600, 1280x720, the full-HD
              scene recipe, grid 84x47, 192 levels on [2, 8], 6 iterations.
4  batched:   32 independent rigs; rig j (seed 400 + j) has U{3..16} views on
              a ceil(sqrt n)-column planar grid (spacing 0.1), resolution
              U{640x480, 1280x720, 1920x1080}, f = 200 W / 160, the tiny scene
              recipe, ~350 px per superpixel, U{128..256} levels, 3 iterations.
5  serving:   6 rigs drawn as in 4 (seeds 500 + j) whose rectangles move by up
              to 0.02 units per frame.

The paper's datasets are not available; these seeded scenes stand in for them
with the view counts, resolutions, level counts and superpixel sizes of the
paper's experiments.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, asdict, field
from typing import List

import numpy as np

from . import rig as rigmod
from .scene import build_rig, grid_for, make_scene, move_scene, scene_velocities


@dataclass
class MethodParams:
    levels: int = 64
    d_min: float = 2.0
    d_max: float = 8.0
    seed: int = 0x5EED
    jitter: int = 1
    tssd_T: float = 0.04          # truncation, squared colour distance in [0,1]^3 units
    sigma: float = 0.05           # depth Gaussian (scene units)
    alpha: float = 0.1            # colour Gaussian ([0,1] RGB units)
    eta: float = 0.5
    occ_tol: float = 1e-3         # relative tolerance of the visible/occluded split
    kernel_step: int = 5
    kernel_radius_init: int = 0   # <= 0: floor(min(W, H) / (2 S))
    term_mask: int = 7            # bit0 smoothness, bit1 consistency, bit2 occlusion
    energy_mode: int = 0          # 0 = E_c * E_s, 1 = data-only (negated normalised TSSD)
    iterations: int = 3

    def as_dict(self):
        return asdict(self)


@dataclass
class Workload:
    name: str
    rig: rigmod.Rig
    params: MethodParams


def config1(seed: int = 1) -> Workload:
    W, H, f = 160, 120, 200.0
    views = rigmod.line_rig(3, 0.1, f, W, H)
    rng = np.random.Generator(np.random.PCG64(seed))
    scene = make_scene(rng, f=f, W=W, H=H, sp_px=64.0, n_rect=3)
    rig = build_rig(views, scene, 20, 15, name="tiny-3x160x120", seed=seed)
    return Workload("tiny-3x160x120", rig, MethodParams(levels=64, d_min=2.0, d_max=8.0, iterations=3))


def config2(seed: int = 2, labels: str = "slic") -> Workload:
    W, H, f = 1920, 1080, 2400.0
    views = rigmod.arc_rig(8, 5.0, 1.5, f, W, H)
    rng = np.random.Generator(np.random.PCG64(seed))
    scene = make_scene(rng, f=f, W=W, H=H, sp_px=347.0, n_rect=20, n_low=6)
    rig = build_rig(views, scene, 103, 58, name="fullhd-8arc-1920x1080", seed=seed, labels=labels)
    return Workload("fullhd-8arc-1920x1080", rig,
                    MethodParams(levels=256, d_min=1.9, d_max=8.6, iterations=8))


def config3(seed: int = 3) -> Workload:
    W, H, f = 1280, 720, 1600.0
    views = rigmod.grid_rig(4, 4, 0.05, f, W, H)
    rng = np.random.Generator(np.random.PCG64(seed))
    scene = make_scene(rng, f=f, W=W, H=H, sp_px=233.0, n_rect=20, n_low=6)
    rig = build_rig(views, scene, 84, 47, name="precision-4x4-1280x720", seed=seed)
    return Workload("precision-4x4-1280x720", rig,
                    MethodParams(levels=192, d_min=2.0, d_max=8.0, iterations=6))


RESOLUTIONS = [(640, 480), (1280, 720), (1920, 1080)]


def rig_batched(j: int, base_seed: int = 400, max_res: int = 3, max_views: int = 16) -> Workload:
    rng = np.random.Generator(np.random.PCG64(base_seed + j))
    n = int(rng.integers(3, max_views + 1))
    W, H = RESOLUTIONS[int(rng.integers(0, max_res))]
    levels = int(rng.integers(128, 257))
    f = 200.0 * W / 160.0
    cols = int(math.ceil(math.sqrt(n)))
    rows = int(math.ceil(n / cols))
    views = rigmod.grid_rig(rows, cols, 0.1, f, W, H, n=n)
    scene = make_scene(rng, f=f, W=W, H=H, sp_px=350.0, n_rect=3)
    gw, gh = grid_for(W, H, 350.0)
    name = "rig%d-%dx%dx%d" % (j, n, W, H)
    rig = build_rig(views, scene, gw, gh, name=name, seed=base_seed + j)
    return Workload(name, rig, MethodParams(levels=levels, d_min=2.0, d_max=8.0, iterations=3))


def tiny_custom(W: int, H: int, gw: int, gh: int, *, n_views: int = 3, baseline: float = 0.1,
                f: float = 200.0, seed: int = 7, levels: int = 32, n_rect: int = 3,
                labels: str = "slic", iterations: int = 2) -> Workload:
    """Small line-rig workload with arbitrary (possibly ragged) sizes, for parity tests."""
    views = rigmod.line_rig(n_views, baseline, f, W, H)
    rng = np.random.Generator(np.random.PCG64(seed))
    scene = make_scene(rng, f=f, W=W, H=H, sp_px=W * H / (gw * gh), n_rect=n_rect)
    rig = build_rig(views, scene, gw, gh, name="custom-%dx%dx%d" % (n_views, W, H), seed=seed, labels=labels)
    return Workload(rig.name, rig, MethodParams(levels=levels, iterations=iterations))


def sensitivity_rig(sp_px: float = 100.0, seed: int = 21, W: int = 450, H: int = 375, n_views: int = 9,
                    levels: int = 80) -> Workload:
    """A Middlebury-like workload for parameter sweeps: 9 rectified views on a
    line (spacing 0.05, f = 400), 450x375, the tiny scene recipe with 5
    rectangles (occlusions), superpixels of about sp_px pixels, 80 levels on
    [2, 8].  The rendering depends on the seed only, so rigs with other
    superpixel sizes see the same images."""
    f = 400.0
    views = rigmod.line_rig(n_views, 0.05, f, W, H)
    rng = np.random.Generator(np.random.PCG64(seed))
    scene = make_scene(rng, f=f, W=W, H=H, sp_px=100.0, n_rect=5)
    gw, gh = grid_for(W, H, sp_px)
    name = "sens-%dx%dx%d-sp%d" % (n_views, W, H, int(round(sp_px)))
    rig = build_rig(views, scene, gw, gh, name=name, seed=seed)
    return Workload(name, rig, MethodParams(levels=levels, d_min=2.0, d_max=8.0, iterations=5))


class Sequence:
    """Frames of a static rig filming a moving scene (the serving workload)."""

    def __init__(self, name, views, scene, vel, gw, gh, params, seed):
        self.name, self.views, self.scene, self.vel = name, views, scene, vel
        self.gw, self.gh, self.params, self.seed = gw, gh, params, seed
        self._cache = {}

    def frame(self, k: int) -> rigmod.Rig:
        if k not in self._cache:
            views = [rigmod.View(K=v.K, R=v.R, t=v.t, W=v.W, H=v.H) for v in self.views]
            self._cache[k] = build_rig(views, move_scene(self.scene, self.vel, k), self.gw, self.gh,
                                       name="%s@%d" % (self.name, k), seed=self.seed)
        return self._cache[k]


def serving_rig(j: int, base_seed: int = 500, max_res: int = 3, max_views: int = 16,
                image_precision: int = 1) -> Sequence:
    """Rig j of the serving workload: drawn as in the batched recipe (views,
    resolution, levels) with 0.05 grid spacing and FP16 texels; every
    rectangle moves by U[-0.02, 0.02]^3 per frame, reflecting in depth
    within [2.5, 7.5]."""
    rng = np.random.Generator(np.random.PCG64(base_seed + j))
    n = int(rng.integers(3, max_views + 1))
    W, H = RESOLUTIONS[int(rng.integers(0, max_res))]
    levels = int(rng.integers(128, 257))
    f = 200.0 * W / 160.0
    cols = int(math.ceil(math.sqrt(n)))
    rows = int(math.ceil(n / cols))
    views = rigmod.grid_rig(rows, cols, 0.05, f, W, H, n=n)
    scene = make_scene(rng, f=f, W=W, H=H, sp_px=350.0, n_rect=3)
    vel = scene_velocities(rng, scene)
    gw, gh = grid_for(W, H, 350.0)
    params = MethodParams(levels=levels, d_min=2.0, d_max=8.0, iterations=3)
    return Sequence("serve%d-%dx%dx%d" % (j, n, W, H), views, scene, vel, gw, gh, params, base_seed + j)


def tiny_sequence(seed: int = 11, W: int = 160, H: int = 120, gw: int = 20, gh: int = 15, n_views: int = 3,
                  levels: int = 32, vmax: float = 0.02) -> Sequence:
    """Small moving-scene sequence on a line rig, for tests."""
    rng = np.random.Generator(np.random.PCG64(seed))
    views = rigmod.line_rig(n_views, 0.1, 200.0, W, H)
    scene = make_scene(rng, f=200.0, W=W, H=H, sp_px=W * H / (gw * gh), n_rect=3)
    vel = scene_velocities(rng, scene, vmax)
    return Sequence("tinyseq-%dx%dx%d" % (n_views, W, H), views, scene, vel, gw, gh,
                    MethodParams(levels=levels, iterations=2), seed)


def by_name(name: str) -> Workload:
    return {"1": config1, "2": config2, "3": config3}[str(name)]()
