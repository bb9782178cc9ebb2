"""Seeded planar scenes, rendered by ray casting, plus grid-seeded SLIC labels.

Scene recipe (all draws from numpy's PCG64 seeded per scene):

* background: a fronto-parallel textured plane at world z = `bg_z`, unbounded;
* `n_rect` foreground rectangles: centre depth ~ U[2.5, 7.5]; normal
  (0, 0, -1) rotated by theta_x, theta_y ~ U[-tilt, tilt]; width covering
  U[15 %, 45 %] of the central view's width at that depth (height likewise of
  its height); centre inside the central frustum; shrunk until every corner
  lies inside the depth band [2, 8];
* textures: two-octave value noise in [0, 255] (coarse lattice cell
  U[1, 2] superpixel widths at the rectangle's depth in the central view,
  fine cell ~2.5 px) or, for the `n_low` low-texture rectangles, a constant
  colour ~ U{40..215}^3 plus integer noise U{-2..2} per ~1 px texel.

Rendering is noise-free, Lambertian and without anti-aliasing: one ray per
pixel centre, nearest hit, colour rounded to uint8.
"""
from __future__ import annotations

import math
from typing import List, Optional

import numpy as np

from . import _native
from .rig import Rig, View

RECT_STRIDE = 20


def _rot(theta_x: float, theta_y: float) -> np.ndarray:
    cx, sx = math.cos(theta_x), math.sin(theta_x)
    cy, sy = math.cos(theta_y), math.sin(theta_y)
    Rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    Ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
    return Ry @ Rx


def make_scene(rng: np.random.Generator, *, f: float, W: int, H: int, sp_px: float, n_rect: int,
               n_low: int = 0, tilt_deg: float = 30.0, bg_z: float = 8.0,
               fronto: bool = False, depths: Optional[List[float]] = None) -> dict:
    """Rectangles (RECT_STRIDE doubles each; layout in csrc/synth.c) and texture seeds.

    Geometry is expressed for a virtual central camera at the origin looking
    down +z with focal length f and a W x H image.  `fronto=True` keeps every
    rectangle fronto-parallel (used by exact-sweep inputs); `depths` fixes the
    rectangles' centre depths instead of drawing them.
    """
    rects = []
    seeds = []
    low_ids = set(rng.choice(n_rect, size=n_low, replace=False).tolist()) if n_low else set()

    def texture(row, depth, low):
        if low:
            row[14] = 1.0
            row[15] = 1.0 * depth / f
            row[17:20] = rng.integers(40, 216, size=3)
        else:
            row[14] = 0.0
            row[15] = rng.uniform(1.0, 2.0) * sp_px * depth / f
            row[16] = 2.5 * depth / f

    # background
    bg = np.zeros(RECT_STRIDE)
    bg[0:3] = [0.0, 0.0, bg_z]
    bg[3:6] = [1.0, 0.0, 0.0]
    bg[6:9] = [0.0, 1.0, 0.0]
    bg[9:12] = [0.0, 0.0, 1.0]
    bg[12] = bg[13] = -1.0
    texture(bg, bg_z, False)
    rects.append(bg)
    seeds.append(int(rng.integers(0, 2**63)))

    for j in range(n_rect):
        z = rng.uniform(2.5, 7.5) if depths is None else float(depths[j])
        if fronto:
            R = np.eye(3)
        else:
            tmax = math.radians(tilt_deg)
            R = _rot(rng.uniform(-tmax, tmax), rng.uniform(-tmax, tmax))
        e1, e2, n = R[:, 0], R[:, 1], R[:, 2]
        hw = z * (W / 2.0) / f
        hh = z * (H / 2.0) / f
        h1 = rng.uniform(0.15, 0.45) * hw
        h2 = rng.uniform(0.15, 0.45) * hh * (W / H) * 0.75
        h2 = min(h2, 0.9 * hh)
        cxy = [rng.uniform(-0.8, 0.8) * hw, rng.uniform(-0.8, 0.8) * hh]
        P0 = np.array([cxy[0], cxy[1], z])
        # shrink until all corners stay inside the depth band [2, 8]
        for _ in range(60):
            zs = [(P0 + a * h1 * e1 + b * h2 * e2)[2] for a in (-1, 1) for b in (-1, 1)]
            if min(zs) >= 2.0 and max(zs) <= 8.0:
                break
            h1 *= 0.9
            h2 *= 0.9
        row = np.zeros(RECT_STRIDE)
        row[0:3] = P0
        row[3:6] = e1
        row[6:9] = e2
        row[9:12] = np.cross(e1, e2)
        row[12], row[13] = h1, h2
        texture(row, z, j in low_ids)
        rects.append(row)
        seeds.append(int(rng.integers(0, 2**63)))
    return {"rects": np.stack(rects), "tex_seeds": np.array(seeds, np.uint64),
            "n_low": n_low, "n_rect": n_rect}


def scene_velocities(rng: np.random.Generator, scene: dict, vmax: float = 0.02) -> np.ndarray:
    """Per-frame velocity of every rectangle centre, U[-vmax, vmax]^3; the background stays."""
    v = rng.uniform(-vmax, vmax, size=(scene["rects"].shape[0], 3))
    v[0] = 0.0
    return v


def move_scene(scene: dict, vel: np.ndarray, frame: int, z_lo: float = 2.5, z_hi: float = 7.5) -> dict:
    """The scene at `frame`: rectangle j's centre moved by frame * vel[j], its depth
    reflected back into [z_lo, z_hi] (a triangle wave); orientation, extent and
    texture move with it."""
    rects = scene["rects"].copy()
    span = z_hi - z_lo
    for j in range(1, rects.shape[0]):
        p = rects[j, 0:3] + frame * vel[j]
        u = (p[2] - z_lo) % (2.0 * span)
        p[2] = z_lo + (u if u <= span else 2.0 * span - u)
        rects[j, 0:3] = p
    out = dict(scene)
    out["rects"] = rects
    return out


def render_view(view: View, scene: dict) -> None:
    rgb, depth, pid = _native.raycast(view.W, view.H, view.K, view.R, view.t, scene["rects"], scene["tex_seeds"])
    view.rgb, view.gt_depth, view.gt_plane = rgb, depth, pid


def segment_view(view: View, gw: int, gh: int, iters: int = 10, compactness: float = 20.0) -> int:
    labels, empty = _native.slic(view.rgb, gw, gh, iters, compactness)
    view.labels, view.gw, view.gh = labels, gw, gh
    return empty


def grid_for(W: int, H: int, sp_px: float):
    """Seed grid with cells of about sp_px pixels."""
    S = math.sqrt(sp_px)
    return max(1, int(round(W / S))), max(1, int(round(H / S)))


def build_rig(views: List[View], scene: dict, gw: int, gh: int, *, name: str = "", seed: int = 0,
              labels: str = "slic") -> Rig:
    """Render every view and segment it.  labels='grid' uses the plain seed grid (no SLIC)."""
    for v in views:
        render_view(v, scene)
        if labels == "slic":
            segment_view(v, gw, gh)
        else:
            v.labels = grid_labels(v.W, v.H, gw, gh)
            v.gw, v.gh = gw, gh
    return Rig(views=views, name=name, seed=seed, scene=scene)


def grid_labels(W: int, H: int, gw: int, gh: int) -> np.ndarray:
    """Labels of a regular grid: pixel (u, v) -> cell (floor(u gw / W), floor(v gh / H))."""
    gx = (np.arange(W) * gw) // W
    gy = (np.arange(H) * gh) // H
    return (gy[:, None] * gw + gx[None, :]).astype(np.int32)
