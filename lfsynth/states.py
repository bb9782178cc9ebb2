"""Seeded plane states (d, nx, ny, nz) per grid cell, used as given refinement inputs.

Depth is a smooth random field over the seed grid (so neighbouring cells hold
similar depths, as after a sweep) plus per-cell jitter, uniform in inverse
depth over [1/d_max, 1/d_min].  Normals are (0, 0, 1) tilted by at most
`max_tilt_deg`; with tilt <= 40 degrees and a field of view below ~45 degrees
every such plane faces the camera at every pixel.
"""
from __future__ import annotations

import math

import numpy as np


def random_planes(rng: np.random.Generator, gw: int, gh: int, d_min: float, d_max: float,
                  max_tilt_deg: float = 40.0, frac_slanted: float = 0.5, smooth_cells: float = 4.0) -> np.ndarray:
    K = gw * gh
    # smooth field: bilinear upsampling of a coarse random lattice
    cw = max(2, int(math.ceil(gw / smooth_cells)) + 2)
    ch = max(2, int(math.ceil(gh / smooth_cells)) + 2)
    lat = rng.uniform(0.0, 1.0, size=(ch, cw))
    gx = np.arange(gw) / smooth_cells
    gy = np.arange(gh) / smooth_cells
    ix = np.minimum(np.floor(gx).astype(int), cw - 2)
    iy = np.minimum(np.floor(gy).astype(int), ch - 2)
    fx = gx - ix
    fy = gy - iy
    top = lat[iy][:, ix] * (1 - fx)[None, :] + lat[iy][:, ix + 1] * fx[None, :]
    bot = lat[iy + 1][:, ix] * (1 - fx)[None, :] + lat[iy + 1][:, ix + 1] * fx[None, :]
    field = top * (1 - fy)[:, None] + bot * fy[:, None]
    field = np.clip(field + rng.normal(0.0, 0.05, size=field.shape), 0.0, 1.0)
    q = 1.0 / d_max + field.reshape(K) * (1.0 / d_min - 1.0 / d_max)
    d = 1.0 / q
    tilt = np.radians(rng.uniform(0.0, max_tilt_deg, size=K)) * (rng.uniform(size=K) < frac_slanted)
    az = rng.uniform(0.0, 2 * math.pi, size=K)
    n = np.stack([np.sin(tilt) * np.cos(az), np.sin(tilt) * np.sin(az), np.cos(tilt)], axis=1)
    return np.concatenate([d[:, None], n], axis=1)
