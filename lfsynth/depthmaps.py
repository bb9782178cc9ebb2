"""Seeded depth-map sets for the depth fusion: the rig's ground-truth depth
maps (ray cast, camera z, 0 where no surface) with relative Gaussian noise,
a fraction of outlier pixels whose depth is scaled by U[0.5, 1.5], and a
fraction of holes (depth 0), all drawn per view from numpy's PCG64.  These
stand in for the refined depth maps of a real light field; they hold none of
the fusion's arithmetic.
"""
from __future__ import annotations

from typing import List

import numpy as np


def noisy_depth_maps(rig, seed: int, noise: float = 0.002, outlier_frac: float = 0.02,
                     hole_frac: float = 0.01) -> List[np.ndarray]:
    out = []
    for v, view in enumerate(rig.views):
        rng = np.random.Generator(np.random.PCG64((seed << 8) + v))
        d = np.asarray(view.gt_depth, np.float64).copy()
        d *= 1.0 + rng.normal(0.0, noise, size=d.shape)
        out_mask = rng.uniform(size=d.shape) < outlier_frac
        d[out_mask] *= rng.uniform(0.5, 1.5, size=int(out_mask.sum()))
        d[rng.uniform(size=d.shape) < hole_frac] = 0.0
        out.append(np.ascontiguousarray(d.astype(np.float32)))
    return out
