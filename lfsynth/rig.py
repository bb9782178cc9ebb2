"""Camera rigs and the per-view input bundle.

Camera convention (shared by every consumer of these inputs): a world point
X maps to camera coordinates X_c = R X + t; the pixel is K X_c dehomogenised,
with K = [[f, 0, (W-1)/2], [0, f, (H-1)/2], [0, 0, 1]] and pixel centres at
integer (u, v), u = column, v = row.  Depth means camera-frame z.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


def intrinsics(f: float, W: int, H: int) -> np.ndarray:
    return np.array([[f, 0.0, (W - 1) / 2.0], [0.0, f, (H - 1) / 2.0], [0.0, 0.0, 1.0]])


def pose_from_centre(C, R=None):
    """(R, t) for a camera centred at world point C with rotation R (rows = camera axes)."""
    R = np.eye(3) if R is None else np.asarray(R, np.float64)
    C = np.asarray(C, np.float64)
    return R, -R @ C


@dataclass
class View:
    W: int
    H: int
    K: np.ndarray
    R: np.ndarray
    t: np.ndarray
    rgb: Optional[np.ndarray] = None        # (H, W, 3) uint8
    labels: Optional[np.ndarray] = None     # (H, W) int32, seed-grid ids
    gw: int = 0
    gh: int = 0
    gt_depth: Optional[np.ndarray] = None   # (H, W) float64 camera z, 0 = no hit
    gt_plane: Optional[np.ndarray] = None   # (H, W) int32 scene rectangle id

    @property
    def centre(self) -> np.ndarray:
        return -self.R.T @ self.t


@dataclass
class Rig:
    views: List[View]
    neighbors: Optional[List[List[int]]] = None   # None = all other views, ascending
    name: str = ""
    seed: int = 0
    scene: Optional[dict] = None

    @property
    def n_views(self) -> int:
        return len(self.views)

    def neighbor_lists(self) -> List[List[int]]:
        if self.neighbors is not None:
            return [list(n) for n in self.neighbors]
        V = self.n_views
        return [[i for i in range(V) if i != r] for r in range(V)]


def line_rig(n: int, baseline: float, f: float, W: int, H: int) -> List[View]:
    """n cameras on the x axis, centred on the origin, spacing `baseline`, R = I."""
    xs = (np.arange(n) - (n - 1) / 2.0) * baseline
    out = []
    for x in xs:
        R, t = pose_from_centre([x, 0.0, 0.0])
        out.append(View(W, H, intrinsics(f, W, H), R, t))
    return out


def grid_rig(rows: int, cols: int, spacing: float, f: float, W: int, H: int, n: Optional[int] = None) -> List[View]:
    """Planar rig in the z = 0 plane, R = I, row-major; first `n` positions of a rows x cols grid."""
    n = rows * cols if n is None else n
    out = []
    for k in range(n):
        r, c = divmod(k, cols)
        x = (c - (cols - 1) / 2.0) * spacing
        y = (r - (rows - 1) / 2.0) * spacing
        R, t = pose_from_centre([x, y, 0.0])
        out.append(View(W, H, intrinsics(f, W, H), R, t))
    return out


def arc_rig(n: int, radius: float, chord: float, f: float, W: int, H: int) -> List[View]:
    """n cameras on a horizontal arc of `radius` about (0, 0, radius), toed in to that point.

    The extreme cameras are `chord` apart; angles are evenly spaced.
    """
    phi_max = math.asin(chord / (2.0 * radius))
    out = []
    for k in range(n):
        phi = -phi_max + 2.0 * phi_max * k / (n - 1) if n > 1 else 0.0
        C = np.array([radius * math.sin(phi), 0.0, radius - radius * math.cos(phi)])
        R = np.array([[math.cos(phi), 0.0, math.sin(phi)],
                      [0.0, 1.0, 0.0],
                      [-math.sin(phi), 0.0, math.cos(phi)]])
        # rows of R are the camera axes in world coordinates; z axis points at (0, 0, radius)
        R, t = pose_from_centre(C, R)
        out.append(View(W, H, intrinsics(f, W, H), R, t))
    return out
