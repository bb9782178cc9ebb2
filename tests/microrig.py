"""Hand-built tiny rigs for oracle pins (no scene generator involved)."""
from __future__ import annotations

import numpy as np

from lfsynth.rig import Rig, View, intrinsics, pose_from_centre
from lfsynth.configs import MethodParams
from lfsynth.scene import grid_labels


def view(W, H, f=100.0, centre=(0.0, 0.0, 0.0), R=None, rgb=None, labels=None, gw=1, gh=1):
    Rm, t = pose_from_centre(centre, R)
    v = View(W, H, intrinsics(f, W, H), Rm, t)
    v.rgb = np.zeros((H, W, 3), np.uint8) if rgb is None else np.ascontiguousarray(rgb, np.uint8)
    v.labels = grid_labels(W, H, gw, gh) if labels is None else np.ascontiguousarray(labels, np.int32)
    v.gw, v.gh = gw, gh
    return v


def block_rgb(W, H, gw, gh, colours):
    """Image whose grid cell k is filled with colours[k] (uint8 triples)."""
    lab = grid_labels(W, H, gw, gh)
    col = np.asarray(colours, np.uint8).reshape(gw * gh, 3)
    return col[lab]


def rig(views, neighbors=None):
    return Rig(views=list(views), neighbors=neighbors)


def params(**kw):
    p = MethodParams()
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def fronto_state(S, d):
    A = np.zeros((S, 4))
    A[:, 0] = d
    A[:, 3] = 1.0
    return A
