"""Seeded synthetic light-field inputs (camera rigs, planar scenes, SLIC labels).

This package generates inputs only and holds none of the depth method's
arithmetic; the FP64 oracle and the HIP library both consume its output.
"""
from .rig import Rig, View, intrinsics, line_rig, grid_rig, arc_rig, pose_from_centre  # noqa: F401
from .configs import MethodParams, Workload, config1, config2, config3, rig_batched, tiny_custom  # noqa: F401
from .states import random_planes  # noqa: F401
