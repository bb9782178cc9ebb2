"""Loader for the harness's native helpers (ray caster, SLIC).

The shared object is built by :func:`build` (called from the repository's
build entry point) into ``lfsynth/_build/``.  Loading never compiles
implicitly unless the library is missing.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "synth.c")
_OUT_DIR = os.path.join(_HERE, "_build")
_LIB = os.path.join(_OUT_DIR, "libsynth.so")
_lib = None


def build(verbose: bool = False) -> str:
    os.makedirs(_OUT_DIR, exist_ok=True)
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", _SRC, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        L.synth_raycast.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, ctypes.c_int, P, P, P, P, P]
        L.synth_raycast.restype = None
        L.synth_slic.argtypes = [ctypes.c_int, ctypes.c_int, P, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_double, P]
        L.synth_slic.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def raycast(W, H, K, R, t, rects, tex_seeds):
    K = np.ascontiguousarray(K, np.float64)
    R = np.ascontiguousarray(R, np.float64)
    t = np.ascontiguousarray(t, np.float64)
    rects = np.ascontiguousarray(rects, np.float64)
    seeds = np.ascontiguousarray(tex_seeds, np.uint64)
    rgb = np.empty((H, W, 3), np.uint8)
    depth = np.empty((H, W), np.float64)
    pid = np.empty((H, W), np.int32)
    lib().synth_raycast(W, H, _p(K), _p(R), _p(t), rects.shape[0], _p(rects), _p(seeds),
                        _p(rgb), _p(depth), _p(pid))
    return rgb, depth, pid


def slic(rgb, gw, gh, iters=10, compactness=10.0):
    rgb = np.ascontiguousarray(rgb, np.uint8)
    H, W, _ = rgb.shape
    labels = np.empty((H, W), np.int32)
    empty = lib().synth_slic(W, H, _p(rgb), gw, gh, iters, float(compactness), _p(labels))
    return labels, int(empty)
