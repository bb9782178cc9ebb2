"""ctypes wrapper of the FP64 CPU oracle (slfo).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The oracle shares no code with the
HIP library and never loads it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "slfo.c"), os.path.join(_HERE, "slfo_fuse.c"), os.path.join(_HERE, "slfo_slic.c")]
_OUT_DIR = os.path.join(_HERE, "_build")
_LIB = os.path.join(_OUT_DIR, "libslfo.so")
_lib = None


def build(verbose: bool = False) -> str:
    os.makedirs(_OUT_DIR, exist_ok=True)
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           "-Wall", "-Wextra", "-Wno-unused-parameter", *_SRCS, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("d_min", ctypes.c_double), ("d_max", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("jitter", ctypes.c_int32), ("tssd_T", ctypes.c_double),
                ("sigma", ctypes.c_double), ("alpha", ctypes.c_double), ("eta", ctypes.c_double),
                ("occ_tol", ctypes.c_double), ("kernel_step", ctypes.c_int32),
                ("kernel_radius_init", ctypes.c_int32), ("term_mask", ctypes.c_uint32),
                ("energy_mode", ctypes.c_int32)]


class _Rig(ctypes.Structure):
    _fields_ = [("n_views", ctypes.c_int32)] + [(n, ctypes.c_void_p) for n in (
        "width", "height", "grid_w", "grid_h", "K", "R", "t", "rgb", "labels", "pix_off", "nbr_off", "nbr")]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        L.slfo_create.argtypes = [ctypes.POINTER(_Rig), ctypes.POINTER(_Params), ctypes.POINTER(ctypes.c_int)]
        L.slfo_create.restype = P
        L.slfo_destroy.argtypes = [P]
        L.slfo_destroy.restype = None
        L.slfo_set_params.argtypes = [P, ctypes.POINTER(_Params)]
        L.slfo_set_threads.argtypes = [I]
        L.slfo_set_threads.restype = None
        L.slfo_sp_offset.argtypes = [P, I]
        L.slfo_sp_offset.restype = ctypes.c_int64
        L.slfo_sp_total.argtypes = [P]
        L.slfo_sp_total.restype = ctypes.c_int64
        L.slfo_sp_stats.argtypes = [P, P, P, P]
        L.slfo_mix64.argtypes = [ctypes.c_uint64]
        L.slfo_mix64.restype = ctypes.c_uint64
        L.slfo_level_q.argtypes = [P, I, I, I]
        L.slfo_level_q.restype = D
        L.slfo_kernel_radius.argtypes = [P, I, I]
        L.slfo_homography.argtypes = [P, I, I, P, D, P]
        L.slfo_sweep_cost_plane.argtypes = [P, I, I, P]
        L.slfo_sweep_cost_plane.restype = D
        L.slfo_sweep_sp.argtypes = [P, I, I, P, P, P, P]
        L.slfo_sweep_all.argtypes = [P, P, P, P, P]
        L.slfo_energy.argtypes = [P, P, I, I, P]
        L.slfo_energy.restype = D
        L.slfo_energy_flip_bound.argtypes = [P, P, I, I, P, D, D]
        L.slfo_energy_flip_bound.restype = D
        L.slfo_refine_sp.argtypes = [P, P, I, I, I, P, P, P, P]
        L.slfo_refine_all.argtypes = [P, P, I, P, P, P, P]
        L.slfo_refine_trace.argtypes = [P, P, I, I, I, P, P, P, I]
        L.slfo_refine_pivot.argtypes = [P, P, I, I, I, I, P, P, P, P, P, P, I]
        L.slfo_render_depth.argtypes = [P, P, I, P]
        L.slfo_slic_weight.argtypes = [I, I, I, I, D]
        L.slfo_slic_weight.restype = ctypes.c_float
        L.slfo_slic_centres_init.argtypes = [I, I, P, I, I, P]
        L.slfo_slic_assign.argtypes = [I, I, P, I, I, P, D, P]
        L.slfo_slic_update.argtypes = [I, I, P, I, I, P, P]
        L.slfo_slic_connectivity.argtypes = [I, I, I, I, P]
        L.slfo_slic.argtypes = [I, I, P, I, I, I, D, I, P]
        L.slfo_fuse_project.argtypes = [I, P, P, P, P, P, I, I, P]
        L.slfo_fuse_vote.argtypes = [I, P, ctypes.c_float, P]
        L.slfo_fuse_view.argtypes = [I, P, P, P, P, P, I, ctypes.c_float, P, P, P, P]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def mix64(z: int) -> int:
    return int(lib().slfo_mix64(ctypes.c_uint64(z & 0xFFFFFFFFFFFFFFFF)))


def set_threads(n: int) -> None:
    lib().slfo_set_threads(int(n))


def make_params(mp) -> _Params:
    g = mp if isinstance(mp, dict) else mp.as_dict()
    return _Params(int(g["levels"]), float(g["d_min"]), float(g["d_max"]), int(g["seed"]) & (2**64 - 1),
                   int(g["jitter"]), float(g["tssd_T"]), float(g["sigma"]), float(g["alpha"]), float(g["eta"]),
                   float(g["occ_tol"]), int(g["kernel_step"]), int(g["kernel_radius_init"]),
                   int(g["term_mask"]), int(g["energy_mode"]))


def warm_start_planes(Kinv, cen_prev, area_prev, A_prev, cen_new, area_new, d_min, d_max):
    """Serving warm start (not in the paper, which treats frames independently):
    the initial state of a new frame of a static rig from the previous frame's
    state, cell by cell.

    Kinv [S, 3, 3] inverse intrinsics of each cell's view; cen_* [S, 2]
    centroids; area_* [S]; A_prev [S, 4] planes (d, n).  A cell that is
    non-empty in both frames keeps its 3D plane n . X = delta, delta =
    d_prev (n . K^-1 (c_prev, 1)), and takes the depth where the ray of its new
    centroid meets that plane, d = delta / (n . K^-1 (c_new, 1)), if positive.
    Otherwise (empty before, or no positive depth) it starts fronto-parallel at
    d = 2 / (1/d_min + 1/d_max).  Cells empty now hold zeros."""
    S = len(area_new)
    out = np.zeros((S, 4))
    d_fb = 2.0 / (1.0 / d_min + 1.0 / d_max)
    for g in range(S):
        if area_new[g] == 0:
            continue
        d_prev = A_prev[g, 0]
        n = np.asarray(A_prev[g, 1:4], np.float64)
        if area_prev[g] > 0 and d_prev > 0:
            ray_prev = Kinv[g] @ np.array([cen_prev[g, 0], cen_prev[g, 1], 1.0])
            ray_new = Kinv[g] @ np.array([cen_new[g, 0], cen_new[g, 1], 1.0])
            delta = d_prev * float(n @ ray_prev)
            t = float(n @ ray_new)
            if t != 0.0 and delta / t > 0.0:
                out[g] = [delta / t, n[0], n[1], n[2]]
                continue
        out[g] = [d_fb, 0.0, 0.0, 1.0]
    return out


class FusionCams:
    """Cameras of a rig for the fusion oracle (Sec. III-D): any sequence of views
    with W, H, K (3x3), R (3x3), t (3)."""

    def __init__(self, views):
        self.V = len(views)
        self.wh = np.ascontiguousarray([[int(v.W), int(v.H)] for v in views], np.int32)
        self.K = np.ascontiguousarray(np.stack([np.asarray(v.K, np.float64).reshape(9) for v in views]))
        self.R = np.ascontiguousarray(np.stack([np.asarray(v.R, np.float64).reshape(9) for v in views]))
        self.t = np.ascontiguousarray(np.stack([np.asarray(v.t, np.float64).reshape(3) for v in views]))

    def _depth(self, depths):
        if len(depths) != self.V:
            raise ValueError("need one depth map per view")
        for v, d in enumerate(depths):
            if np.shape(d) != (self.wh[v, 1], self.wh[v, 0]):
                raise ValueError("depth map %d has shape %s" % (v, np.shape(d)))
        return np.ascontiguousarray(np.concatenate([np.asarray(d, np.float32).reshape(-1) for d in depths]))

    def project(self, depths, ref, src):
        """Pass 1: candidate depths of view `src` at the pixels of view `ref` (0 = none)."""
        D = self._depth(depths)
        W, H = self.wh[ref]
        out = np.empty((H, W), np.float32)
        if lib().slfo_fuse_project(self.V, _p(self.wh), _p(self.K), _p(self.R), _p(self.t), _p(D), ref, src,
                                   _p(out)):
            raise ValueError("bad views")
        return out

    def fuse(self, depths, ref, tau):
        """Both passes for view `ref`: (fused, winner view, winner stability, candidate count)."""
        D = self._depth(depths)
        W, H = self.wh[ref]
        fused = np.empty((H, W), np.float32)
        win = np.empty((H, W), np.int32)
        stab = np.empty((H, W), np.int32)
        nc = np.empty((H, W), np.int32)
        if lib().slfo_fuse_view(self.V, _p(self.wh), _p(self.K), _p(self.R), _p(self.t), _p(D), ref,
                                float(tau), _p(fused), _p(win), _p(stab), _p(nc)):
            raise ValueError("bad arguments")
        return fused, win, stab, nc


def fuse_vote(cands, tau):
    """Pass 2 on one pixel: (winner index or -1, stability per candidate)."""
    c = np.ascontiguousarray(cands, np.float32)
    s = np.empty(len(c), np.int32)
    b = lib().slfo_fuse_vote(len(c), _p(c), ctypes.c_float(tau), _p(s))
    return int(b), s


def slic(rgb, gw, gh, iterations=10, compactness=20.0, connectivity=True):
    """Grid-seeded SLIC labels [H, W] int32 (see oracle/slfo_slic.c)."""
    rgb = np.ascontiguousarray(rgb, np.uint8)
    H, W, _ = rgb.shape
    out = np.empty((H, W), np.int32)
    rc = lib().slfo_slic(W, H, _p(rgb), gw, gh, iterations, float(compactness), int(bool(connectivity)), _p(out))
    if rc:
        raise ValueError("slfo_slic failed: %d" % rc)
    return out


def slic_centres_init(rgb, gw, gh):
    rgb = np.ascontiguousarray(rgb, np.uint8)
    H, W, _ = rgb.shape
    cen = np.empty((gw * gh, 5), np.float32)
    if lib().slfo_slic_centres_init(W, H, _p(rgb), gw, gh, _p(cen)):
        raise ValueError("bad arguments")
    return cen


def slic_assign(rgb, gw, gh, cen, compactness=20.0):
    rgb = np.ascontiguousarray(rgb, np.uint8)
    H, W, _ = rgb.shape
    cen = np.ascontiguousarray(cen, np.float32)
    out = np.empty((H, W), np.int32)
    if lib().slfo_slic_assign(W, H, _p(rgb), gw, gh, _p(cen), float(compactness), _p(out)):
        raise ValueError("bad arguments")
    return out


def slic_update(rgb, gw, gh, labels, cen):
    rgb = np.ascontiguousarray(rgb, np.uint8)
    H, W, _ = rgb.shape
    labels = np.ascontiguousarray(labels, np.int32)
    cen = np.array(cen, np.float32, copy=True)
    rc = lib().slfo_slic_update(W, H, _p(rgb), gw, gh, _p(labels), _p(cen))
    if rc:
        raise ValueError("slfo_slic_update failed: %d" % rc)
    return cen


def slic_connectivity(labels, gw, gh):
    lab = np.array(labels, np.int32, copy=True)
    H, W = lab.shape
    if lib().slfo_slic_connectivity(W, H, gw, gh, _p(lab)):
        raise ValueError("slfo_slic_connectivity failed")
    return lab


class Oracle:
    """FP64 oracle bound to one rig.  Planes are float64 arrays [S_total, 4] = (d, nx, ny, nz)."""

    def __init__(self, rig, params):
        self._L = lib()
        views = rig.views
        V = len(views)
        self.V = V
        self._keep = []
        W = np.array([v.W for v in views], np.int32)
        H = np.array([v.H for v in views], np.int32)
        gw = np.array([v.gw for v in views], np.int32)
        gh = np.array([v.gh for v in views], np.int32)
        K = np.ascontiguousarray(np.stack([np.asarray(v.K, np.float64).reshape(9) for v in views]))
        R = np.ascontiguousarray(np.stack([np.asarray(v.R, np.float64).reshape(9) for v in views]))
        t = np.ascontiguousarray(np.stack([np.asarray(v.t, np.float64).reshape(3) for v in views]))
        rgb = np.ascontiguousarray(np.concatenate([np.asarray(v.rgb, np.uint8).reshape(-1) for v in views]))
        labels = np.ascontiguousarray(np.concatenate([np.asarray(v.labels, np.int32).reshape(-1) for v in views]))
        pix_off = np.zeros(V + 1, np.int64)
        pix_off[1:] = np.cumsum(W.astype(np.int64) * H)
        nl = rig.neighbor_lists()
        nbr_off = np.zeros(V + 1, np.int32)
        nbr_off[1:] = np.cumsum([len(n) for n in nl])
        nbr = np.array([x for n in nl for x in n] or [0], np.int32)
        self._keep = [W, H, gw, gh, K, R, t, rgb, labels, pix_off, nbr_off, nbr]
        self._rig = _Rig(V, *[_p(a) for a in self._keep])
        self._params = make_params(params)
        err = ctypes.c_int(0)
        self._c = self._L.slfo_create(ctypes.byref(self._rig), ctypes.byref(self._params), ctypes.byref(err))
        if not self._c:
            raise ValueError("slfo_create failed: %d" % err.value)
        self.S = int(self._L.slfo_sp_total(self._c))
        self.sp_off = np.array([self._L.slfo_sp_offset(self._c, v) for v in range(V)] + [self.S], np.int64)
        self.dims = [(int(v.W), int(v.H)) for v in views]

    def __del__(self):
        c = getattr(self, "_c", None)
        if c:
            self._L.slfo_destroy(c)
            self._c = None

    def set_params(self, params):
        self._params = make_params(params)
        rc = self._L.slfo_set_params(self._c, ctypes.byref(self._params))
        if rc:
            raise ValueError("bad params")

    # -- statistics
    def sp_stats(self):
        area = np.empty(self.S, np.int32)
        cen = np.empty((self.S, 2))
        col = np.empty((self.S, 3))
        self._L.slfo_sp_stats(self._c, _p(area), _p(cen), _p(col))
        return area, cen, col

    def level_q(self, view, sp, k):
        return float(self._L.slfo_level_q(self._c, view, sp, k))

    def kernel_radius(self, view, it):
        return int(self._L.slfo_kernel_radius(self._c, view, it))

    def homography(self, r, i, n, delta):
        n = np.ascontiguousarray(n, np.float64)
        H = np.empty(9)
        if self._L.slfo_homography(self._c, r, i, _p(n), float(delta), _p(H)):
            raise ValueError("bad views")
        return H.reshape(3, 3)

    # -- sweep
    def sweep_cost(self, view, sp, plane):
        pl = np.ascontiguousarray(plane, np.float64)
        return float(self._L.slfo_sweep_cost_plane(self._c, view, sp, _p(pl)))

    def sweep_sp(self, view, sp):
        pl = np.empty(4)
        cost = ctypes.c_double()
        ch = ctypes.c_int32()
        mg = ctypes.c_double()
        if self._L.slfo_sweep_sp(self._c, view, sp, _p(pl), ctypes.byref(cost), ctypes.byref(ch), ctypes.byref(mg)):
            raise ValueError("bad superpixel")
        return pl, cost.value, ch.value, mg.value

    def sweep(self):
        planes = np.empty((self.S, 4))
        cost = np.empty(self.S)
        ch = np.empty(self.S, np.int32)
        mg = np.empty(self.S)
        if self._L.slfo_sweep_all(self._c, _p(planes), _p(cost), _p(ch), _p(mg)):
            raise RuntimeError("sweep failed")
        return planes, cost, ch, mg

    # -- refinement
    def energy(self, A, view, sp, plane):
        A = np.ascontiguousarray(A, np.float64)
        pl = np.ascontiguousarray(plane, np.float64)
        return float(self._L.slfo_energy(self._c, _p(A), view, sp, _p(pl)))

    def energy_flip_bound(self, A, view, sp, plane, eps_px=1e-4, eps_rel=1e-5):
        """Upper bound of the energy change from flipping sample decisions that
        lie within eps_px / eps_rel of their thresholds (parity instrument)."""
        A = np.ascontiguousarray(A, np.float64)
        pl = np.ascontiguousarray(plane, np.float64)
        return float(self._L.slfo_energy_flip_bound(self._c, _p(A), view, sp, _p(pl), eps_px, eps_rel))

    def refine_sp(self, A, it, view, sp):
        A = np.ascontiguousarray(A, np.float64)
        pl = np.empty(4)
        e = ctypes.c_double()
        ch = ctypes.c_int32()
        mg = ctypes.c_double()
        if self._L.slfo_refine_sp(self._c, _p(A), it, view, sp, _p(pl), ctypes.byref(e), ctypes.byref(ch),
                                  ctypes.byref(mg)):
            raise ValueError("bad superpixel")
        return pl, e.value, ch.value, mg.value

    def refine(self, A, it):
        A = np.ascontiguousarray(A, np.float64)
        B = np.empty((self.S, 4))
        e = np.empty(self.S)
        ch = np.empty(self.S, np.int32)
        mg = np.empty(self.S)
        if self._L.slfo_refine_all(self._c, _p(A), it, _p(B), _p(e), _p(ch), _p(mg)):
            raise RuntimeError("refine failed")
        return B, e, ch, mg

    def refine_trace(self, A, it, view, sp, cap=256):
        A = np.ascontiguousarray(A, np.float64)
        slots = np.empty(cap, np.int32)
        planes = np.empty((cap, 4))
        en = np.empty(cap)
        n = self._L.slfo_refine_trace(self._c, _p(A), it, view, sp, _p(slots), _p(planes), _p(en), cap)
        if n < 0:
            raise ValueError("bad superpixel")
        return slots[:n], planes[:n], en[:n]

    def refine_pivot(self, A, it, view, sp, pivot_slot, cap=1024):
        """Refinement of one superpixel with the propagation stage resolved toward
        pivot_slot.  Returns (plane, energy, choice, trace_slots, trace_planes, trace_energies)."""
        A = np.ascontiguousarray(A, np.float64)
        pl = np.empty(4)
        e = ctypes.c_double()
        ch = ctypes.c_int32()
        slots = np.empty(cap, np.int32)
        planes = np.empty((cap, 4))
        en = np.empty(cap)
        n = self._L.slfo_refine_pivot(self._c, _p(A), it, view, sp, pivot_slot, _p(pl), ctypes.byref(e),
                                      ctypes.byref(ch), _p(slots), _p(planes), _p(en), cap)
        if n < 0:
            raise ValueError("bad pivot or superpixel (%d)" % n)
        return pl, e.value, ch.value, slots[:n], planes[:n], en[:n]

    def render_depth(self, planes, view):
        """Depth map of `view` from the full plane state [S_total, 4] (all views)."""
        planes = np.ascontiguousarray(planes, np.float64)
        if planes.shape != (self.S, 4):
            raise ValueError("render_depth needs the state of every view, shape (%d, 4)" % self.S)
        W, H = self.dims[view]
        out = np.empty((H, W))
        self._L.slfo_render_depth(self._c, _p(planes), view, _p(out))
        return out

    def warm_start(self, prev: "Oracle", A_prev):
        """Initial state of this rig's frame from `prev` (the same cameras and
        grids, the previous frame) and its state A_prev; see warm_start_planes."""
        area0, cen0, _ = prev.sp_stats()
        area1, cen1, _ = self.sp_stats()
        K = self._keep[4].reshape(-1, 3, 3)
        Kinv = np.concatenate([np.repeat(np.linalg.inv(K[v])[None], int(self.sp_off[v + 1] - self.sp_off[v]), 0)
                               for v in range(self.V)])
        p = self._params
        return warm_start_planes(Kinv, cen0, area0, np.asarray(A_prev, np.float64), cen1, area1, p.d_min, p.d_max)

    # -- convenience
    def view_slice(self, view):
        return slice(int(self.sp_off[view]), int(self.sp_off[view + 1]))

    def run(self, iterations):
        """Sweep then `iterations` refinement steps; returns the list of states and outputs."""
        A, cost, ch, mg = self.sweep()
        hist = [(A, cost, ch, mg)]
        for it in range(1, iterations + 1):
            B, e, c2, m2 = self.refine(A, it)
            hist.append((B, e, c2, m2))
            A = B
        return hist
