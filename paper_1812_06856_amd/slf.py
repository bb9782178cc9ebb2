"""Python binding of libslf (include/slf.h): argument marshalling only.

Every step of the depth path runs in the HIP library.  torch is imported
first so that the library binds to the HIP runtime torch already loaded (one
runtime per process); torch supplies device memory and streams only.  If the
built library is missing, loading fails loudly: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch  # noqa: F401  (must precede loading libslf: shared HIP runtime)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libslf.so")

SLF_OK, SLF_EINVAL, SLF_ESTATE, SLF_ENOMEM, SLF_EDEVICE, SLF_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
SLF_IMAGE_U8, SLF_IMAGE_F16, SLF_IMAGE_F32 = 0, 1, 2

EXPORTED = [
    "slf_default_params", "slf_create", "slf_destroy", "slf_set_stream", "slf_set_params", "slf_set_cameras",
    "slf_set_neighbors", "slf_set_image_rgb8", "slf_set_labels", "slf_prepare", "slf_sweep", "slf_set_planes", "slf_propagate",
    "slf_get_planes", "slf_get_depth", "slf_get_superpixels", "slf_get_work", "slf_get_sweep_work", "slf_get_sweep_levels", "slf_reset_work", "slf_synchronize",
    "slf_status_string", "slf_last_error", "slf_warm_start", "slf_get_footprint",
    "slf_fuse", "slf_get_fused_depth", "slf_fuse_depth", "slf_fuse_depth_static", "slf_segment", "slf_get_labels",
    "slf_pool_default_config", "slf_pool_create", "slf_pool_destroy", "slf_pool_set_stream", "slf_pool_set_config",
    "slf_pool_get_config", "slf_pool_attach", "slf_pool_detach", "slf_pool_usage", "slf_pool_submit", "slf_pool_step",
    "slf_pool_run", "slf_pool_poll", "slf_pool_synchronize", "slf_pool_autotune", "slf_pool_last_error",
]
SLF_POOL_SOLVE, SLF_POOL_PROPAGATE = 0, 1


class slf_params(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("levels", ctypes.c_int32), ("d_min", ctypes.c_double),
                ("d_max", ctypes.c_double), ("seed", ctypes.c_uint64), ("jitter", ctypes.c_int32),
                ("tssd_T", ctypes.c_float), ("sigma", ctypes.c_float), ("alpha", ctypes.c_float),
                ("eta", ctypes.c_float), ("occ_tol", ctypes.c_float), ("kernel_step", ctypes.c_int32),
                ("kernel_radius_init", ctypes.c_int32), ("term_mask", ctypes.c_uint32),
                ("image_precision", ctypes.c_int32), ("homography_fp64", ctypes.c_int32),
                ("energy_mode", ctypes.c_int32), ("exact_margin", ctypes.c_int32)]


class slf_pool_config(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("sweep_level_chunk", ctypes.c_int32),
                ("sweep_tile", ctypes.c_int32), ("refine_tile", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("sweep_level_split", ctypes.c_int32)]

    def as_dict(self):
        return {f[0]: getattr(self, f[0]) for f in self._fields_}


_lib = None


def load(path: str = LIB_PATH):
    """Loads libslf.so and declares the ABI; raises if the library was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libslf.so not found at %s: build it first (paper_1812_06856_amd/build.py)" % path)
    L = ctypes.CDLL(path)
    P, I, I64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
    L.slf_default_params.argtypes = [ctypes.POINTER(slf_params)]
    L.slf_default_params.restype = None
    L.slf_create.argtypes = [I, ctypes.POINTER(P)]
    L.slf_destroy.argtypes = [P]
    L.slf_set_stream.argtypes = [P, P]
    L.slf_set_params.argtypes = [P, ctypes.POINTER(slf_params)]
    L.slf_set_cameras.argtypes = [P, I, P, P, P, P]
    L.slf_set_neighbors.argtypes = [P, I, I, P]
    L.slf_set_image_rgb8.argtypes = [P, I, P, I64, I]
    L.slf_set_labels.argtypes = [P, I, P, I64, I, I, I]
    L.slf_prepare.argtypes = [P]
    L.slf_sweep.argtypes = [P]
    L.slf_set_planes.argtypes = [P, I, P]
    L.slf_propagate.argtypes = [P, I, I]
    L.slf_get_planes.argtypes = [P, I, P, P, P, P]
    L.slf_get_depth.argtypes = [P, I, P, I64, I]
    L.slf_get_superpixels.argtypes = [P, I, P, P, P]
    L.slf_get_work.argtypes = [P, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64),
                               ctypes.POINTER(ctypes.c_uint64)]
    L.slf_get_sweep_work.argtypes = [P, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)]
    L.slf_get_sweep_levels.argtypes = [P, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)]
    L.slf_reset_work.argtypes = [P]
    L.slf_synchronize.argtypes = [P]
    L.slf_status_string.argtypes = [I]
    L.slf_status_string.restype = ctypes.c_char_p
    L.slf_last_error.argtypes = [P]
    L.slf_last_error.restype = ctypes.c_char_p
    U64, PU64, PI = ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_int)
    L.slf_warm_start.argtypes = [P]
    L.slf_get_footprint.argtypes = [P, PU64]
    L.slf_fuse.argtypes = [P, ctypes.c_float]
    L.slf_segment.argtypes = [P, I, I, I, I, ctypes.c_float]
    L.slf_get_labels.argtypes = [P, I, P, I64, I]
    L.slf_get_fused_depth.argtypes = [P, I, P, I64, P, I]
    L.slf_fuse_depth.argtypes = [P, P, P, P, ctypes.c_float]
    L.slf_fuse_depth_static.argtypes = [P, P, P, P, ctypes.c_float]
    L.slf_pool_default_config.argtypes = [ctypes.POINTER(slf_pool_config)]
    L.slf_pool_default_config.restype = None
    L.slf_pool_create.argtypes = [I, U64, ctypes.POINTER(P)]
    L.slf_pool_destroy.argtypes = [P]
    L.slf_pool_set_stream.argtypes = [P, P]
    L.slf_pool_set_config.argtypes = [P, ctypes.POINTER(slf_pool_config)]
    L.slf_pool_get_config.argtypes = [P, ctypes.POINTER(slf_pool_config)]
    L.slf_pool_attach.argtypes = [P, P]
    L.slf_pool_detach.argtypes = [P, P]
    L.slf_pool_usage.argtypes = [P, PU64, PU64, PI, PI]
    L.slf_pool_submit.argtypes = [P, P, I, I, I, U64]
    L.slf_pool_step.argtypes = [P, PI]
    L.slf_pool_run.argtypes = [P]
    L.slf_pool_poll.argtypes = [P, P, I, PI]
    L.slf_pool_synchronize.argtypes = [P]
    L.slf_pool_autotune.argtypes = [P, PI]
    L.slf_pool_last_error.argtypes = [P]
    L.slf_pool_last_error.restype = ctypes.c_char_p
    for name in EXPORTED:
        getattr(L, name)  # every declared entry point must be exported
    _lib = L
    return L


class SlfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s (%d): %s" % (_status_name(status), status, msg))
        self.status = status


def _status_name(s):
    return {0: "SLF_OK", -1: "SLF_EINVAL", -2: "SLF_ESTATE", -3: "SLF_ENOMEM", -4: "SLF_EDEVICE",
            -5: "SLF_EUNSUPPORTED"}.get(s, "?")


def _ptr(a):
    if isinstance(a, torch.Tensor):
        return ctypes.c_void_p(a.data_ptr())
    return a.ctypes.data_as(ctypes.c_void_p)


def default_params(**overrides) -> slf_params:
    p = slf_params()
    load().slf_default_params(ctypes.byref(p))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def params_from(mp, **overrides) -> slf_params:
    """slf_params from any object/dict with the method parameter names."""
    g = mp if isinstance(mp, dict) else mp.as_dict()
    names = [f[0] for f in slf_params._fields_]
    kw = {k: g[k] for k in names if k in g}
    kw.update(overrides)
    return default_params(**kw)


class Context:
    """One slf context on a HIP device; methods mirror the C calls."""

    def __init__(self, device: int = 0):
        self._L = load()
        h = ctypes.c_void_p()
        self._check(self._L.slf_create(device, ctypes.byref(h)), ctx=None)
        self._h = h
        self.device = device
        self.dims = []
        self.grids = []
        self._pool = None

    def close(self):
        if getattr(self, "_h", None):
            if self._pool is not None:
                try:
                    self._pool.detach(self)
                except SlfError:  # stages not yet launched: finish them first
                    self._pool.run()
                    self._pool.synchronize()
                    self._pool.detach(self)
            self._L.slf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, ctx="self"):
        if rc != SLF_OK:
            msg = self._L.slf_last_error(self._h).decode() if ctx == "self" and self._h else ""
            raise SlfError(rc, msg)
        return rc

    def last_error(self) -> str:
        return self._L.slf_last_error(self._h).decode()

    # -- configuration
    def set_stream(self, stream) -> None:
        ptr = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream or 0)
        self._check(self._L.slf_set_stream(self._h, ctypes.c_void_p(ptr)))

    def set_params(self, p: slf_params) -> None:
        self._check(self._L.slf_set_params(self._h, ctypes.byref(p)))

    def set_cameras(self, wh, K, R, t) -> None:
        wh = np.ascontiguousarray(wh, np.int32).reshape(-1, 2)
        K = np.ascontiguousarray(K, np.float64).reshape(-1, 9)
        R = np.ascontiguousarray(R, np.float64).reshape(-1, 9)
        t = np.ascontiguousarray(t, np.float64).reshape(-1, 3)
        self._check(self._L.slf_set_cameras(self._h, wh.shape[0], _ptr(wh), _ptr(K), _ptr(R), _ptr(t)))
        self.dims = [tuple(x) for x in wh.tolist()]
        self.grids = [None] * wh.shape[0]

    def set_neighbors(self, view: int, views: Sequence[int]) -> None:
        a = np.ascontiguousarray(views, np.int32)
        self._check(self._L.slf_set_neighbors(self._h, view, a.size, _ptr(a)))

    def set_image(self, view: int, rgb) -> None:
        """rgb: (H, W, 3) uint8 numpy array (host) or torch uint8 tensor on the device."""
        if isinstance(rgb, torch.Tensor) and rgb.is_cuda:
            assert rgb.dtype == torch.uint8 and rgb.dim() == 3 and rgb.stride(2) == 1 and rgb.stride(1) == 3
            self._check(self._L.slf_set_image_rgb8(self._h, view, _ptr(rgb), rgb.stride(0), 1))
        else:
            a = np.ascontiguousarray(rgb, np.uint8)
            self._check(self._L.slf_set_image_rgb8(self._h, view, _ptr(a), a.strides[0], 0))

    def set_labels(self, view: int, labels, grid_w: int, grid_h: int) -> None:
        if isinstance(labels, torch.Tensor) and labels.is_cuda:
            assert labels.dtype == torch.int32 and labels.dim() == 2 and labels.stride(1) == 1
            self._check(self._L.slf_set_labels(self._h, view, _ptr(labels), labels.stride(0), grid_w, grid_h, 1))
        else:
            a = np.ascontiguousarray(labels, np.int32)
            self._check(self._L.slf_set_labels(self._h, view, _ptr(a), a.shape[1], grid_w, grid_h, 0))
        self.grids[view] = (grid_w, grid_h)

    def segment(self, view: int, grid_w: int, grid_h: int, iterations: int = 10, compactness: float = 20.0) -> None:
        """GPU SLIC of the view's image into the view's labels (slf_segment)."""
        self._check(self._L.slf_segment(self._h, view, grid_w, grid_h, iterations, float(compactness)))
        self.grids[view] = (grid_w, grid_h)

    def get_labels(self, view: int, out: Optional[torch.Tensor] = None):
        W, H = self.dims[view]
        if out is not None:
            assert out.is_cuda and out.dtype == torch.int32 and out.stride(1) == 1
            self._check(self._L.slf_get_labels(self._h, view, _ptr(out), out.stride(0), 1))
            return out
        a = np.empty((H, W), np.int32)
        self._check(self._L.slf_get_labels(self._h, view, _ptr(a), W, 0))
        return a

    def load_rig(self, rig, params=None) -> None:
        """Cameras, neighbour lists, images and labels of an input rig (host arrays)."""
        vs = rig.views
        self.set_cameras([(v.W, v.H) for v in vs], [v.K for v in vs], [v.R for v in vs], [v.t for v in vs])
        if params is not None:
            self.set_params(params)
        if rig.neighbors is not None:
            for r, nb in enumerate(rig.neighbor_lists()):
                self.set_neighbors(r, nb)
        for i, v in enumerate(vs):
            self.set_image(i, v.rgb)
            self.set_labels(i, v.labels, v.gw, v.gh)

    # -- the path
    def prepare(self) -> None:
        self._check(self._L.slf_prepare(self._h))

    def sweep(self) -> None:
        self._check(self._L.slf_sweep(self._h))

    def set_planes(self, view: int, planes) -> None:
        a = np.ascontiguousarray(planes, np.float32).reshape(-1, 4)
        self._check(self._L.slf_set_planes(self._h, view, _ptr(a)))

    def propagate(self, first_iter: int, n_iters: int) -> None:
        self._check(self._L.slf_propagate(self._h, first_iter, n_iters))

    def get_planes(self, view: int):
        gw, gh = self.grids[view]
        K = gw * gh
        planes = np.empty((K, 4), np.float32)
        e = np.empty(K, np.float32)
        ch = np.empty(K, np.int32)
        mg = np.empty(K, np.float32)
        self._check(self._L.slf_get_planes(self._h, view, _ptr(planes), _ptr(e), _ptr(ch), _ptr(mg)))
        return planes, e, ch, mg

    def get_depth(self, view: int, out: Optional[torch.Tensor] = None):
        W, H = self.dims[view]
        if out is not None:
            assert out.is_cuda and out.dtype == torch.float32 and out.stride(1) == 1
            self._check(self._L.slf_get_depth(self._h, view, _ptr(out), out.stride(0), 1))
            return out
        a = np.empty((H, W), np.float32)
        self._check(self._L.slf_get_depth(self._h, view, _ptr(a), W, 0))
        return a

    def get_superpixels(self, view: int):
        gw, gh = self.grids[view]
        K = gw * gh
        area = np.empty(K, np.int32)
        cen = np.empty((K, 2), np.float32)
        col = np.empty((K, 3), np.float32)
        self._check(self._L.slf_get_superpixels(self._h, view, _ptr(area), _ptr(cen), _ptr(col)))
        return area, cen, col

    def work(self):
        """(hypotheses decided, px-view samples computed)."""
        return self.work_detail()[:2]

    def sweep_work(self):
        """(sweep px-view samples computed, samples without the level bound)."""
        c, t = ctypes.c_uint64(), ctypes.c_uint64()
        self._check(self._L.slf_get_sweep_work(self._h, ctypes.byref(c), ctypes.byref(t)))
        return int(c.value), int(t.value)

    def sweep_levels(self):
        """(sweep levels scored in full, sweep levels decided)."""
        a, b = ctypes.c_uint64(), ctypes.c_uint64()
        self._check(self._L.slf_get_sweep_levels(self._h, ctypes.byref(a), ctypes.byref(b)))
        return int(a.value), int(b.value)

    def work_detail(self):
        """(hypotheses decided, px-view samples computed, refinement candidates pruned)."""
        e, s, pr = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        self._check(self._L.slf_get_work(self._h, ctypes.byref(e), ctypes.byref(s), ctypes.byref(pr)))
        return int(e.value), int(s.value), int(pr.value)

    def warm_start(self) -> None:
        self._check(self._L.slf_warm_start(self._h))

    def footprint(self) -> int:
        b = ctypes.c_uint64()
        self._check(self._L.slf_get_footprint(self._h, ctypes.byref(b)))
        return int(b.value)

    # -- depth fusion
    def fuse(self, agree_tol: float = 0.01) -> None:
        self._check(self._L.slf_fuse(self._h, float(agree_tol)))

    def get_fused_depth(self, view: int, out: Optional[torch.Tensor] = None, votes: Optional[torch.Tensor] = None):
        """Host: returns (fused [H, W] float32, votes [H, W] int32).  Device: fills
        the given tensors (row stride of `out`, or of `votes` if out is None)."""
        W, H = self.dims[view]
        if out is not None or votes is not None:
            ref = out if out is not None else votes
            for tsr in (out, votes):
                assert tsr is None or (tsr.is_cuda and tsr.stride(1) == 1 and tsr.stride(0) == ref.stride(0))
            self._check(self._L.slf_get_fused_depth(self._h, view, None if out is None else _ptr(out), ref.stride(0),
                                                    None if votes is None else _ptr(votes), 1))
            return out, votes
        a = np.empty((H, W), np.float32)
        v = np.empty((H, W), np.int32)
        self._check(self._L.slf_get_fused_depth(self._h, view, _ptr(a), W, _ptr(v), 0))
        return a, v

    def fuse_depth(self, depth: Sequence[torch.Tensor], fused: Sequence[torch.Tensor],
                   votes: Optional[Sequence[torch.Tensor]] = None, agree_tol: float = 0.01,
                   static_scratch: bool = False) -> None:
        """Fusion of caller depth maps: device float32 tensors [H_v, W_v] (contiguous) per view.
        static_scratch: slf_fuse_depth_static (no allocation; the library's fixed scratch)."""
        V = len(self.dims)
        assert len(depth) == V and len(fused) == V and (votes is None or len(votes) == V)
        for v in range(V):
            W, H = self.dims[v]
            for tsr, dt in ((depth[v], torch.float32), (fused[v], torch.float32)) + (
                    ((votes[v], torch.int32),) if votes is not None else ()):
                assert tsr.is_cuda and tsr.dtype == dt and tuple(tsr.shape) == (H, W) and tsr.is_contiguous()
        arr = lambda ts: (ctypes.c_void_p * V)(*[t.data_ptr() for t in ts])
        dv = arr(votes) if votes is not None else None
        fn = self._L.slf_fuse_depth_static if static_scratch else self._L.slf_fuse_depth
        self._check(fn(self._h, arr(depth), arr(fused), dv, float(agree_tol)))

    def reset_work(self) -> None:
        self._check(self._L.slf_reset_work(self._h))

    def synchronize(self) -> None:
        self._check(self._L.slf_synchronize(self._h))


def default_pool_config(**overrides) -> slf_pool_config:
    c = slf_pool_config()
    load().slf_pool_default_config(ctypes.byref(c))
    for k, v in overrides.items():
        if not hasattr(c, k):
            raise KeyError(k)
        setattr(c, k, v)
    return c


class Pool:
    """A rig pool (slf_pool_*): admission against an HBM budget, pooled
    persistent launches, graph replay and iteration-level batching."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self._L = load()
        h = ctypes.c_void_p()
        rc = self._L.slf_pool_create(device, hbm_budget_bytes, ctypes.byref(h))
        if rc != SLF_OK:
            raise SlfError(rc, "slf_pool_create")
        self._h = h
        self.device = device
        self._rigs = []

    def close(self):
        if getattr(self, "_h", None):
            for c in list(self._rigs):
                c._pool = None
            self._rigs = []
            self._L.slf_pool_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != SLF_OK:
            raise SlfError(rc, self._L.slf_pool_last_error(self._h).decode())
        return rc

    def last_error(self) -> str:
        return self._L.slf_pool_last_error(self._h).decode()

    def set_stream(self, stream) -> None:
        ptr = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream or 0)
        self._check(self._L.slf_pool_set_stream(self._h, ctypes.c_void_p(ptr)))

    def set_config(self, cfg: slf_pool_config) -> None:
        self._check(self._L.slf_pool_set_config(self._h, ctypes.byref(cfg)))

    def get_config(self) -> slf_pool_config:
        c = slf_pool_config()
        self._check(self._L.slf_pool_get_config(self._h, ctypes.byref(c)))
        return c

    def attach(self, ctx: Context) -> None:
        self._check(self._L.slf_pool_attach(self._h, ctx._h))
        ctx._pool = self
        self._rigs.append(ctx)

    def detach(self, ctx: Context) -> None:
        self._check(self._L.slf_pool_detach(self._h, ctx._h))
        ctx._pool = None
        self._rigs.remove(ctx)

    def usage(self):
        b, u = ctypes.c_uint64(), ctypes.c_uint64()
        nr, na = ctypes.c_int(), ctypes.c_int()
        self._check(self._L.slf_pool_usage(self._h, ctypes.byref(b), ctypes.byref(u), ctypes.byref(nr),
                                           ctypes.byref(na)))
        return {"budget": int(b.value), "used": int(u.value), "rigs": nr.value, "active": na.value}

    def submit(self, ctx: Context, op: int, first_iter: int, n_iters: int, tag: int) -> None:
        self._check(self._L.slf_pool_submit(self._h, ctx._h, op, first_iter, n_iters, tag))

    def step(self) -> int:
        n = ctypes.c_int()
        self._check(self._L.slf_pool_step(self._h, ctypes.byref(n)))
        return n.value

    def run(self) -> None:
        self._check(self._L.slf_pool_run(self._h))

    def poll(self, max_tags: int = 256):
        tags = np.zeros(max_tags, np.uint64)
        n = ctypes.c_int()
        self._check(self._L.slf_pool_poll(self._h, _ptr(tags), max_tags, ctypes.byref(n)))
        return [int(t) for t in tags[:n.value]]

    def synchronize(self) -> None:
        self._check(self._L.slf_pool_synchronize(self._h))

    def autotune(self) -> bool:
        """Returns True when the configuration came from the pool's cache."""
        hit = ctypes.c_int()
        self._check(self._L.slf_pool_autotune(self._h, ctypes.byref(hit)))
        return bool(hit.value)
