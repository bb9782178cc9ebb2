"""slf_fuse_depth_static, the allocation-free form of slf_fuse_depth for
callers that cannot allocate, against slf_fuse_depth through the C ABI: the
same kernels run one reference view at a time in the library's fixed scratch,
so every fused depth and vote must be identical.  Two calls in a row share the
scratch, the second on a smaller rig; a rig too large for the scratch is
refused before anything runs."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

from lfsynth.depthmaps import noisy_depth_maps
from lfsynth.rig import arc_rig, line_rig
from lfsynth.scene import build_rig, make_scene

pytestmark = pytest.mark.gpu


def _rig(views, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    W, H, f = views[0].W, views[0].H, views[0].K[0, 0]
    scene = make_scene(rng, f=f, W=W, H=H, sp_px=64.0, n_rect=4)
    return build_rig(views, scene, max(1, W // 8), max(1, H // 8), labels="grid")


def _both(rig, seed, tau=0.01):
    import torch
    from paper_1812_06856_amd import slf

    ctx = slf.Context(0)
    vs = rig.views
    ctx.set_cameras([(v.W, v.H) for v in vs], [v.K for v in vs], [v.R for v in vs], [v.t for v in vs])
    depths = noisy_depth_maps(rig, seed=seed)
    din = [torch.from_numpy(d).cuda() for d in depths]
    outs = []
    for static in (True, False):
        f = [torch.full_like(d, -7.0) for d in din]
        vt = [torch.full(d.shape, -7, dtype=torch.int32, device="cuda") for d in din]
        print("fuse_depth static=%s views=%d %dx%d" % (static, len(vs), vs[0].W, vs[0].H), flush=True)
        ctx.fuse_depth(din, f, vt, tau, static_scratch=static)
        torch.cuda.synchronize()
        outs.append(([x.cpu().numpy() for x in f], [x.cpu().numpy() for x in vt]))
    (fs, vs_), (fa, va) = outs
    for v in range(len(vs)):
        assert np.array_equal(fs[v].view(np.uint32), fa[v].view(np.uint32)), v
        assert np.array_equal(vs_[v], va[v]), v
        assert (fa[v] > 0).mean() > 0.5
    return ctx


def test_static_scratch_fusion_matches_the_allocating_form_twice():
    _both(_rig(arc_rig(6, 5.0, 1.5, 180.0, 203, 151), 71), seed=3)
    # second call: a smaller rig on the same device scratch
    _both(_rig(line_rig(3, 0.1, 100.0, 97, 61), 72), seed=4)


def test_static_scratch_refuses_a_rig_beyond_its_size():
    from paper_1812_06856_amd import slf

    ctx = slf.Context(0)
    n, W, H = 18, 1920, 1080                     # 17 x 2073600 x 4 bytes > 64 MiB
    vs = line_rig(n, 0.05, 2000.0, W, H)
    ctx.set_cameras([(v.W, v.H) for v in vs], [v.K for v in vs], [v.R for v in vs], [v.t for v in vs])
    ptrs = (ctypes.c_void_p * n)(*([1] * n))       # never dereferenced: the size check comes first
    rc = slf.load().slf_fuse_depth_static(ctx._h, ptrs, ptrs, None, ctypes.c_float(0.01))
    assert rc == slf.SLF_EUNSUPPORTED
    assert "static scratch" in ctx.last_error()
