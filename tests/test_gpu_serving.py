"""The serving loop (paper_1812_06856_amd.serve) on the GPU against the oracle.

Two rigs of different sizes share one pool.  Each rig's first frame is solved
cold; then its planes are set to the oracle's final frame-0 state, so that the
warm frame that follows starts from a state the oracle knows.  The served warm
frame (warm start, then 2 iterations inside the pool, in the mix with the
other rig) must equal, bit for bit, the same chain run alone through the
per-rig calls, and that chain must match the oracle step by step: the warm
start within FP32 rounding and each iteration in lockstep (Sec. III-C
parity protocol).  End to end, the served depth maps are compared with the
oracle's warm start plus 2 iterations.
"""
from __future__ import annotations

import numpy as np
import pytest

from lfsynth import configs
from oracle.oracle import Oracle
from tests import parity

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _ctx(rig, params):
    from paper_1812_06856_amd import slf

    c = slf.Context(0)
    c.load_rig(rig, slf.params_from(params))
    return c


def _dev(rig):
    import torch

    return ([torch.from_numpy(v.rgb).cuda() for v in rig.views],
            [torch.from_numpy(v.labels).cuda() for v in rig.views])


def _set_inputs(ctx, rig):
    for v, view in enumerate(rig.views):
        ctx.set_image(v, view.rgb)
        ctx.set_labels(v, view.labels, view.gw, view.gh)


def test_served_warm_frames_match_the_oracle():
    import torch
    from paper_1812_06856_amd import serve, slf

    seqs = [configs.tiny_sequence(seed=61), configs.tiny_sequence(seed=62, W=128, H=96, gw=16, gh=12, n_views=4)]
    warm_iters = 2
    pool = slf.Pool(0)
    srv = serve.Server(pool)
    ctxs, depth, frames = [], [], []
    for j, s in enumerate(seqs):
        f0, f1 = s.frame(0), s.frame(1)
        frames.append((f0, f1))
        c = _ctx(f0, s.params)
        st = torch.cuda.Stream()
        c.set_stream(st)
        pool.attach(c)
        depth.append([torch.empty((v.H, v.W), dtype=torch.float32, device="cuda") for v in f0.views])
        srv.add_rig(c, st, depth[-1], s.params.iterations, warm_iters)
        ctxs.append(c)
    dev = [[_dev(f) for f in fr] for fr in frames]
    # frame 0 of both rigs, cold
    for j in range(len(seqs)):
        srv.submit(j, 0, *dev[j][0])
    done = srv.drain()
    assert sorted((d.rig, d.cold) for d in done) == [(0, True), (1, True)]
    # the oracle's frame-0 state replaces the GPU's, so the warm frame starts where the oracle's does
    orcs = []
    for j, s in enumerate(seqs):
        o0 = Oracle(frames[j][0], s.params)
        A0 = parity.round_state(o0.run(s.params.iterations)[-1][0])
        for v in range(o0.V):
            ctxs[j].set_planes(v, A0[o0.view_slice(v)])
        orcs.append((o0, A0))
    for j in range(len(seqs)):
        srv.submit(j, 1, *dev[j][1])
    done = srv.drain()
    assert sorted((d.rig, d.cold) for d in done) == [(0, False), (1, False)]
    torch.cuda.synchronize()
    for j, s in enumerate(seqs):
        o0, A0 = orcs[j]
        f0, f1 = frames[j]
        o1 = Oracle(f1, s.params)
        served = parity.gpu_state(ctxs[j], o1.V)
        served_depth = [d.cpu().numpy() for d in depth[j]]
        # the same chain alone through the per-rig calls: bit for bit
        alone = _ctx(f0, s.params)
        for v in range(o0.V):
            alone.set_planes(v, A0[o0.view_slice(v)])
        _set_inputs(alone, f1)
        alone.warm_start()
        alone.propagate(1, warm_iters)
        st = parity.gpu_state(alone, o1.V)
        for a, b, name in zip(served, st, ["planes", "energy", "choice", "margin"]):
            same = (a == b) | (np.isnan(a) & np.isnan(b)) if a.dtype.kind == "f" else (a == b)
            assert same.all(), "rig %d: served %s differs from the rig alone" % (j, name)
        # the chain step by step against the oracle
        lock = _ctx(f0, s.params)
        for v in range(o0.V):
            lock.set_planes(v, A0[o0.view_slice(v)])
        _set_inputs(lock, f1)
        lock.warm_start()
        P = parity.gpu_state(lock, o1.V)[0].astype(np.float64)
        E = o1.warm_start(o0, A0)
        nz = o1.sp_stats()[0] > 0
        rel = np.abs(P[nz, 0] - E[nz, 0]) / E[nz, 0]
        _say("rig %d warm start: max rel depth %.3g over %d cells" % (j, rel.max(), nz.sum()))
        assert rel.max() < 1e-5 and np.array_equal(P[nz, 1:], E[nz, 1:].astype(np.float32).astype(np.float64))
        A = parity.round_state(E)
        for it in range(1, warm_iters + 1):
            for v in range(o1.V):
                lock.set_planes(v, A[o1.view_slice(v)])
            lock.propagate(it, 1)
            B, En, K, M = o1.refine(A, it)
            rep = parity.check_refine(o1, lock, A, it, B, En, K, M)
            _say("rig %d warm iteration %d: %s" % (j, it, {k: (v if k != "bad" else len(v)) for k, v in rep.items()}))
            assert not rep["bad"], rep["bad"][:5]
            A = parity.round_state(B)
        # end to end: served depth maps against the oracle's warm start plus 2 iterations
        within = []
        for v in range(o1.V):
            D_o = o1.render_depth(A, v)
            m = (D_o > 0) & (served_depth[v] > 0)
            within.append(np.abs(served_depth[v][m] - D_o[m]) / D_o[m] <= parity.DEPTH_REL)
        frac = float(np.concatenate(within).mean())
        _say("rig %d served depth within 0.5%% of the oracle: %.4f" % (j, frac))
        assert frac >= 0.99
        alone.close()
        lock.close()
    for c in ctxs:
        pool.detach(c)
        c.close()
    pool.close()


def test_latest_frame_policy_drops_stale_frames():
    """Three frames of one rig queued while it is idle: with latest_only the
    newest is served and the two older are dropped; with every frame all
    three are served in order."""
    import torch
    from paper_1812_06856_amd import serve, slf

    s = configs.tiny_sequence(seed=63)
    frames = [s.frame(k) for k in range(3)]
    dev = [_dev(f) for f in frames]
    for latest in (True, False):
        pool = slf.Pool(0)
        srv = serve.Server(pool, latest_only=latest)
        c = _ctx(frames[0], s.params)
        st = torch.cuda.Stream()
        c.set_stream(st)
        pool.attach(c)
        depth = [torch.empty((v.H, v.W), dtype=torch.float32, device="cuda") for v in frames[0].views]
        srv.add_rig(c, st, depth, s.params.iterations, 2)
        for k in range(3):
            srv.submit(0, k, *dev[k])
        done = srv.drain()
        if latest:
            assert [d.frame for d in done] == [2] and srv.dropped == 2 and done[0].cold
        else:
            assert [d.frame for d in done] == [0, 1, 2] and srv.dropped == 0
            assert [d.cold for d in done] == [True, False, False]
        assert all(d.latency_ms >= 0 for d in done)
        pool.detach(c)
        c.close()
        pool.close()


def test_served_frames_with_fusion():
    """With fusion on, a served frame's fused maps equal slf_fuse on the same
    rig alone (the fusion's own parity is tested against the oracle)."""
    import torch
    from paper_1812_06856_amd import serve, slf

    s = configs.tiny_sequence(seed=64)
    f0 = s.frame(0)
    pool = slf.Pool(0)
    srv = serve.Server(pool, fuse_tol=0.01)
    c = _ctx(f0, s.params)
    st = torch.cuda.Stream()
    c.set_stream(st)
    pool.attach(c)
    depth = [torch.empty((v.H, v.W), dtype=torch.float32, device="cuda") for v in f0.views]
    fused = [torch.empty_like(d) for d in depth]
    srv.add_rig(c, st, depth, s.params.iterations, 2, fused=fused)
    srv.submit(0, 0, *_dev(f0))
    assert len(srv.drain()) == 1
    alone = _ctx(f0, s.params)
    alone.sweep()
    alone.propagate(1, s.params.iterations)
    alone.fuse(0.01)
    for v in range(len(f0.views)):
        ref, _ = alone.get_fused_depth(v)
        assert np.array_equal(fused[v].cpu().numpy().view(np.uint32), ref.view(np.uint32))
        assert (ref > 0).mean() > 0.5
    pool.detach(c)
    c.close()
    alone.close()
    pool.close()


def test_served_frames_segmented_on_the_gpu():
    """Frames submitted without labels are segmented on the GPU when admitted:
    the served result equals the same frame served with the oracle's SLIC
    labels (the segmentation's own parity is tested against the oracle)."""
    import torch
    from oracle import oracle
    from paper_1812_06856_amd import serve, slf

    s = configs.tiny_sequence(seed=65)
    f0 = s.frame(0)
    out = []
    for gpu_slic in (True, False):
        pool = slf.Pool(0)
        srv = serve.Server(pool, segment=(10, 20.0))
        c = _ctx(f0, s.params)
        st = torch.cuda.Stream()
        c.set_stream(st)
        pool.attach(c)
        depth = [torch.empty((v.H, v.W), dtype=torch.float32, device="cuda") for v in f0.views]
        srv.add_rig(c, st, depth, s.params.iterations, 2)
        imgs = [torch.from_numpy(v.rgb).cuda() for v in f0.views]
        labs = None if gpu_slic else [torch.from_numpy(oracle.slic(v.rgb, v.gw, v.gh, 10, 20.0)).cuda()
                                      for v in f0.views]
        srv.submit(0, 0, imgs, labs)
        assert len(srv.drain()) == 1
        out.append([d.cpu().numpy() for d in depth])
        pool.detach(c)
        c.close()
        pool.close()
    for a, b in zip(*out):
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
