"""Batched and serving forms on the GPU: the rig pool (persistent pooled
launches, graph replay, continuous batching, admission, autotuning) and the
warm start.  A rig's results through a pool must equal, bit for bit, those of
the same rig run alone through the per-rig calls; the warm start is checked
against the oracle."""
from __future__ import annotations

import numpy as np
import pytest

from lfsynth import configs, states, tiny_custom
from oracle.oracle import Oracle
from tests import parity

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _slf():
    from paper_1812_06856_amd import slf

    return slf


def _ctx(w, **over):
    slf = _slf()
    ctx = slf.Context(0)
    ctx.load_rig(w.rig, slf.params_from(w.params, **over))
    return ctx


def _state(ctx, n_views):
    out = [ctx.get_planes(v) for v in range(n_views)]
    return [np.concatenate([o[i] for o in out]) for i in range(4)]


def _same(a, b, what):
    for i, name in enumerate(["planes", "energy", "choice", "margin"]):
        x, y = a[i], b[i]
        assert x.shape == y.shape
        same = (x == y) | (np.isnan(x) & np.isnan(y)) if x.dtype.kind == "f" else (x == y)
        assert same.all(), "%s: %s differs at %d entries" % (what, name, int((~same).sum()))


def _rigs():
    return [tiny_custom(160, 120, 20, 15, seed=31, levels=48, iterations=2),
            tiny_custom(97, 61, 9, 7, seed=32, levels=24, iterations=2, n_views=4),
            tiny_custom(200, 80, 17, 6, seed=33, levels=40, iterations=2, n_views=2)]


def _solo(w, n_iters, **over):
    ctx = _ctx(w, **over)
    ctx.sweep()
    ctx.propagate(1, n_iters)
    st = _state(ctx, len(w.rig.views))
    depth = [ctx.get_depth(v) for v in range(len(w.rig.views))]
    ctx.close()
    return st, depth


@pytest.mark.parametrize("mode", ["graph", "eager", "tiles"])
def test_pool_solve_equals_solo(mode):
    slf = _slf()
    _say("pool solve vs solo: %s" % mode)
    ws = _rigs()
    solo = [_solo(w, 2) for w in ws]
    pool = slf.Pool(0)
    cfg = slf.default_pool_config(use_graph=1 if mode == "graph" else 0)
    if mode == "tiles":
        cfg.sweep_tile, cfg.refine_tile, cfg.blocks_per_cu = 3, 2, 1
    pool.set_config(cfg)
    ctxs = [_ctx(w) for w in ws]
    for c in ctxs:
        pool.attach(c)
    for j, c in enumerate(ctxs):
        pool.submit(c, slf.SLF_POOL_SOLVE, 1, 2, 100 + j)
    pool.run()
    pool.synchronize()
    assert sorted(pool.poll()) == [100, 101, 102]
    for j, (w, c) in enumerate(zip(ws, ctxs)):
        _same(_state(c, len(w.rig.views)), solo[j][0], "%s rig %d" % (mode, j))
        for v in range(len(w.rig.views)):
            assert np.array_equal(c.get_depth(v), solo[j][1][v])
    for c in ctxs:
        c.close()
    pool.close()


@pytest.mark.parametrize("kc", [4, 16])
def test_pool_level_chunk_does_not_change_results(kc):
    slf = _slf()
    _say("pool level chunk %d" % kc)
    ws = _rigs()[:2]
    solo = [_solo(w, 1) for w in ws]
    pool = slf.Pool(0)
    pool.set_config(slf.default_pool_config(sweep_level_chunk=kc))
    ctxs = [_ctx(w) for w in ws]
    for j, c in enumerate(ctxs):
        pool.attach(c)
        pool.submit(c, slf.SLF_POOL_SOLVE, 1, 1, j)
    pool.run()
    for j, (w, c) in enumerate(zip(ws, ctxs)):
        _same(_state(c, len(w.rig.views)), solo[j][0], "kc %d rig %d" % (kc, j))
        c.close()
    pool.close()


def test_graph_replays_match_eager():
    slf = _slf()
    _say("graph replays vs eager")
    ws = _rigs()
    eager = [_solo(w, 2)[0] for w in ws]
    pool = slf.Pool(0)
    ctxs = [_ctx(w) for w in ws]
    for c in ctxs:
        pool.attach(c)
    for rep in range(4):
        for j, c in enumerate(ctxs):
            pool.submit(c, slf.SLF_POOL_SOLVE, 1, 2, 10 * rep + j)
        pool.run()
        # eager work and synchronisation between replays
        for j, (w, c) in enumerate(zip(ws, ctxs)):
            _same(_state(c, len(w.rig.views)), eager[j], "replay %d rig %d" % (rep, j))
            c.get_depth(0)
    assert sorted(pool.poll()) == sorted(10 * r + j for r in range(4) for j in range(3))
    for c in ctxs:
        c.close()
    pool.close()


def test_continuous_batching_joins_at_stage_boundaries():
    slf = _slf()
    _say("continuous batching")
    ws = _rigs()
    solo = [_solo(w, 3)[0] for w in ws]
    pool = slf.Pool(0)
    ctxs = [_ctx(w) for w in ws]
    for c in ctxs:
        pool.attach(c)
    pool.submit(ctxs[0], slf.SLF_POOL_SOLVE, 1, 3, 0)
    assert pool.step() == 1
    pool.submit(ctxs[1], slf.SLF_POOL_SOLVE, 1, 3, 1)
    assert pool.step() == 2
    with pytest.raises(slf.SlfError) as e:
        ctxs[0].sweep()  # stages not yet launched
    assert e.value.status == slf.SLF_ESTATE
    pool.submit(ctxs[2], slf.SLF_POOL_SOLVE, 1, 3, 2)
    steps = 2
    done = []
    while pool.step():
        steps += 1
        done += pool.poll()
    pool.synchronize()
    done += pool.poll()
    assert sorted(done) == [0, 1, 2]
    assert steps == 2 + 3  # the last request needs 4 stages, joining at stage 3
    for j, (w, c) in enumerate(zip(ws, ctxs)):
        _same(_state(c, len(w.rig.views)), solo[j], "batched rig %d" % j)
        c.close()
    pool.close()


def test_admission_refuses_over_budget_rigs():
    slf = _slf()
    _say("admission")
    ws = _rigs()
    ctxs = [_ctx(w) for w in ws]
    fps = [c.footprint() for c in ctxs]
    assert all(f > 0 for f in fps)
    pool = slf.Pool(0, hbm_budget_bytes=fps[0] + fps[1] + fps[2] - 1)
    pool.attach(ctxs[0])
    pool.attach(ctxs[1])
    with pytest.raises(slf.SlfError) as e:
        pool.attach(ctxs[2])
    assert e.value.status == slf.SLF_ENOMEM
    assert pool.usage() == {"budget": sum(fps) - 1, "used": fps[0] + fps[1], "rigs": 2, "active": 0}
    pool.detach(ctxs[0])
    pool.attach(ctxs[2])
    assert pool.usage()["used"] == fps[1] + fps[2]
    tiny = slf.Pool(0, hbm_budget_bytes=1024)
    with pytest.raises(slf.SlfError) as e:
        tiny.attach(ctxs[0])
    assert e.value.status == slf.SLF_ENOMEM
    for x in ctxs:
        x.close()
    tiny.close()
    pool.close()


def test_warm_start_matches_oracle():
    _say("warm start vs oracle")
    seq = configs.tiny_sequence(seed=41)
    r0, r1 = seq.frame(0), seq.frame(1)
    w0 = configs.Workload("f0", r0, seq.params)
    ctx = _ctx(w0)
    rng = np.random.default_rng(9)
    o0, o1 = Oracle(r0, seq.params), Oracle(r1, seq.params)
    area0 = o0.sp_stats()[0]
    A = np.concatenate([states.random_planes(rng, v.gw, v.gh, 2.0, 8.0, max_tilt_deg=30) for v in r0.views])
    A[area0 == 0] = 0
    A = parity.round_state(A)
    for v in range(o0.V):
        ctx.set_planes(v, A[o0.view_slice(v)])
    for v, view in enumerate(r1.views):
        ctx.set_image(v, view.rgb)
        ctx.set_labels(v, view.labels, view.gw, view.gh)
    ctx.warm_start()
    P = _state(ctx, o1.V)[0].astype(np.float64)
    E = o1.warm_start(o0, A)
    area1 = o1.sp_stats()[0]
    nz = area1 > 0
    assert np.array_equal(P[~nz], E[~nz])
    assert np.array_equal(P[nz, 1:], E[nz, 1:].astype(np.float32).astype(np.float64))
    rel = np.abs(P[nz, 0] - E[nz, 0]) / E[nz, 0]
    _say("warm start depth: max rel %.3g over %d cells" % (rel.max(), nz.sum()))
    assert rel.max() < 1e-5
    # then the refinement runs from it in lockstep with the oracle
    ctx.propagate(1, 1)
    A1 = parity.round_state(E)
    rep = parity.check_refine(o1, ctx, A1, 1)
    assert not rep["bad"], rep["bad"][:5]
    # a rig without a previous state cannot warm start
    slf = _slf()
    c2 = _ctx(w0)
    with pytest.raises(slf.SlfError) as e:
        c2.warm_start()
    assert e.value.status == slf.SLF_ESTATE
    ctx.close()
    c2.close()


def _serve_solo(seq, frames, iters):
    ctx = _ctx(configs.Workload(seq.name, seq.frame(0), seq.params))
    ctx.sweep()
    ctx.propagate(1, iters)
    out = []
    for k in range(1, frames):
        for v, view in enumerate(seq.frame(k).views):
            ctx.set_image(v, view.rgb)
            ctx.set_labels(v, view.labels, view.gw, view.gh)
        ctx.warm_start()
        ctx.propagate(1, iters)
        out.append(_state(ctx, len(seq.views)))
    ctx.close()
    return out


def test_served_frames_equal_alone_and_in_the_mix():
    slf = _slf()
    _say("serving: alone vs in the mix")
    seqs = [configs.tiny_sequence(seed=51), configs.tiny_sequence(seed=52, W=128, H=96, gw=16, gh=12, n_views=4),
            configs.tiny_sequence(seed=53, levels=20)]
    frames, iters = 3, 2
    alone = [_serve_solo(s, frames, iters) for s in seqs]
    pool = slf.Pool(0)
    ctxs = [_ctx(configs.Workload(s.name, s.frame(0), s.params)) for s in seqs]
    for c in ctxs:
        pool.attach(c)
    # frame 0: full solves, staggered so that requests overlap in stages
    for j, c in enumerate(ctxs):
        pool.submit(c, slf.SLF_POOL_SOLVE, 1, iters, j)
        pool.step()
    pool.run()
    pool.synchronize()
    for k in range(1, frames):
        order = [(k + j) % len(seqs) for j in range(len(seqs))]
        for j in order:
            c, s = ctxs[j], seqs[j]
            for v, view in enumerate(s.frame(k).views):
                c.set_image(v, view.rgb)
                c.set_labels(v, view.labels, view.gw, view.gh)
            c.warm_start()
            pool.submit(c, slf.SLF_POOL_PROPAGATE, 1, iters, 100 * k + j)
            pool.step()
        pool.run()
        pool.synchronize()
        for j, (c, s) in enumerate(zip(ctxs, seqs)):
            _same(_state(c, len(s.views)), alone[j][k - 1], "frame %d rig %d" % (k, j))
    for c in ctxs:
        c.close()
    pool.close()


def test_autotune_caches_and_keeps_results():
    """The autotuner's trials leave every rig as after a plain sweep.  With
    the default bound the reported margins are upper bounds whose value
    depends on the level chunk and split the autotuner picks, so the rigs
    run with exact margins here: every output is then independent of the
    schedule and must equal the plain sweep's bit for bit."""
    slf = _slf()
    _say("autotune")
    ws = _rigs()[:2]
    swept = []
    for w in ws:
        c = _ctx(w, exact_margin=1)
        c.sweep()
        swept.append(_state(c, len(w.rig.views)))
        c.close()
    pool = slf.Pool(0)
    ctxs = [_ctx(w, exact_margin=1) for w in ws]
    for c in ctxs:
        pool.attach(c)
    w0 = [c.work() for c in ctxs]
    assert pool.autotune() is False
    cfg = pool.get_config()
    _say("autotuned: %s" % cfg.as_dict())
    assert cfg.sweep_level_chunk in (4, 8, 16) and 1 <= cfg.sweep_tile <= 4 and 1 <= cfg.refine_tile <= 4
    assert [c.work() for c in ctxs] == w0
    for j, (w, c) in enumerate(zip(ws, ctxs)):
        _same(_state(c, len(w.rig.views)), swept[j], "after autotune rig %d" % j)
    assert pool.autotune() is True
    for c in ctxs:
        c.close()
    pool.close()


def test_autotune_on_rigs_larger_than_its_trial_cap():
    """The autotuner times stages cut to the first 2048 superpixels of each
    rig, with level splits among the schedules it tries.  On rigs with more
    superpixels than that, a cut stage must take superpixels 0..2047 in index
    order (its split records are reserved for 2048 superpixels), while full
    stages take the rig's strip order; afterwards every output equals a plain
    sweep's."""
    slf = _slf()
    _say("autotune on rigs above the trial cap")
    ws = [tiny_custom(640, 360, 64, 36, seed=41, levels=24, iterations=1, labels="grid"),
          tiny_custom(320, 240, 50, 48, seed=42, levels=16, iterations=1, n_views=4, labels="grid")]
    assert all(w.rig.views[0].gw * w.rig.views[0].gh * w.rig.n_views > 2048 for w in ws)
    swept = []
    for w in ws:
        c = _ctx(w, exact_margin=1)
        c.sweep()
        swept.append(_state(c, len(w.rig.views)))
        c.close()
    pool = slf.Pool(0)
    ctxs = [_ctx(w, exact_margin=1) for w in ws]
    for c in ctxs:
        pool.attach(c)
    assert pool.autotune() is False
    _say("autotuned: %s" % pool.get_config().as_dict())
    for j, (w, c) in enumerate(zip(ws, ctxs)):
        _same(_state(c, len(w.rig.views)), swept[j], "after autotune rig %d" % j)
    for c in ctxs:
        c.close()
    pool.close()


def test_pool_argument_errors():
    slf = _slf()
    _say("pool errors")
    w = _rigs()[0]
    pool = slf.Pool(0)
    c = _ctx(w)
    with pytest.raises(slf.SlfError):
        pool.submit(c, slf.SLF_POOL_SOLVE, 1, 1, 0)  # not attached
    pool.attach(c)
    with pytest.raises(slf.SlfError) as e:
        pool.attach(c)
    assert e.value.status == slf.SLF_ESTATE
    with pytest.raises(slf.SlfError) as e:
        pool.submit(c, slf.SLF_POOL_PROPAGATE, 1, 1, 0)  # no planes yet
    assert e.value.status == slf.SLF_ESTATE
    with pytest.raises(slf.SlfError):
        pool.submit(c, 7, 1, 1, 0)
    with pytest.raises(slf.SlfError):
        pool.set_config(slf.default_pool_config(sweep_level_chunk=5))
    pool.submit(c, slf.SLF_POOL_SOLVE, 1, 1, 0)
    with pytest.raises(slf.SlfError) as e:
        pool.detach(c)
    assert e.value.status == slf.SLF_ESTATE
    with pytest.raises(slf.SlfError) as e:
        pool.submit(c, slf.SLF_POOL_SOLVE, 1, 1, 1)
    assert e.value.status == slf.SLF_ESTATE
    pool.run()
    pool.synchronize()
    assert pool.poll() == [0]
    pool.detach(c)
    c.close()
    pool.close()


def test_pool_mixed_formats_equal_solo():
    """Rigs with different image storage share a pool: each stage runs one
    launch per (operation, format) group, results as alone."""
    slf = _slf()
    _say("pool with mixed image formats")
    ws = _rigs()
    fmts = [slf.SLF_IMAGE_U8, slf.SLF_IMAGE_F16, slf.SLF_IMAGE_F32]
    solo = [_solo(w, 2, image_precision=f)[0] for w, f in zip(ws, fmts)]
    pool = slf.Pool(0)
    ctxs = [_ctx(w, image_precision=f) for w, f in zip(ws, fmts)]
    for j, c in enumerate(ctxs):
        pool.attach(c)
        pool.submit(c, slf.SLF_POOL_SOLVE, 1, 2, j)
    pool.run()
    for j, (w, c) in enumerate(zip(ws, ctxs)):
        _same(_state(c, len(w.rig.views)), solo[j], "mixed formats rig %d" % j)
        c.close()
    pool.close()


def test_graph_recaptured_when_the_stage_shape_changes():
    """Solve, then propagate-only, then solve again through graph runs: each
    shape is captured on its own and every run equals the eager result."""
    slf = _slf()
    _say("graph shape changes")
    ws = _rigs()[:2]
    eager = []
    for w in ws:
        c = _ctx(w)
        c.sweep()
        c.propagate(1, 2)
        first = _state(c, len(w.rig.views))
        c.propagate(3, 1)
        second = _state(c, len(w.rig.views))
        eager.append((first, second))
        c.close()
    pool = slf.Pool(0)
    ctxs = [_ctx(w) for w in ws]
    for c in ctxs:
        pool.attach(c)
    for rep in range(2):
        for j, c in enumerate(ctxs):
            pool.submit(c, slf.SLF_POOL_SOLVE, 1, 2, j)
        pool.run()
        for j, (w, c) in enumerate(zip(ws, ctxs)):
            _same(_state(c, len(w.rig.views)), eager[j][0], "solve run %d rig %d" % (rep, j))
        for j, c in enumerate(ctxs):
            pool.submit(c, slf.SLF_POOL_PROPAGATE, 3, 1, 10 + j)
        pool.run()
        for j, (w, c) in enumerate(zip(ws, ctxs)):
            _same(_state(c, len(w.rig.views)), eager[j][1], "propagate run %d rig %d" % (rep, j))
    for c in ctxs:
        c.close()
    pool.close()


@pytest.mark.parametrize("split,kc", [(2, 8), (3, 4), (4, 8)])
def test_pool_level_split_equals_solo(split, kc):
    """Sweep work items of 1/split of the levels (hypothesis chunks) merged in
    level order give the single-pass result bit for bit, including parts left
    empty when the levels do not divide evenly."""
    slf = _slf()
    _say("pool level split %d, chunk %d" % (split, kc))
    ws = _rigs()
    solo = [_solo(w, 1)[0] for w in ws]
    pool = slf.Pool(0)
    pool.set_config(slf.default_pool_config(sweep_level_split=split, sweep_level_chunk=kc, sweep_tile=2))
    ctxs = [_ctx(w) for w in ws]
    for j, c in enumerate(ctxs):
        pool.attach(c)
        pool.submit(c, slf.SLF_POOL_SOLVE, 1, 1, j)
    pool.run()
    for j, (w, c) in enumerate(zip(ws, ctxs)):
        _same(_state(c, len(w.rig.views)), solo[j], "split %d rig %d" % (split, j))
        c.close()
    pool.close()
