"""GPU (HIP, through the C ABI) vs FP64 oracle parity on seeded synthetic inputs."""
from __future__ import annotations

import numpy as np
import pytest

from lfsynth import config1, tiny_custom
from lfsynth.rig import line_rig, grid_rig
from lfsynth.scene import make_scene, build_rig, grid_labels
from oracle.oracle import Oracle
from tests import parity

pytestmark = pytest.mark.gpu


def _ctx(workload, **over):
    from paper_1812_06856_amd import slf

    ctx = slf.Context(0)
    p = slf.params_from(workload.params, **over)
    ctx.load_rig(workload.rig, p)
    return ctx


def _oracle(workload, **over):
    p = workload.params
    for k, v in over.items():
        setattr(p, k, v)
    return Oracle(workload.rig, p)


def _say(msg):
    print(msg, flush=True)


def _assert_clean(rep, what):
    _say("%s: %s" % (what, {k: (v if k != "bad" else len(v)) for k, v in rep.items()}))
    assert not rep["bad"], rep["bad"][:10]


def _lockstep(w, iters, ctx=None, orc=None, **over):
    ctx = ctx or _ctx(w, **over)
    orc = orc or _oracle(w, **over)
    A = orc.sweep()[0]
    for it in range(1, iters + 1):
        A64 = parity.round_state(A)
        for v in range(orc.V):
            ctx.set_planes(v, A64[orc.view_slice(v)])
        ctx.propagate(it, 1)
        B, E, K, M = orc.refine(A64, it)
        rep = parity.check_refine(orc, ctx, A64, it, B, E, K, M)
        _assert_clean(rep, "%s refine iter %d" % (w.name, it))
        A = B
    return ctx, orc


# ------------------------------------------------------------------ a1: superpixel setup

@pytest.mark.parametrize("case", ["config1", "ragged161x117", "holes"])
def test_superpixel_statistics(case):
    _say("superpixels: %s" % case)
    if case == "config1":
        w = config1()
    elif case == "ragged161x117":
        w = tiny_custom(161, 117, 13, 9, seed=3)
    else:
        w = tiny_custom(96, 64, 8, 6, seed=4, labels="grid")
        for v in w.rig.views:
            v.labels[v.labels == 9] = 10
            v.labels[v.labels == 30] = 22
    ctx = _ctx(w)
    orc = _oracle(w)
    ctx.sweep()
    area_o, cen_o, col_o = orc.sp_stats()
    for v in range(orc.V):
        sl = orc.view_slice(v)
        area, cen, col = ctx.get_superpixels(v)
        assert np.array_equal(area, area_o[sl])
        assert np.allclose(cen, cen_o[sl], rtol=0, atol=2e-4)
        assert np.allclose(col, col_o[sl], rtol=0, atol=1e-6)


# ------------------------------------------------------------------ a2-a5: sweep

@pytest.mark.parametrize("fmt", [0, 2])
def test_sweep_parity_tiny(fmt):
    _say("sweep parity tiny, image format %d" % fmt)
    w = config1()
    ctx = _ctx(w, image_precision=fmt)
    orc = _oracle(w)
    ctx.sweep()
    rep = parity.check_sweep(orc, ctx)
    _assert_clean(rep, "sweep fmt %d" % fmt)
    assert rep["n"] == 900


def test_precision_form_sweep_and_depth_error():
    """Precision form (FP16 texels, FP32 interpolation and accumulation, FP64
    composition): the plain bar against the oracle for the sweep, end-to-end
    depth within 0.5 % (mean relative error) after 3 refinement iterations,
    and, since 8-bit colours are exact in FP16, every output equal bit for bit
    to the FP32-texel form's."""
    _say("precision form: tiny workload")
    w = config1()
    ctx = _ctx(w, image_precision=1)
    ref = _ctx(w, image_precision=2)
    orc = _oracle(w)
    ctx.sweep()
    ref.sweep()
    rep = parity.check_sweep(orc, ctx)
    _assert_clean(rep, "precision-form sweep")
    ctx.propagate(1, 3)
    ref.propagate(1, 3)
    for v in range(orc.V):
        a, b = ctx.get_planes(v), ref.get_planes(v)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
        assert np.array_equal(ctx.get_depth(v), ref.get_depth(v))
    hist = orc.run(3)
    errs = [parity.depth_mare(ctx.get_depth(v), orc.render_depth(hist[-1][0], v))[0] for v in range(orc.V)]
    _say("precision form depth MARE per view: %s" % errs)
    assert max(errs) <= parity.DEPTH_REL


@pytest.mark.parametrize("case", ["ragged", "tiny_sp", "large_sp", "two_views", "one_level", "no_jitter",
                                  "neighbour_subset", "mixed_sizes"])
def test_sweep_parity_edge_cases(case):
    _say("sweep edge case %s" % case)
    if case == "ragged":
        w = tiny_custom(161, 117, 13, 9, seed=3, levels=24)
    elif case == "tiny_sp":
        w = tiny_custom(160, 120, 40, 30, seed=5, levels=16, labels="grid")
    elif case == "large_sp":
        w = tiny_custom(160, 120, 2, 2, seed=6, levels=8, labels="grid")
    elif case == "two_views":
        w = tiny_custom(96, 72, 8, 6, n_views=2, seed=8, levels=20)
    elif case == "one_level":
        w = tiny_custom(96, 72, 8, 6, seed=9, levels=1)
    elif case == "no_jitter":
        w = tiny_custom(96, 72, 8, 6, seed=10, levels=20)
        w.params.jitter = 0
    elif case == "neighbour_subset":
        w = tiny_custom(96, 72, 8, 6, n_views=4, seed=11, levels=20)
        w.rig.neighbors = [[1], [0, 2], [3, 1], [2]]
    else:
        w = _mixed_size_workload()
    ctx = _ctx(w)
    orc = _oracle(w)
    ctx.sweep()
    rep = parity.check_sweep(orc, ctx)
    _assert_clean(rep, "sweep %s" % case)


def test_sweep_level_bound_exact():
    """Superpixels of 128 x 96 px in 3 views (24 576 px-view pairs, 384 lane
    passes per level chunk) over 48 levels: the sweep's level bound stops
    chunks once every level in them is bounded above a complete level's cost.
    With exact_margin that is the second best, and the margin must match
    the oracle's; by default it is the best, which must leave the level, plane
    and cost bit for bit as they are and give a margin no smaller than the
    exact one, with fewer samples computed.  Both must match the oracle's full
    sweep, and both must have skipped samples."""
    _say("sweep level bound, large superpixels")
    w = tiny_custom(256, 192, 2, 2, n_views=3, seed=21, levels=48, labels="grid")
    orc = _oracle(w)
    area = orc.sp_stats()[0]
    runs = {}
    for exact in (1, 0):
        ctx = _ctx(w, exact_margin=exact)
        ctx.reset_work()
        ctx.sweep()
        _assert_clean(parity.check_sweep(orc, ctx), "level-bound sweep, exact margin %d" % exact)
        computed, total = ctx.sweep_work()
        _say("exact margin %d: sweep samples computed %d of %d" % (exact, computed, total))
        assert total == int(area.sum()) * 2 * 48
        assert 0 < computed < total
        assert ctx.work()[1] == computed
        runs[exact] = (parity.gpu_state(ctx, orc.V), computed)
        ctx.close()
    (P1, C1, K1, M1), n1 = runs[1]
    (P0, C0, K0, M0), n0 = runs[0]
    assert np.array_equal(P1, P0) and np.array_equal(C1, C0) and np.array_equal(K1, K0)
    full = K1 >= 0
    assert (M0[full] >= M1[full]).all()
    assert n0 <= n1
    for v in range(orc.V):
        for s in range(int(orc.sp_off[v + 1] - orc.sp_off[v])):
            g = int(orc.sp_off[v]) + s
            if area[g] == 0:
                continue
            _, _, k_o, m_o = orc.sweep_sp(v, s)
            if int(K1[g]) == k_o:
                assert abs(float(M1[g]) - m_o) <= parity.MARGIN + parity.REL * abs(m_o), (v, s, M1[g], m_o)


def test_sweep_parity_many_views():
    """66 views in a line (65 neighbour views per reference view): more
    neighbours than lanes in a wave, so per-view tables and flags indexed by
    lane must not be taken for views past the 64th; then one refinement
    iteration in lockstep with the oracle."""
    _say("sweep parity with 65 neighbour views")
    w = tiny_custom(40, 30, 2, 2, n_views=66, seed=23, levels=12, labels="grid")
    ctx = _ctx(w)
    orc = _oracle(w)
    ctx.sweep()
    _assert_clean(parity.check_sweep(orc, ctx), "sweep 66 views")
    _lockstep(w, 1, ctx=ctx, orc=orc)  # refinement: neighbour-view constants in passes of 16


def _mixed_size_workload():
    from lfsynth.configs import MethodParams, Workload
    from lfsynth.rig import View, intrinsics, pose_from_centre

    rng = np.random.Generator(np.random.PCG64(12))
    views = []
    for (W, H, f, x) in ((160, 120, 200.0, -0.1), (200, 150, 250.0, 0.0), (128, 96, 160.0, 0.1)):
        R, t = pose_from_centre([x, 0, 0])
        views.append(View(W, H, intrinsics(f, W, H), R, t))
    scene = make_scene(rng, f=200.0, W=160, H=120, sp_px=64.0, n_rect=3)
    r = build_rig(views[:1], scene, 20, 15)
    r2 = build_rig(views[1:2], scene, 25, 19)
    r3 = build_rig(views[2:], scene, 16, 12)
    r.views = r.views + r2.views + r3.views
    return Workload("mixed-sizes", r, MethodParams(levels=24, iterations=2))


# ------------------------------------------------------------------ a6-a8: refinement (lockstep)

def test_refine_lockstep_tiny():
    _say("refine lockstep tiny, 3 iterations")
    _lockstep(config1(), 3)


@pytest.mark.parametrize("case", ["ragged", "holes", "two_views", "neighbour_subset", "large_sp"])
def test_refine_lockstep_edge_cases(case):
    _say("refine lockstep edge case %s" % case)
    if case == "ragged":
        w = tiny_custom(161, 117, 13, 9, seed=3, levels=24)
    elif case == "holes":
        w = tiny_custom(96, 64, 8, 6, seed=4, labels="grid", levels=16)
        for v in w.rig.views:
            v.labels[v.labels == 9] = 10
            v.labels[v.labels == 30] = 22
    elif case == "two_views":
        w = tiny_custom(96, 72, 8, 6, n_views=2, seed=8, levels=20)
    elif case == "neighbour_subset":
        w = tiny_custom(96, 72, 8, 6, n_views=4, seed=11, levels=20)
        w.rig.neighbors = [[1], [0, 2], [3, 1], [2]]
    else:
        w = tiny_custom(160, 120, 4, 3, seed=6, levels=8, labels="grid")
    _lockstep(w, 2)


def _max_side_workload(case):
    """Views with the largest side the boundary accepts (65535 px): a wide
    strip seen by three cameras on a horizontal line and a tall one seen by
    three on a vertical line, 256-pixel grid cells, 40 rectangles.  The
    cameras sit 0.0002 off the line, so that no row (column) maps exactly onto
    the image's last one, where the inside test would be decided by rounding."""
    from lfsynth.configs import Workload, MethodParams
    from lfsynth.rig import View, intrinsics, pose_from_centre

    W, H, gw, gh = (65535, 8, 2048, 1) if case == "wide" else (8, 65535, 1, 2048)
    views = []
    for i in (-1, 0, 1):
        centre = [0.1 * i, 0.0002 * i, 0.0] if case == "wide" else [0.0002 * i, 0.1 * i, 0.0]
        R, t = pose_from_centre(centre)
        views.append(View(W, H, intrinsics(200.0, W, H), R, t))
    rng = np.random.Generator(np.random.PCG64(12))
    scene = make_scene(rng, f=200.0, W=W, H=H, sp_px=W * H / (gw * gh), n_rect=40)
    rig = build_rig(views, scene, gw, gh, name="maxside-%s-3x%dx%d" % (case, W, H), seed=12, labels="grid")
    return Workload(rig.name, rig, MethodParams(levels=16, iterations=1))


@pytest.mark.parametrize("case,storage", [("wide", "u8"), ("tall", "u8"), ("wide", "f16"), ("wide", "f32")])
def test_maximum_image_side(case, storage):
    """The sweep and one lockstep refinement iteration on 65535 x 8 and
    8 x 65535 views (texel rows of 65536 entries, pixel coordinates up to
    65534 through the 24-bit index products), with each texel storage form,
    and a 65536-pixel side refused."""
    from paper_1812_06856_amd import slf

    _say("maximum image side, %s, %s texels" % (case, storage))
    w = _max_side_workload(case)
    fmt = {"u8": slf.SLF_IMAGE_U8, "f16": slf.SLF_IMAGE_F16, "f32": slf.SLF_IMAGE_F32}[storage]
    ctx = _ctx(w, image_precision=fmt)
    orc = _oracle(w)
    ctx.sweep()
    _assert_clean(parity.check_sweep(orc, ctx), "sweep %s" % w.name)
    _lockstep(w, 1, ctx=ctx, orc=orc)
    vs = w.rig.views
    big = slf.Context(0)
    sides = [(v.W + (1 if case == "wide" else 0), v.H + (1 if case == "tall" else 0)) for v in vs]
    with pytest.raises(slf.SlfError) as e:
        big.set_cameras(sides, [v.K for v in vs], [v.R for v in vs], [v.t for v in vs])
    assert e.value.status == slf.SLF_EUNSUPPORTED and "65535" in big.last_error()


@pytest.mark.parametrize("dims", [(2, 2, 1, 1), (5, 2, 2, 1), (2, 7, 1, 3)])
def test_minimum_image_side(dims):
    """Views of 2 x 2, 5 x 2 and 2 x 7 pixels (the smallest side the boundary
    accepts is 2): the sweep, two lockstep refinement iterations and the depth
    readout against the oracle, and a 1-pixel side refused."""
    from paper_1812_06856_amd import slf

    W, H, gw, gh = dims
    _say("minimum image side %dx%d" % (W, H))
    w = tiny_custom(W, H, gw, gh, n_views=3, seed=21, levels=8, labels="grid", f=2.0 * max(W, H))
    ctx = _ctx(w)
    orc = _oracle(w)
    ctx.sweep()
    _assert_clean(parity.check_sweep(orc, ctx), "sweep %s" % w.name)
    ctx, orc = _lockstep(w, 2, ctx=ctx, orc=orc)
    planes = np.concatenate([ctx.get_planes(v)[0] for v in range(orc.V)]).astype(np.float64)
    for v in range(orc.V):
        D_g = ctx.get_depth(v).astype(np.float64)
        D_o = orc.render_depth(planes, v)
        np.testing.assert_allclose(D_g, D_o, rtol=2e-5, atol=0)
    vs = w.rig.views
    small = slf.Context(0)
    with pytest.raises(slf.SlfError) as e:
        small.set_cameras([(1, H)] * len(vs), [v.K for v in vs], [v.R for v in vs], [v.t for v in vs])
    assert e.value.status == slf.SLF_EINVAL


def test_regridded_labels_on_one_context():
    """One context through three grids: 20 x 15 cells, then 15 x 20 (the same
    superpixel count, so the buffers stay and only the claim order and tables
    must follow the new grid), then 10 x 8 (fewer superpixels), each swept and
    checked against the oracle of that grid, then one lockstep iteration on
    the last."""
    import copy

    _say("regridded labels on one context")
    w = tiny_custom(160, 120, 20, 15, seed=31, levels=16, labels="grid")
    ctx = _ctx(w)
    for gw, gh in [(20, 15), (15, 20), (10, 8)]:
        wk = copy.deepcopy(w)
        for i, v in enumerate(wk.rig.views):
            v.labels = grid_labels(v.W, v.H, gw, gh)
            v.gw, v.gh = gw, gh
            ctx.set_labels(i, v.labels, gw, gh)
        orc = _oracle(wk)
        ctx.sweep()
        _assert_clean(parity.check_sweep(orc, ctx), "sweep on a %dx%d grid" % (gw, gh))
    _lockstep(wk, 1, ctx=ctx, orc=orc)


@pytest.mark.parametrize("mask", [1, 2, 6, 3])
def test_refine_lockstep_term_ablations(mask):
    _say("refine lockstep term_mask %d" % mask)
    w = config1()
    w.params.term_mask = mask
    _lockstep(w, 1)


@pytest.mark.parametrize("occ_tol", [0.0, 1e-3])
def test_refine_lockstep_literal_and_tolerant_visibility_split(occ_tol):
    """Eqs. (10)-(11) split the samples into visible (X) and occluded (Y) by
    comparing depths; tau = 0 is the literal comparison, tau = 1e-3 the default
    tolerance.  Both run in lockstep against the oracle on a slanted state,
    where consistent surfaces put many samples at z = D(p^i) up to rounding."""
    from lfsynth import random_planes

    _say("refine lockstep occ_tol %g" % occ_tol)
    w = config1()
    w.params.occ_tol = occ_tol
    ctx = _ctx(w)
    orc = _oracle(w)
    for start in ("sweep", "slanted"):
        if start == "sweep":
            A64 = parity.round_state(orc.sweep()[0])
        else:
            rng = np.random.default_rng(17)
            A64 = parity.round_state(np.concatenate([random_planes(rng, v.gw, v.gh, 2.0, 8.0) for v in w.rig.views]))
        for v in range(orc.V):
            ctx.set_planes(v, A64[orc.view_slice(v)])
        ctx.propagate(1, 1)
        rep = parity.check_refine(orc, ctx, A64, 1)
        _assert_clean(rep, "refine occ_tol %g from the %s state" % (occ_tol, start))


def test_refine_lockstep_data_only_mode():
    _say("refine lockstep data-only energy")
    w = config1()
    w.params.energy_mode = 1
    _lockstep(w, 2)


def test_refine_lockstep_random_state():
    """A given (non-sweep) state with slanted planes exercises every normal and
    occlusion path."""
    from lfsynth import random_planes

    _say("refine lockstep random slanted state")
    w = config1()
    ctx = _ctx(w)
    orc = _oracle(w)
    rng = np.random.default_rng(5)
    A = np.concatenate([random_planes(rng, v.gw, v.gh, 2.0, 8.0) for v in w.rig.views])
    A64 = parity.round_state(A)
    for v in range(orc.V):
        ctx.set_planes(v, A64[orc.view_slice(v)])
    ctx.propagate(1, 1)
    rep = parity.check_refine(orc, ctx, A64, 1)
    _assert_clean(rep, "random-state refine")


def test_refine_pruning_floor_modes():
    """Refinement candidates stop once their energy bound falls below the best
    energy so far (default) or the second best (exact_margin = 1).  Both must
    give the same winners, planes and energies bit for bit, the default's
    margins no smaller than the exact ones, more candidates pruned and fewer
    samples.  The exact mode is also checked in lockstep against the oracle."""
    _say("refinement pruning against the best vs the second best")
    w = config1()
    res = {}
    for exact in (1, 0):
        ctx = _ctx(w, exact_margin=exact)
        ctx.sweep()
        ctx.reset_work()
        ctx.propagate(1, 2)
        res[exact] = (parity.gpu_state(ctx, len(w.rig.views)), ctx.work_detail())
        ctx.close()
    (P1, E1, K1, M1), (ev1, smp1, pr1) = res[1]
    (P0, E0, K0, M0), (ev0, smp0, pr0) = res[0]
    _say("exact: %d evaluated, %d samples, %d pruned; default: %d, %d, %d" % (ev1, smp1, pr1, ev0, smp0, pr0))
    assert np.array_equal(P1, P0) and np.array_equal(E1, E0) and np.array_equal(K1, K0)
    full = K1 >= 0
    assert (M0[full] >= M1[full]).all()
    assert ev0 == ev1 and pr0 >= pr1 and smp0 <= smp1
    ctx = _ctx(w, exact_margin=1)
    _lockstep(w, 1, ctx=ctx)
    ctx.close()


def test_refine_lockstep_far_pixels():
    """4200-px-wide views whose last grid cell also owns the leftmost 100
    columns: its pixels lie up to 3359 px from its centroid, beyond what the
    FP16 offsets staged for the projection hold exactly (2048), so it reads
    every pixel from the list; the other cells are staged, with tails past
    the staging capacity."""
    _say("refine lockstep with pixels far from their centroid")
    w = tiny_custom(4200, 24, 4, 1, n_views=2, seed=17, labels="grid", levels=8, iterations=2)
    for v in w.rig.views:
        v.labels[:, :100] = 3
    ctx = _ctx(w)
    orc = _oracle(w)
    ctx.sweep()
    _assert_clean(parity.check_sweep(orc, ctx), "far-pixel sweep")
    _lockstep(w, 2, ctx=ctx, orc=orc)


def test_refine_wide_labels_sampled():
    """Views of 320 x 240 = 76800 cells: label gathers take the 32-bit path
    (16-bit labels cover at most 65536 cells), with many labels above 65535."""
    from lfsynth import random_planes

    _say("refine with 76800-cell views (32-bit label gathers)")
    w = tiny_custom(640, 480, 320, 240, n_views=2, seed=13, labels="grid", levels=8, iterations=1)
    ctx = _ctx(w)
    orc = _oracle(w)
    rng = np.random.default_rng(5)
    # tilts up to 20 degrees: every plane faces the camera out to the image
    # corners, 63 degrees off axis at f = 200 px
    A64 = parity.round_state(np.concatenate([random_planes(rng, v.gw, v.gh, 2.0, 8.0, max_tilt_deg=20.0)
                                             for v in w.rig.views]))
    for v in range(orc.V):
        ctx.set_planes(v, A64[orc.view_slice(v)])
    ctx.propagate(1, 1)
    sample = [(v, int(s)) for v in range(2) for s in rng.integers(0, 76800, 30)]
    sample += [(v, int(s)) for v in range(2) for s in rng.integers(65536, 76800, 15)]
    rep = parity.check_refine(orc, ctx, A64, 1, sample=sample)
    _assert_clean(rep, "wide-label refine")


# ------------------------------------------------------------------ a9: depth readout

def test_depth_readout_matches_oracle():
    from lfsynth import random_planes

    _say("depth readout")
    w = config1()
    ctx = _ctx(w)
    orc = _oracle(w)
    rng = np.random.default_rng(9)
    A64 = parity.round_state(np.concatenate([random_planes(rng, v.gw, v.gh, 2.0, 8.0) for v in w.rig.views]))
    for v in range(orc.V):
        ctx.set_planes(v, A64[orc.view_slice(v)])
    for v in range(orc.V):
        D_g = ctx.get_depth(v)
        D_o = orc.render_depth(A64, v)
        assert np.all((D_g > 0) == (D_o > 0))
        assert np.allclose(D_g, D_o, rtol=2e-5, atol=0)


def test_depth_readout_to_device_buffer_with_stride():
    import torch

    _say("depth readout into a strided device tensor")
    w = config1()
    ctx = _ctx(w)
    ctx.sweep()
    host = ctx.get_depth(1)
    buf = torch.full((120, 200), -1.0, device="cuda:0")
    ctx.get_depth(1, out=buf[:, 10:170])
    ctx.synchronize()
    got = buf.cpu().numpy()
    assert np.array_equal(got[:, 10:170], host)
    assert np.all(got[:, :10] == -1) and np.all(got[:, 170:] == -1)


# ------------------------------------------------------------------ end to end

def test_end_to_end_depth_error_tiny():
    _say("end to end tiny: sweep + 3 iterations, independent runs")
    w = config1()
    ctx = _ctx(w)
    orc = _oracle(w)
    ctx.sweep()
    ctx.propagate(1, 3)
    hist = orc.run(3)
    errs = []
    for v in range(orc.V):
        mare, rel = parity.depth_mare(ctx.get_depth(v), orc.render_depth(hist[-1][0], v))
        errs.append(mare)
    _say("end-to-end depth MARE per view: %s" % errs)
    assert max(errs) <= parity.DEPTH_REL


def test_device_inputs_match_host_inputs():
    import torch

    _say("device-resident inputs")
    w = config1()
    ctx_h = _ctx(w)
    ctx_h.sweep()
    ctx_h.propagate(1, 2)
    from paper_1812_06856_amd import slf

    ctx_d = slf.Context(0)
    vs = w.rig.views
    ctx_d.set_cameras([(v.W, v.H) for v in vs], [v.K for v in vs], [v.R for v in vs], [v.t for v in vs])
    ctx_d.set_params(slf.params_from(w.params))
    for i, v in enumerate(vs):
        ctx_d.set_image(i, torch.from_numpy(v.rgb).cuda())
        ctx_d.set_labels(i, torch.from_numpy(v.labels).cuda(), v.gw, v.gh)
    ctx_d.sweep()
    ctx_d.propagate(1, 2)
    for v in range(3):
        a, b = ctx_h.get_planes(v), ctx_d.get_planes(v)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


# ------------------------------------------------------------------ error paths through the ABI

def test_error_paths():
    import torch
    from paper_1812_06856_amd import slf

    _say("error paths")
    w = config1()
    vs = w.rig.views
    ctx = slf.Context(0)
    with pytest.raises(slf.SlfError) as e:
        ctx.sweep()
    assert e.value.status == slf.SLF_ESTATE
    ctx.set_cameras([(v.W, v.H) for v in vs], [v.K for v in vs], [v.R for v in vs], [v.t for v in vs])
    with pytest.raises(slf.SlfError) as e:
        ctx.sweep()
    assert e.value.status == slf.SLF_ESTATE
    for i, v in enumerate(vs):
        ctx.set_image(i, v.rgb)
    bad = vs[0].labels.copy()
    bad[3, 4] = 300
    with pytest.raises(slf.SlfError) as e:
        ctx.set_labels(0, bad, 20, 15)
    assert e.value.status == slf.SLF_EINVAL
    for i, v in enumerate(vs):
        ctx.set_labels(i, torch.from_numpy(bad if i == 0 else v.labels).cuda(), v.gw, v.gh)
    with pytest.raises(slf.SlfError) as e:
        ctx.sweep()
    assert e.value.status == slf.SLF_EINVAL and "label" in ctx.last_error()
    ctx.set_labels(0, vs[0].labels, 20, 15)
    with pytest.raises(slf.SlfError) as e:
        ctx.propagate(1, 1)
    assert e.value.status == slf.SLF_ESTATE
    ctx.sweep()
    planes = ctx.get_planes(0)[0].copy()
    planes[5, 1:] = [0, 0, -1]
    with pytest.raises(slf.SlfError) as e:
        ctx.set_planes(0, planes)
    assert e.value.status == slf.SLF_EINVAL
    with pytest.raises(slf.SlfError) as e:
        ctx.propagate(0, 1)
    assert e.value.status == slf.SLF_EINVAL
    with pytest.raises(slf.SlfError) as e:
        ctx.set_params(slf.default_params(d_min=3.0, d_max=2.0))
    assert e.value.status == slf.SLF_EINVAL
    with pytest.raises(slf.SlfError) as e:
        ctx.set_params(slf.default_params(exact_margin=2))
    assert e.value.status == slf.SLF_EINVAL and "exact_margin" in ctx.last_error()
    ctx.propagate(1, 1)
    ctx.synchronize()
