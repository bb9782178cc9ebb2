#!/usr/bin/env python3
"""Benchmark: superpixel-plane matching cost on the full-HD 8-view workload.

One step = the whole depth path on one multi-view frame whose images and
labels are already resident in device memory: texel build and superpixel
setup, the 256-level plane sweep of every superpixel of every view, 8
refinement iterations over all views, and the depth readout of every view.

Prints ONE JSON line (metric: SP-plane hypothesis evaluations per second).

Other workloads (--workload): `precision` (4x4 rig at 720p, each image
storage form timed and its end-to-end depth compared with the FP64 oracle's),
`batched` (32 rigs of uneven size through one rig pool) and `serving` (6 rigs,
Poisson frame arrivals, warm start, continuous batching; p50/p99 latency).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FP32 VALU operations per px-view sample (FMA = 1 op): the
# minimum the method itself needs per sample.
OPS_PER_SAMPLE_SWEEP = 35.0
OPS_PER_SAMPLE_REFINE = 55.0
# FP32 VALU lane-ops/s of MI355X (FMA = 1 op): 256 CUs x 128 FP32 lanes per
# clock x 2.4 GHz = 78.6e12, i.e. the published 157.3 TFLOP/s FP32 vector peak
# with an FMA counted as 2 flops.
PEAK_VALU_OPS = 256 * 128 * 2.4e9


def _progress(msg):
    print("[bench %s] %s" % (time.strftime("%H:%M:%S"), msg), file=sys.stderr, flush=True)


def hbm_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, calibrated by a plain device copy), or
    None when the kernel source has changed since the counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "hbm_traffic_fullhd_8view.json")
    src = os.path.join(ROOT, "paper_1812_06856_amd", "csrc", "slf_kernels.hip")
    try:
        rec = json.load(open(path))
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256_16") != sha:
        return None
    for name, k in rec["kernels"].items():
        if name.endswith(kernel) or name.split("<")[0].endswith(kernel):
            return k["read_bytes"] + k["write_bytes"]
    return None


FUSE_TOL = 0.01   # agreement tolerance of the depth fusion (relative depth)
SLIC_ITERATIONS, SLIC_COMPACTNESS = 10, 20.0   # the GPU segmentation timed beside the step


def sweep_evals_per_frame(ctx, w):
    """Sweep hypotheses decided per frame: levels x non-empty superpixels."""
    n = sum(int((ctx.get_superpixels(v)[0] > 0).sum()) for v in range(w.rig.n_views))
    return w.params.levels * n


def fusion_record(w, ms):
    """Depth fusion of all views of the frame: time and algorithmic HBM bytes.
    Per frame of P pixels over V views: the depth readout (label read and
    depth write, 8 B/px), pass 1 (depth read, 4 B/px, and the candidate
    layers written once, 4 (V-1) B/px), pass 2 (layers read once, own depth
    read, fused and votes written: 4 (V-1) + 12 B/px).  The layer clear
    (4 (V-1) B/px) is counted apart."""
    V = w.rig.n_views
    P = sum(v.W * v.H for v in w.rig.views)
    algo = P * (8 + 4 + 12) + 2 * 4 * (V - 1) * P
    return {"ms": ms, "ms_per_view": ms / V, "agree_tol": FUSE_TOL, "algorithmic_hbm_bytes": algo,
            "clear_bytes": 4 * (V - 1) * P, "achieved_gbs": algo / (ms * 1e-3) / 1e9,
            "frac_of_8tbs": algo / (ms * 1e-3) / 8e12}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=8192, help="superpixels in the oracle's timed sample")
    ap.add_argument("--workload", default="fullhd",
                    choices=["fullhd", "precision", "batched", "serving", "sensitivity", "temporal"])
    ap.add_argument("--temporal-frames", type=int, default=8, help="temporal: frames per serving rig")
    ap.add_argument("--temporal-rigs", type=int, default=3, help="temporal: serving rigs measured")
    ap.add_argument("--rigs", type=int, default=32, help="batched: number of rigs")
    ap.add_argument("--serve-rigs", type=int, default=6)
    ap.add_argument("--serve-frames", type=int, default=6, help="serving: distinct frames rendered per rig")
    ap.add_argument("--serve-rate", type=float, default=60.0,
                    help="serving: mean arrivals per second of the latest-frame run")
    ap.add_argument("--serve-rates", default="5,10,20,30,60", help="serving: arrival rates run in turn")
    ap.add_argument("--serve-seconds", type=float, default=10.0, help="serving: measured seconds per rate")
    ap.add_argument("--serve-warmup-s", type=float, default=2.0)
    ap.add_argument("--serve-p99-bound-ms", type=float, default=500.0,
                    help="serving: p99 bound defining the sustained rate reported as value")
    ap.add_argument("--serve-seed", type=int, default=5)
    ap.add_argument("--image-precision", type=int, default=0)
    ap.add_argument("--issue-rates", action="store_true",
                    help="run the VALU issue-rate probe (paper_1812_06856_amd/_build/issue_rates) and exit")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run a plain device-to-device copy of this many MiB (HBM counter calibration)")
    return ap.parse_args()


def copy_calibration(mib):
    """A plain device copy of known size: hardware read/write byte counters
    of this kernel calibrate the counters of the path's kernels."""
    import torch

    n = mib << 20
    src = torch.randint(0, 255, (n,), dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": n, "launches": 3}), flush=True)


def cpu_baseline(w, n_sp):
    """The FP64 oracle, untuned, on a bounded sample of the same workload: n_sp
    superpixels swept over all levels and refined for all 8 iterations (from a
    seeded plane state), spread over the host's cores with one thread per core."""
    import concurrent.futures as cf

    import numpy as np

    from lfsynth import random_planes
    from oracle.oracle import Oracle

    orc = Oracle(w.rig, w.params)
    area = orc.sp_stats()[0]
    rng = np.random.default_rng(123)
    cand = np.nonzero(area > 0)[0]
    picks = rng.choice(cand, size=n_sp, replace=False)
    jobs = []
    for g in picks:
        v = int(np.searchsorted(orc.sp_off, g, side="right") - 1)
        jobs.append((v, int(g - orc.sp_off[v])))
    A = np.concatenate([random_planes(np.random.default_rng(7 + v), vw.gw, vw.gh, w.params.d_min, w.params.d_max)
                        for v, vw in enumerate(w.rig.views)])
    iters = w.params.iterations
    host = host_cpus()
    # one thread per core of the process's CPU affinity, at most 16 (a one-GPU share of the host)
    cores = max(1, min(host["affinity"], 16))

    def one(job):
        v, s = job
        orc.sweep_sp(v, s)
        n = w.params.levels
        for it in range(1, iters + 1):
            n += len(orc.refine_trace(A, it, v, s, cap=1024)[0])
        return n

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=cores) as ex:
        evals = sum(ex.map(one, jobs))
    dt = time.perf_counter() - t0
    return {"value": evals / dt, "unit": "evals/s", "cores": cores, "kind": "oracle",
            "sample": "%d superpixels of the full-HD workload: %d-level sweep + %d refinement iterations each "
                      "(refinement from a seeded plane state); %.1f s wall on %d threads (host: %d CPUs, %d in "
                      "this process's affinity, %s)" % (n_sp, w.params.levels, iters, dt, cores, host["nproc"],
                                                       host["affinity"], host["model"]),
            "host": host, "seconds": dt}


def host_cpus():
    """CPU count of the machine, of this process's affinity mask, and the model name."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return {"nproc": os.cpu_count() or 1, "affinity": aff, "model": model}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: runs on one GPU only; --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.issue_rates:
        import subprocess

        probe = os.path.join(ROOT, "paper_1812_06856_amd", "_build", "issue_rates")
        if not os.path.exists(probe):
            sys.exit("bench.py: %s is not built (paper_1812_06856_amd/build.py builds it)" % probe)
        sys.exit(subprocess.run([probe]).returncode)
    if args.copy_calibration_mib:
        copy_calibration(args.copy_calibration_mib)
        return
    if args.workload != "fullhd":
        {"precision": run_precision, "batched": run_batched, "serving": run_serving, "sensitivity": run_sensitivity,
         "temporal": run_temporal}[args.workload](args)
        return
    import numpy as np
    import torch

    from lfsynth import config2
    from paper_1812_06856_amd import slf

    w = config2()
    p = w.params
    V = w.rig.n_views
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    ctx = slf.Context(0)
    ctx.set_stream(stream)
    vs = w.rig.views
    ctx.set_cameras([(v.W, v.H) for v in vs], [v.K for v in vs], [v.R for v in vs], [v.t for v in vs])
    ctx.set_params(slf.params_from(p, image_precision=args.image_precision))
    with torch.cuda.stream(stream):
        imgs = [torch.from_numpy(v.rgb).to(dev) for v in vs]
        labs = [torch.from_numpy(v.labels).to(dev) for v in vs]
        depth = torch.empty((V, vs[0].H, vs[0].W), dtype=torch.float32, device=dev)
    stream.synchronize()
    for i, v in enumerate(vs):
        ctx.grids[i] = (v.gw, v.gh)

    ev = {}

    def rec(name):
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        ev.setdefault(name, []).append(e)

    def step(timed_events):
        if timed_events:
            rec("setup0")
        for i in range(V):
            ctx.set_image(i, imgs[i])
            ctx.set_labels(i, labs[i], vs[i].gw, vs[i].gh)
        ctx.prepare()  # texels + superpixel lists
        if timed_events:
            rec("sweep0")
        ctx.sweep()
        if timed_events:
            rec("sweep1")
        for it in range(1, p.iterations + 1):
            if timed_events:
                rec("ref%d_0" % it)
            ctx.propagate(it, 1)
            if timed_events:
                rec("ref%d_1" % it)
        for i in range(V):
            ctx.get_depth(i, out=depth[i])
        if timed_events:
            rec("end")

    for _ in range(args.warmup):
        step(False)
    ctx.synchronize()
    torch.cuda.synchronize()
    ctx.reset_work()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    ctx.synchronize()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    evals, samples, pruned = ctx.work_detail()
    sweep_computed, sweep_total = ctx.sweep_work()
    K = args.steps
    sweep_evals_frame = sweep_evals_per_frame(ctx, w)
    sweep_scored, sweep_decided = ctx.sweep_levels()
    # depth fusion of the frame's refined depth maps (Sec. III-D), timed on its own
    ctx.fuse(FUSE_TOL)
    for _ in range(K):
        rec("fuse0")
        ctx.fuse(FUSE_TOL)
        rec("fuse1")
    torch.cuda.synchronize()

    def span(a, b):
        return [ev[a][k].elapsed_time(ev[b][k]) for k in range(K)]

    # GPU SLIC of every view of the frame (Sec. III-A; the step before the hot path), timed on its own
    for _ in range(K):
        rec("seg0")
        for i in range(V):
            ctx.segment(i, vs[i].gw, vs[i].gh, SLIC_ITERATIONS, SLIC_COMPACTNESS)
        rec("seg1")
    torch.cuda.synchronize()
    t_seg = span("seg0", "seg1")
    t_fuse = span("fuse0", "fuse1")
    t_setup = span("setup0", "sweep0")
    t_sweep = span("sweep0", "sweep1")
    t_ref = [span("ref%d_0" % it, "ref%d_1" % it) for it in range(1, p.iterations + 1)]
    ms_ref_total = float(np.mean([sum(t_ref[i][k] for i in range(len(t_ref))) for k in range(K)]))

    # per-step work: px-view samples computed (the sweep's level bound skips
    # samples of levels that can be neither chosen nor second best)
    n_pairs = V - 1
    sweep_samples = sweep_computed // K
    refine_samples = samples // K - sweep_samples
    sweep_ms = float(np.mean(t_sweep))
    ref_ms = ms_ref_total
    ops_sweep = OPS_PER_SAMPLE_SWEEP * sweep_samples
    ops_ref = OPS_PER_SAMPLE_REFINE * refine_samples
    k_ref = {"kernel": "k_refine", "ops": ops_ref, "ms": ref_ms, "launches": p.iterations,
             "ops_per_sample": OPS_PER_SAMPLE_REFINE}
    k_swp = {"kernel": "k_sweep", "ops": ops_sweep, "ms": sweep_ms, "launches": 1,
             "ops_per_sample": OPS_PER_SAMPLE_SWEEP}
    dom, other = (k_ref, k_swp) if ref_ms >= sweep_ms else (k_swp, k_ref)
    achieved = dom["ops"] / (dom["ms"] * 1e-3) / 1e12
    peak = PEAK_VALU_OPS / 1e12
    other_achieved = other["ops"] / (other["ms"] * 1e-3) / 1e12

    out = {
        "metric": "SP-plane hypothesis evals/s",
        "value": evals / dt,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": dt / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "views": V, "resolution": "1920x1080", "grid": "103x58",
                   "superpixels_per_view": 5974, "levels": p.levels, "iterations": p.iterations,
                   "neighbour_views": n_pairs, "image_storage": ["u8", "f16", "f32"][args.image_precision]},
        "ms_per_view": dt / K * 1e3 / V,
        "px_view_samples_per_s": samples / dt,
        "evals_per_step": evals // K,
        "refine_candidates_pruned_per_step": pruned // K,
        "sweep_samples_computed_frac": sweep_computed / max(1, sweep_total),
        "stage_ms": {"setup": float(np.mean(t_setup)), "sweep": sweep_ms, "refine_total": ref_ms,
                     "refine_per_iteration": [float(np.mean(t)) for t in t_ref]},
        "refine_candidates_scored_in_full_per_s": (evals - pruned - K * sweep_evals_frame) / dt,
        "hypotheses_scored_in_full_per_s": (sweep_scored + evals - pruned - sweep_decided) / dt,
        "sweep_levels_scored_frac": sweep_scored / max(1, sweep_decided),
        "fusion": fusion_record(w, float(np.mean(t_fuse))),
        "segmentation": {"ms": float(np.mean(t_seg)), "ms_per_view": float(np.mean(t_seg)) / V,
                         "iterations": SLIC_ITERATIONS, "compactness": SLIC_COMPACTNESS, "grid": [vs[0].gw, vs[0].gh]},
        "roofline": {"bound": "alu", "kernel": dom["kernel"], "achieved": achieved, "peak": peak,
                     "unit": "Tops/s", "frac": achieved / peak, "traffic": hbm_traffic(dom["kernel"]),
                     "traffic_unit": "HBM bytes per launch",
                     "ops_per_sample": dom["ops_per_sample"], "launches_per_step": dom["launches"]},
        # the same figures for the other hot kernel
        "roofline_other": {"bound": "alu", "kernel": other["kernel"], "achieved": other_achieved, "peak": peak,
                           "unit": "Tops/s", "frac": other_achieved / peak, "traffic": hbm_traffic(other["kernel"]),
                           "traffic_unit": "HBM bytes per launch", "ops_per_sample": other["ops_per_sample"],
                           "launches_per_step": other["launches"]},
    }
    if not args.no_cpu_baseline:
        cb = cpu_baseline(w, args.cpu_sample)
        cb.pop("seconds", None)
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


def _load_rig_inputs(ctx, w, dev, stream, image_precision):
    """Cameras and params on ctx; images and labels copied to device tensors."""
    import torch

    from paper_1812_06856_amd import slf

    vs = w.rig.views
    ctx.set_cameras([(v.W, v.H) for v in vs], [v.K for v in vs], [v.R for v in vs], [v.t for v in vs])
    ctx.set_params(slf.params_from(w.params, image_precision=image_precision))
    with torch.cuda.stream(stream):
        imgs = [torch.from_numpy(v.rgb).to(dev) for v in vs]
        labs = [torch.from_numpy(v.labels).to(dev) for v in vs]
        depth = [torch.empty((v.H, v.W), dtype=torch.float32, device=dev) for v in vs]
    for i, v in enumerate(vs):
        ctx.grids[i] = (v.gw, v.gh)
    return imgs, labs, depth


def run_precision(args):
    """Precision form on the 4x4 720p workload (192 levels, 6 iterations): the
    whole path timed with each image storage form (f32: the plain FP32 form;
    f16: FP16 texels, FP32 accumulation, FP64 composition; u8: exact 8-bit
    texels), alone and through a rig pool, and each form's end-to-end depth
    maps compared with the FP64 oracle's.  The oracle's final planes come from
    tests/golden/oracle_state_precision.npz (written by the oracle alone) and
    are read out to depth by the oracle."""
    import numpy as np
    import torch

    from lfsynth import config3
    from paper_1812_06856_amd import slf

    w = config3()
    p = w.params
    vs = w.rig.views
    V = len(vs)
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    ref_path = os.path.join(ROOT, "tests", "golden", "oracle_state_precision.npz")
    orc_depth = None
    if os.path.exists(ref_path):
        from oracle.oracle import Oracle

        ref = np.load(ref_path)
        orc = Oracle(w.rig, p)
        planes = ref["planes"].astype(np.float64)
        orc_depth = [orc.render_depth(planes, v) for v in range(V)]

    def ev():
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        return e

    forms = {}
    for name, fmt in [("f32", slf.SLF_IMAGE_F32), ("f16", slf.SLF_IMAGE_F16), ("u8", slf.SLF_IMAGE_U8)]:
        _progress("precision form %s" % name)
        ctx = slf.Context(0)
        ctx.set_stream(stream)
        imgs, labs, depth = _load_rig_inputs(ctx, w, dev, stream, fmt)

        def load():
            for i, v in enumerate(vs):
                ctx.set_image(i, imgs[i])
                ctx.set_labels(i, labs[i], v.gw, v.gh)
            ctx.prepare()

        def solo():
            load()
            e0 = ev()
            ctx.sweep()
            ctx.propagate(1, p.iterations)
            for i in range(V):
                ctx.get_depth(i, out=depth[i])
            return e0, ev()

        for _ in range(args.warmup):
            solo()
        torch.cuda.synchronize()
        ctx.reset_work()
        marks = [solo() for _ in range(args.steps)]
        torch.cuda.synchronize()
        evals, samples = ctx.work()
        ms = float(np.mean([a.elapsed_time(b) for a, b in marks]))
        d_solo = [depth[i].cpu().numpy() for i in range(V)]
        pool = slf.Pool(0)
        pool.set_stream(stream)
        pool.attach(ctx)

        def pooled():
            load()
            e0 = ev()
            pool.submit(ctx, slf.SLF_POOL_SOLVE, 1, p.iterations, 0)
            pool.run()
            for i in range(V):
                ctx.get_depth(i, out=depth[i])
            return e0, ev()

        for _ in range(args.warmup):
            pooled()
        pmarks = [pooled() for _ in range(args.steps)]
        torch.cuda.synchronize()
        pool.poll(64)
        pool_ms = float(np.mean([a.elapsed_time(b) for a, b in pmarks]))
        same = all(np.array_equal(d_solo[i], depth[i].cpu().numpy()) for i in range(V))
        rec = {"ms_per_frame": ms, "ms_per_view": ms / V, "pooled_ms_per_frame": pool_ms,
               "pooled_equals_solo": bool(same), "evals_per_s": evals / args.steps / (ms / 1e3),
               "px_view_samples_per_s": samples / args.steps / (ms / 1e3)}
        if orc_depth is not None:
            rel = np.concatenate([np.abs(d_solo[i][m] - orc_depth[i][m]) / orc_depth[i][m]
                                  for i in range(V) for m in [(orc_depth[i] > 0) & (d_solo[i] > 0)]])
            rec.update({"depth_mare_vs_oracle": float(rel.mean()), "depth_p99_rel_vs_oracle": float(np.percentile(rel, 99)),
                        "frac_px_over_0p5pct": float((rel > 5e-3).mean())})
        forms[name] = rec
        pool.close()
        ctx.close()
    out = {
        "metric": "SP-plane hypothesis evals/s", "value": forms["f16"]["evals_per_s"], "unit": "evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": forms["f16"]["ms_per_frame"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "views": V, "resolution": "1280x720", "levels": p.levels,
                   "iterations": p.iterations, "image_storage": "f16", "parallelism": "none"},
        "forms": forms,
        # the plain path stores its 8-bit images exactly as RGBA8 texels (u8): that is the form to beat;
        # a ratio below 1 means the FP16 form is slower
        "plain_storage": "u8",
        "f16_vs_u8_speedup": forms["u8"]["ms_per_frame"] / forms["f16"]["ms_per_frame"],
        "pooled_f16_vs_solo_u8_speedup": forms["u8"]["ms_per_frame"] / forms["f16"]["pooled_ms_per_frame"],
        "f16_vs_f32_storage_speedup": forms["f32"]["ms_per_frame"] / forms["f16"]["ms_per_frame"],
        "oracle_reference": os.path.relpath(ref_path, ROOT) if orc_depth is not None else None,
    }
    print(json.dumps(out), flush=True)


def run_batched(args):
    """Batched form: 32 independent rigs (3-16 views, 640x480 to 1920x1080,
    128-256 levels) solved together through one rig pool.  One step = every
    rig's texel and superpixel setup, the pooled sweep and 3 pooled refinement
    iterations (one HIP-graph replay of persistent launches) and the depth
    readout of every view.  The same rigs run one after another through the
    per-rig calls give the solo time beside it."""
    import numpy as np
    import torch

    from lfsynth import configs
    from paper_1812_06856_amd import slf

    t_gen = time.perf_counter()
    ws = []
    for j in range(args.rigs):
        ws.append(configs.rig_batched(j))
        _progress("generated %s" % ws[-1].rig.name)
    t_gen = time.perf_counter() - t_gen
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    pool = slf.Pool(0)
    pool.set_stream(stream)
    ctxs, inputs = [], []
    for w in ws:
        c = slf.Context(0)
        c.set_stream(stream)
        inputs.append(_load_rig_inputs(c, w, dev, stream, args.image_precision))
        ctxs.append(c)
    stream.synchronize()

    def load_and_prepare():
        for c, w, (imgs, labs, _) in zip(ctxs, ws, inputs):
            for i, v in enumerate(w.rig.views):
                c.set_image(i, imgs[i])
                c.set_labels(i, labs[i], v.gw, v.gh)
            c.prepare()

    def readout():
        for c, (_, _, depth) in zip(ctxs, inputs):
            for i in range(len(depth)):
                c.get_depth(i, out=depth[i])

    load_and_prepare()
    for c in ctxs:
        pool.attach(c)
    _progress("autotuning")
    t_tune = time.perf_counter()
    pool.autotune()
    t_tune = time.perf_counter() - t_tune
    _progress("autotuned in %.1f s: %s" % (t_tune, pool.get_config().as_dict()))
    cfg = pool.get_config().as_dict()

    def ev():
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        return e

    def pooled_step():
        e0 = ev()
        load_and_prepare()
        e1 = ev()
        for j, (c, w) in enumerate(zip(ctxs, ws)):
            pool.submit(c, slf.SLF_POOL_SOLVE, 1, w.params.iterations, j)
        pool.run()
        e2 = ev()
        readout()
        e3 = ev()
        return e0, e1, e2, e3

    def solo_step():
        e0 = ev()
        load_and_prepare()
        e1 = ev()
        for c, w in zip(ctxs, ws):
            c.sweep()
            c.propagate(1, w.params.iterations)
        e2 = ev()
        readout()
        e3 = ev()
        return e0, e1, e2, e3

    for _ in range(args.warmup):
        pooled_step()
        solo_step()
    torch.cuda.synchronize()
    _progress("warm-up done")
    for c in ctxs:
        c.reset_work()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    marks = [pooled_step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    pool.poll(4096)
    evals = sum(c.work()[0] for c in ctxs)
    samples = sum(c.work()[1] for c in ctxs)
    solo = [solo_step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    step_ms = [m[0].elapsed_time(m[3]) for m in marks]
    solve_ms = [m[1].elapsed_time(m[2]) for m in marks]
    solo_solve_ms = [m[1].elapsed_time(m[2]) for m in solo]
    ms = float(np.mean(step_ms))
    n_views = sum(w.rig.n_views for w in ws)
    out = {
        "metric": "SP-plane hypothesis evals/s", "value": evals / args.steps / (ms / 1e3), "unit": "evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batched-%drigs" % len(ws), "rigs": [w.rig.name for w in ws],
                   "views": n_views, "levels": [w.params.levels for w in ws], "iterations": 3,
                   "image_precision": args.image_precision, "parallelism": "none"},
        "px_view_samples_per_s": samples / args.steps / (ms / 1e3),
        "stage_ms": {"setup": float(np.mean([m[0].elapsed_time(m[1]) for m in marks])),
                     "pooled_solve": float(np.mean(solve_ms)),
                     "readout": float(np.mean([m[2].elapsed_time(m[3]) for m in marks])),
                     "solo_solve": float(np.mean(solo_solve_ms))},
        "pooled_vs_solo": float(np.mean(solo_solve_ms) / np.mean(solve_ms)),
        "pool_config": cfg, "autotune_s": t_tune, "input_generation_s": t_gen,
        "wall_s": dt,
    }
    print(json.dumps(out), flush=True)


def run_serving(args):
    """Serving form: 6 rigs drawn as in the batched workload (FP16 texels,
    0.05 grid spacing) film moving scenes; frames arrive as one Poisson stream
    (rig chosen uniformly).  A rig's first frame is solved in full (sweep + 3
    iterations); later frames warm-start from the rig's previous planes and run
    2 iterations.  Requests share the pool and join its stages as they come
    (continuous batching).  Latency = arrival to the depth maps of all the
    frame's views in device memory.  Runs every rate of --serve-rates in turn
    (frames of a rig served in order), then the --serve-rate stream with a
    latest-frame policy (a rig that frees up takes its newest waiting frame
    and drops older ones), then times one cold solve and one warm frame of
    each rig alone."""
    import numpy as np
    import torch

    from lfsynth import configs
    from paper_1812_06856_amd import serve as serving
    from paper_1812_06856_amd import slf

    t_gen = time.perf_counter()
    seqs = [configs.serving_rig(j) for j in range(args.serve_rigs)]
    F = args.serve_frames
    frames = []
    for s in seqs:
        frames.append([s.frame(k) for k in range(F)])
        _progress("rendered %d frames of %s" % (F, s.name))
    t_gen = time.perf_counter() - t_gen
    dev = torch.device("cuda:0")
    pool = slf.Pool(0)
    streams, ctxs, data, depth = [], [], [], []
    for j, s in enumerate(seqs):
        st = torch.cuda.Stream(device=dev)
        c = slf.Context(0)
        c.set_stream(st)
        w0 = configs.Workload(s.name, frames[j][0], s.params)
        _, _, dep = _load_rig_inputs(c, w0, dev, st, 1)
        with torch.cuda.stream(st):
            data.append([([torch.from_numpy(v.rgb).to(dev) for v in fr.views],
                          [torch.from_numpy(v.labels).to(dev) for v in fr.views]) for fr in frames[j]])
        for i, v in enumerate(frames[j][0].views):  # frame 0 inputs: the label grids the footprint needs
            c.set_image(i, data[j][0][0][i])
            c.set_labels(i, data[j][0][1][i], v.gw, v.gh)
        streams.append(st)
        ctxs.append(c)
        depth.append(dep)
        pool.attach(c)
    torch.cuda.synchronize()
    footprints = [c.footprint() for c in ctxs]
    iters_warm = 2
    n_frame = [0] * len(seqs)
    period = 2 * (F - 1)

    def next_frame(j):
        """Index of rig j's next frame: frames 0 .. F-1 .. 1 .. played back and forth."""
        k = n_frame[j]
        n_frame[j] += 1
        return k % period if k % period < F else period - k % period

    def serve(rate, seconds, warmup_s, latest_only, seed):
        rng = np.random.default_rng(seed)
        horizon = warmup_s + seconds
        arrivals = serving.poisson_arrivals(rate, horizon, len(seqs), rng)
        srv = serving.Server(pool, latest_only=latest_only)
        for j, c in enumerate(ctxs):
            srv.add_rig(c, streams[j], depth[j], seqs[j].params.iterations, iters_warm)
            srv.rigs[j].has_state = n_frame[j] > 0
        latency = []
        a = 0
        samples0 = sum(c.work()[1] for c in ctxs)
        _progress("rate %.0f/s%s: %d arrivals over %.0f s" % (rate, " (latest frame)" if latest_only else "",
                                                            len(arrivals), horizon))
        t0 = time.perf_counter()
        srv.clock = lambda: time.perf_counter() - t0
        next_report = 5.0
        while a < len(arrivals) or srv.busy():
            now = srv.clock()
            while a < len(arrivals) and arrivals[a][0] <= now:
                t_arr, j = arrivals[a]
                fk = next_frame(j)
                srv.submit(j, fk, data[j][fk][0], data[j][fk][1], arrival=t_arr)
                a += 1
            for d in srv.tick():
                if d.arrival >= warmup_s:
                    latency.append(d.latency_ms)
            if now >= next_report:
                _progress("  t=%.0f s: %d arrived, %d measured" % (now, a, len(latency)))
                next_report += 5.0
            if not pool.usage()["active"]:
                time.sleep(0.0002)
        wall = time.perf_counter() - t0
        lat = np.array(latency) if latency else np.array([np.nan])
        offered = sum(1 for x in arrivals if x[0] >= warmup_s)
        return {"rate_fps": rate, "policy": "latest frame" if latest_only else "every frame",
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "max_ms": float(np.max(lat)), "frames_measured": int(len(latency)), "frames_offered": offered,
                "dropped": srv.dropped, "served_fps": len(latency) / seconds,
                "px_view_samples_per_s": (sum(c.work()[1] for c in ctxs) - samples0) / wall, "wall_s": wall}

    rates = [float(x) for x in args.serve_rates.split(",")]
    results = []
    for i, rate in enumerate(rates):
        results.append(serve(rate, args.serve_seconds, args.serve_warmup_s, False, args.serve_seed + i))
        _progress("rate %.0f/s: p50 %.1f ms, p99 %.1f ms" % (rate, results[-1]["p50_ms"], results[-1]["p99_ms"]))
    latest = serve(args.serve_rate, args.serve_seconds, args.serve_warmup_s, True, args.serve_seed + 100)
    _progress("latest-frame policy at %.0f/s: p50 %.1f ms, p99 %.1f ms, dropped %d"
              % (args.serve_rate, latest["p50_ms"], latest["p99_ms"], latest["dropped"]))

    # one cold solve and one warm frame of each rig alone (per-rig calls)
    pool.synchronize()
    def load_frame(j):
        fk = next_frame(j)
        imgs, labs = data[j][fk]
        for i, v in enumerate(frames[j][fk].views):
            ctxs[j].set_image(i, imgs[i])
            ctxs[j].set_labels(i, labs[i], v.gw, v.gh)

    solo = []
    for j, c in enumerate(ctxs):
        st = streams[j]
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record(st)
        load_frame(j)
        c.prepare()
        c.sweep()
        c.propagate(1, seqs[j].params.iterations)
        e1.record(st)
        load_frame(j)
        c.warm_start()
        c.propagate(1, iters_warm)
        e2.record(st)
        st.synchronize()
        solo.append({"rig": seqs[j].name, "cold_ms": e0.elapsed_time(e1), "warm_ms": e1.elapsed_time(e2)})
    ok = [r for r in results if r["p99_ms"] <= args.serve_p99_bound_ms]
    best = max(ok, key=lambda r: r["rate_fps"]) if ok else min(results, key=lambda r: r["p99_ms"])
    out = {
        "metric": "served frame latency p99", "value": best["p99_ms"], "unit": "ms",
        "n_gpus": 1, "steps": best["frames_measured"], "warmup": 0, "ms_per_step": best["p50_ms"],
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "serving-%drigs" % len(seqs), "rigs": [s.name for s in seqs],
                   "rate_fps": best["rate_fps"], "seconds": args.serve_seconds, "warm_iterations": iters_warm,
                   "image_precision": 1, "p99_bound_ms": args.serve_p99_bound_ms, "parallelism": "none"},
        "p50_ms": best["p50_ms"], "p99_ms": best["p99_ms"], "rates": results, "latest_frame_policy": latest,
        "solo_cold_vs_warm": solo, "footprint_bytes": footprints, "input_generation_s": t_gen,
    }
    print(json.dumps(out), flush=True)

def run_sensitivity(args):
    """Fig. 5 / Fig. 6 analogues on a Middlebury-like synthetic rig (9 rectified
    views of 450x375, 80 levels) with ground-truth depth: bad-pixel rates (1 px
    and 0.5 px of disparity towards the nearest camera) and GPU time against
    the number of iterations, the superpixel size, the kernel step and the
    initial kernel radius, and with each energy term left out."""
    from lfsynth.configs import sensitivity_rig
    from paper_1812_06856_amd import experiments

    t0 = time.perf_counter()
    out = experiments.sensitivity(lambda sp: sensitivity_rig(sp))
    base = out["vs_iterations"][5]
    print(json.dumps({"metric": "bad pixels (1 px disparity)", "value": base["bad_1"], "unit": "fraction",
                      "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": base["total_ms"],
                      "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
                      "data": "synthetic", "config": {"workload": out["workload"], "iterations": 5},
                      "sensitivity": out, "wall_s": time.perf_counter() - t0}), flush=True)


def run_temporal(args):
    """Temporal consistency on the serving rigs' video (Sec. IV-F): flicker of
    static scene parts between consecutive frames, each frame solved on its own
    against the warm-started serving form."""
    import numpy as np

    from lfsynth import configs
    from paper_1812_06856_amd import experiments

    recs = []
    for j in range(args.temporal_rigs):
        seq = configs.serving_rig(j)
        _progress("temporal %s" % seq.name)
        recs.append(experiments.temporal_consistency(seq, args.temporal_frames))
    cold = float(np.mean([r["cold"]["mean_flicker"] for r in recs])) if recs else float("nan")
    warm = float(np.mean([r["warm"]["mean_flicker"] for r in recs])) if recs else float("nan")
    print(json.dumps({"metric": "static-region flicker (mean relative frame difference)", "value": warm,
                      "unit": "fraction", "n_gpus": 1, "steps": args.temporal_frames, "warmup": 0, "ms_per_step": None,
                      "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
                      "data": "synthetic", "config": {"workload": "serving-video", "rigs": [r["sequence"] for r in recs]},
                      "cold_flicker": cold, "warm_flicker": warm, "rigs": recs}), flush=True)


if __name__ == "__main__":
    main()
