#!/usr/bin/env python3
"""Benchmark: superpixel-plane matching cost on the full-HD 8-view workload.

One step = the whole depth path on one multi-view frame whose images and
labels are already resident in device memory: texel build and superpixel
setup, the 256-level plane sweep of every superpixel of every view, 8
refinement iterations over all views, and the depth readout of every view.

Prints ONE JSON line (metric: SP-plane hypothesis evaluations per second).
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
# Non-packed FP32 VALU lane-ops/s of MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz.
PEAK_VALU_OPS = 256 * 4 * 16 * 2.4e9


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1024, help="superpixels in the oracle's timed sample")
    ap.add_argument("--image-precision", type=int, default=0)
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
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    cores = max(1, min(cores, 16))

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
                      "(refinement from a seeded plane state); %.1f s wall" % (n_sp, w.params.levels, iters, dt),
            "seconds": dt}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration_mib:
        copy_calibration(args.copy_calibration_mib)
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
    evals, samples = ctx.work()
    K = args.steps

    def span(a, b):
        return [ev[a][k].elapsed_time(ev[b][k]) for k in range(K)]

    t_setup = span("setup0", "sweep0")
    t_sweep = span("sweep0", "sweep1")
    t_ref = [span("ref%d_0" % it, "ref%d_1" % it) for it in range(1, p.iterations + 1)]
    ms_ref_total = float(np.mean([sum(t_ref[i][k] for i in range(len(t_ref))) for k in range(K)]))

    # per-step algorithmic work
    area = np.concatenate([ctx.get_superpixels(i)[0] for i in range(V)])
    n_pairs = V - 1
    sweep_samples = int(area.sum()) * n_pairs * p.levels
    refine_samples = samples // K - sweep_samples
    sweep_ms = float(np.mean(t_sweep))
    ref_ms = ms_ref_total
    ops_sweep = OPS_PER_SAMPLE_SWEEP * sweep_samples
    ops_ref = OPS_PER_SAMPLE_REFINE * refine_samples
    if ref_ms >= sweep_ms:
        dom = {"kernel": "k_refine", "ops": ops_ref, "ms": ref_ms, "launches": p.iterations,
               "ops_per_sample": OPS_PER_SAMPLE_REFINE}
    else:
        dom = {"kernel": "k_sweep", "ops": ops_sweep, "ms": sweep_ms, "launches": 1,
               "ops_per_sample": OPS_PER_SAMPLE_SWEEP}
    achieved = dom["ops"] / (dom["ms"] * 1e-3) / 1e12
    peak = PEAK_VALU_OPS / 1e12

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
        "stage_ms": {"setup": float(np.mean(t_setup)), "sweep": sweep_ms, "refine_total": ref_ms,
                     "refine_per_iteration": [float(np.mean(t)) for t in t_ref]},
        "roofline": {"bound": "alu", "kernel": dom["kernel"], "achieved": achieved, "peak": peak,
                     "unit": "Tops/s", "frac": achieved / peak, "traffic": None,
                     "ops_per_sample": dom["ops_per_sample"], "launches_per_step": dom["launches"]},
    }
    if not args.no_cpu_baseline:
        cb = cpu_baseline(w, args.cpu_sample)
        cb.pop("seconds", None)
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
