"""Accuracy experiments on synthetic light fields with ground-truth depth.

The paper measures its parameter sensitivity and the effect of each energy
term on Middlebury scenes (Sec. IV-A, Fig. 5; Sec. IV-C, Fig. 6) and the
temporal stability of its depth on video (Sec. IV-F).  Here the ground truth
comes from the ray-cast synthetic scenes: the error of a depth map is the
share of bad pixels, whose disparity towards the nearest other camera is off
by more than a threshold (1 px and 0.5 px, as in the paper's bad-pixel
rates), and the mean relative depth error.

Every depth map comes from libslf (the sweep, the refinement iterations, the
readout); this module only sets parameters, reads the depth back and scores
it, and times the GPU stages with events on the context's stream.
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence

import numpy as np
import torch

from . import slf


def nearest_baseline(views, v: int) -> float:
    """Distance from camera v's centre to the nearest other camera centre."""
    C = [-np.asarray(x.R).T @ np.asarray(x.t) for x in views]
    return min(float(np.linalg.norm(C[v] - C[i])) for i in range(len(views)) if i != v)


def depth_errors(depth, gt, focal: float, baseline: float, thresholds=(1.0, 0.5)) -> Dict[str, float]:
    """Bad-pixel rates and mean relative error of one depth map against ground
    truth (pixels without ground truth are ignored; a missing estimate, depth
    <= 0, counts as bad).  Disparity error = focal * baseline * |1/d - 1/gt|."""
    gt = np.asarray(gt, np.float64)
    d = np.asarray(depth, np.float64)
    valid = gt > 0
    est = valid & (d > 0)
    err = np.full(gt.shape, np.inf)
    err[est] = focal * baseline * np.abs(1.0 / d[est] - 1.0 / gt[est])
    out = {"pixels": int(valid.sum()), "missing": float((valid & ~est).sum() / max(1, valid.sum()))}
    for t in thresholds:
        out["bad_%g" % t] = float((err[valid] > t).sum() / max(1, valid.sum()))
    rel = np.abs(d[est] - gt[est]) / gt[est]
    out["mare"] = float(rel.mean()) if rel.size else float("nan")
    return out


def rig_errors(depths: Sequence[np.ndarray], views) -> Dict[str, float]:
    """Pixel-weighted errors over all views of a rig."""
    per = [depth_errors(depths[v], views[v].gt_depth, float(views[v].K[0][0]), nearest_baseline(views, v))
           for v in range(len(views))]
    n = sum(p["pixels"] for p in per)
    out = {"pixels": n}
    for k in per[0]:
        if k != "pixels":
            out[k] = float(sum(p[k] * p["pixels"] for p in per) / max(1, n))
    return out


class _Timer:
    def __init__(self, stream):
        self.stream = stream
        self.marks = []

    def mark(self):
        e = torch.cuda.Event(enable_timing=True)
        e.record(self.stream)
        self.marks.append(e)

    def spans(self):
        self.stream.synchronize()
        return [a.elapsed_time(b) for a, b in zip(self.marks, self.marks[1:])]


def solve_with_history(workload, iterations: int, **param_overrides) -> List[Dict]:
    """Sweep then `iterations` refinement iterations of one rig on the GPU;
    after the sweep and after each iteration the depth maps are scored.  Each
    record holds the iteration (0 = the sweep), the errors and the GPU time of
    that stage and of all stages so far (ms)."""
    rig = workload.rig
    stream = torch.cuda.Stream()
    ctx = slf.Context(0)
    ctx.set_stream(stream)
    ctx.load_rig(rig, slf.params_from(workload.params, **param_overrides))
    ctx.prepare()
    tm = _Timer(stream)
    tm.mark()
    ctx.sweep()
    tm.mark()
    depths_per_stage = [[ctx.get_depth(v) for v in range(rig.n_views)]]
    for it in range(1, iterations + 1):
        tm.mark()
        ctx.propagate(it, 1)
        tm.mark()
        depths_per_stage.append([ctx.get_depth(v) for v in range(rig.n_views)])
    spans = tm.spans()
    stage_ms = [spans[0]] + [spans[2 * k] for k in range(1, iterations + 1)]
    out, total = [], 0.0
    for it, (ms, depths) in enumerate(zip(stage_ms, depths_per_stage)):
        total += ms
        rec = {"iteration": it, "stage_ms": ms, "total_ms": total}
        rec.update(rig_errors(depths, rig.views))
        out.append(rec)
    ctx.close()
    return out


def final(workload, iterations: int, **over) -> Dict:
    return solve_with_history(workload, iterations, **over)[-1]


def sensitivity(make_workload, sp_sizes=(50, 100, 200, 400), kernel_steps=(1, 2, 3, 5, 8),
                kernel_radii=(2, 5, 10, 20, 0), iterations: int = 5) -> Dict:
    """Fig. 5 and Fig. 6 analogues.  make_workload(sp_px) builds the rig with
    superpixels of about sp_px pixels (the same scene for every size)."""
    base = make_workload(100.0)
    out = {"workload": base.name, "iterations": iterations}
    out["vs_iterations"] = solve_with_history(base, 8)
    out["vs_superpixel_size"] = []
    for sp in sp_sizes:
        w = make_workload(float(sp))
        rec = final(w, iterations)
        rec["superpixel_px"] = sp
        rec["grid"] = [w.rig.views[0].gw, w.rig.views[0].gh]
        out["vs_superpixel_size"].append(rec)
    out["vs_kernel_step"] = []
    for st in kernel_steps:
        rec = final(base, iterations, kernel_step=st)
        rec["kernel_step"] = st
        out["vs_kernel_step"].append(rec)
    out["vs_kernel_radius"] = []
    for kr in kernel_radii:
        rec = final(base, iterations, kernel_radius_init=kr)
        rec["kernel_radius_init"] = kr  # 0: the smallest image dimension (the paper's default)
        out["vs_kernel_radius"].append(rec)
    out["energy_terms"] = []
    for name, mask in [("all terms", 7), ("without smoothness", 6), ("without consistency", 5),
                       ("without occlusion", 3)]:
        rec = final(base, iterations, term_mask=mask)
        rec["terms"] = name
        rec["term_mask"] = mask
        out["energy_terms"].append(rec)
    rec = final(base, iterations, energy_mode=1)
    rec["terms"] = "data term only (TSSD)"
    out["energy_terms"].append(rec)
    return out


def frame_difference(a, b, static) -> float:
    """Mean |a - b| / b over static pixels where both frames have a depth."""
    m = static & (a > 0) & (b > 0)
    return float((np.abs(a[m] - b[m]) / b[m]).mean()) if m.any() else float("nan")


def temporal_consistency(seq, frames: int, warm_iters: int = 2) -> Dict:
    """Flicker of the depth of static scene parts over a video (Sec. IV-F
    frame-difference maps): every frame solved on its own (sweep + the rig's
    iterations) against the serving form (the first frame solved, later
    frames warm-started from the previous planes with `warm_iters`
    iterations).  Static pixels: ground truth unchanged between consecutive
    frames.  Also the bad-pixel rate of both against ground truth."""
    rigs = [seq.frame(k) for k in range(frames)]
    V = rigs[0].n_views
    p = slf.params_from(seq.params)
    cold, warm = [], []
    ctx_c, ctx_w = slf.Context(0), slf.Context(0)
    for k, rig in enumerate(rigs):
        ctx_c.load_rig(rig, p)
        ctx_c.sweep()
        ctx_c.propagate(1, seq.params.iterations)
        cold.append([ctx_c.get_depth(v) for v in range(V)])
        if k == 0:
            ctx_w.load_rig(rig, p)
            ctx_w.sweep()
            ctx_w.propagate(1, seq.params.iterations)
        else:
            for v, view in enumerate(rig.views):
                ctx_w.set_image(v, view.rgb)
                ctx_w.set_labels(v, view.labels, view.gw, view.gh)
            ctx_w.warm_start()
            ctx_w.propagate(1, warm_iters)
        warm.append([ctx_w.get_depth(v) for v in range(V)])
    out = {"sequence": seq.name, "frames": frames, "warm_iterations": warm_iters,
           "cold": {"flicker": [], "bad_1": []}, "warm": {"flicker": [], "bad_1": []}, "static_frac": []}
    for k in range(frames):
        for name, seqd in (("cold", cold), ("warm", warm)):
            out[name]["bad_1"].append(rig_errors(seqd[k], rigs[k].views)["bad_1"])
        if k == 0:
            continue
        st = [(rigs[k].views[v].gt_depth == rigs[k - 1].views[v].gt_depth) & (rigs[k].views[v].gt_depth > 0)
              for v in range(V)]
        out["static_frac"].append(float(np.mean([s.mean() for s in st])))
        for name, seqd in (("cold", cold), ("warm", warm)):
            out[name]["flicker"].append(float(np.nanmean([frame_difference(seqd[k][v], seqd[k - 1][v], st[v])
                                                         for v in range(V)])))
    for name in ("cold", "warm"):
        out[name]["mean_flicker"] = float(np.mean(out[name]["flicker"])) if out[name]["flicker"] else float("nan")
        out[name]["mean_bad_1"] = float(np.mean(out[name]["bad_1"]))
    ctx_c.close()
    ctx_w.close()
    return out
