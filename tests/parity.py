"""GPU-vs-oracle parity checks (test infrastructure).

Tolerances (stated for the FP32 GPU path against the FP64 oracle):
  * discrete choices (sweep level, refinement slot) equal wherever the
    oracle's margin exceeds MARGIN = 1e-4 (normalised cost or energy units);
  * per-superpixel cost / energy within REL = 1e-3 relative + ABS = 1e-6;
  * centroid depth within DEPTH_REL = 0.5 %.
Where the margin is below MARGIN and the choices differ, the GPU's pick must
score within MARGIN of the oracle's best under the oracle's own arithmetic, and
its cost or energy and its centroid depth must match the oracle's for that same
level or slot.

The consistency energy takes discrete decisions per sample (the nearest pixel
of eq. 9, the visible / occluded split of eqs. 10-11).  A decision whose value
lies within FP32 rounding of its threshold may legitimately fall either way
on the GPU.  Where the energies disagree, the oracle's bound of what flipping
the decisions within FLIP_EPS_PX (nearest pixel) or FLIP_EPS_REL (split) of
their thresholds can change (Oracle.energy_flip_bound) widens the energy
tolerance and the margin of that candidate; it is 0 for candidates with no
such decision.
"""
from __future__ import annotations

import numpy as np

MARGIN = 1e-4
REL = 1e-3
ABS = 1e-6
DEPTH_REL = 5e-3
FLIP_EPS_PX = 1e-4   # the GPU's nearest-pixel decision is exact to about 1e-6 px
FLIP_EPS_REL = 1e-5  # its relative error of z and D(p^i) is about 1e-6


def close(a, b, rel=REL, abs_=ABS):
    return abs(a - b) <= rel * abs(b) + abs_


def gpu_state(ctx, n_views):
    out = [ctx.get_planes(v) for v in range(n_views)]
    return [np.concatenate([o[i] for o in out]) for i in range(4)]


def check_sweep(orc, ctx, sample=None, margin=MARGIN, rel=REL, abs_=ABS):
    """Compares the GPU's sweep output with the oracle's per superpixel.

    sample: None (all superpixels) or an iterable of (view, sp); margin and
    rel default to the FP32 path's bar.  Returns a report dict.
    """
    P_g, C_g, K_g, M_g = gpu_state(ctx, orc.V)
    area = orc.sp_stats()[0]
    if sample is None:
        sample = [(v, s) for v in range(orc.V) for s in range(int(orc.sp_off[v + 1] - orc.sp_off[v]))]
    rep = {"n": 0, "empty": 0, "mismatch_choice": 0, "near_tie_flips": 0, "bad": []}
    for v, s in sample:
        g = int(orc.sp_off[v]) + s
        if area[g] == 0:
            rep["empty"] += 1
            if K_g[g] != -1:
                rep["bad"].append((v, s, "empty cell has choice %d" % K_g[g]))
            continue
        rep["n"] += 1
        pl_o, c_o, k_o, m_o = orc.sweep_sp(v, s)
        k_g = int(K_g[g])
        if not (0 <= k_g < orc_levels(orc)):
            rep["bad"].append((v, s, "choice %d out of range" % k_g))
            continue
        c_o_at_g = orc.sweep_cost(v, s, [1.0 / orc.level_q(v, s, k_g), 0, 0, 1])
        if not close(float(C_g[g]), c_o_at_g, rel=rel, abs_=abs_):
            rep["bad"].append((v, s, "cost %.9g vs oracle %.9g at level %d" % (C_g[g], c_o_at_g, k_g)))
        d_o_at_g = 1.0 / orc.level_q(v, s, k_g)
        if abs(P_g[g, 0] - d_o_at_g) > DEPTH_REL * d_o_at_g or not np.allclose(P_g[g, 1:], [0, 0, 1]):
            rep["bad"].append((v, s, "plane %s vs depth %.9g" % (P_g[g], d_o_at_g)))
        if k_g != k_o:
            rep["mismatch_choice"] += 1
            if m_o > margin:
                rep["bad"].append((v, s, "level %d vs oracle %d with margin %.3g" % (k_g, k_o, m_o)))
            elif c_o_at_g - c_o > margin:
                rep["bad"].append((v, s, "near-tie pick %.9g worse than best %.9g" % (c_o_at_g, c_o)))
            else:
                rep["near_tie_flips"] += 1
        if m_o > margin and np.isfinite(M_g[g]) and M_g[g] < 0:
            rep["bad"].append((v, s, "negative margin"))
    return rep


def orc_levels(orc):
    return int(orc._params.levels)


def check_refine(orc, ctx, A64, it, B_o=None, E_o=None, K_o=None, M_o=None, sample=None):
    """One lockstep iteration: the GPU must already hold state A64 (rounded to FP32)
    and have run iteration `it`.  Compares against the oracle run from A64.

    A refinement step takes two argmax decisions: the propagation winner
    (which fixes the depth the triangle normals pivot at) and the final
    winner.  Where the oracle's propagation stage is a near-tie (margin <=
    MARGIN), every tied propagation candidate is a legitimate pivot; the GPU's
    result must then equal the oracle's outcome for one of them."""
    P_g, E_g, K_g, M_g = gpu_state(ctx, orc.V)
    area = orc.sp_stats()[0]
    if sample is None:
        sample = [(v, s) for v in range(orc.V) for s in range(int(orc.sp_off[v + 1] - orc.sp_off[v]))]
    rep = {"n": 0, "mismatch_choice": 0, "near_tie_flips": 0, "pivot_ties": 0, "flip_bound_used": 0, "bad": []}
    for v, s in sample:
        g = int(orc.sp_off[v]) + s
        if area[g] == 0:
            if K_g[g] != -1:
                rep["bad"].append((v, s, "empty cell has choice %d" % K_g[g]))
            continue
        rep["n"] += 1
        if B_o is None:
            pl_o, e_o, k_o, m_o = orc.refine_sp(A64, it, v, s)
        else:
            pl_o, e_o, k_o, m_o = B_o[g], E_o[g], K_o[g], M_o[g]
        k_g = int(K_g[g])
        e_g = float(E_g[g])
        if k_g == k_o and close(e_g, e_o) and abs(P_g[g, 0] - pl_o[0]) <= DEPTH_REL * pl_o[0]:
            continue
        rep["mismatch_choice"] += k_g != k_o

        def bound(plane, _v=v, _s=s):
            return orc.energy_flip_bound(A64, _v, _s, plane, FLIP_EPS_PX, FLIP_EPS_REL)

        slots, planes, ens = orc.refine_trace(A64, it, v, s, cap=1024)
        prop = np.nonzero(slots < 1000)[0]
        order = prop[np.argsort(-ens[prop], kind="stable")]
        best = order[0]
        prop_margin = ens[order[0]] - ens[order[1]] if len(order) > 1 else np.inf
        b_best = bound(planes[best]) if prop_margin <= MARGIN + 1.0 else 0.0
        tied = [int(slots[c]) for c in order[1:]
                if ens[best] - ens[c] <= MARGIN + b_best + (bound(planes[c]) if ens[best] - ens[c] <= MARGIN + 1.0 else 0.0)]
        if not tied:
            outcomes = [(k_o, e_o, pl_o, slots, planes, ens)]
        else:  # the pivot itself is a near-tie: every tied propagation candidate may pivot
            rep["pivot_ties"] += 1
            outcomes = []
            for c in [int(slots[best])] + tied:
                pl_c, e_c, k_c, sl_c, pls_c, en_c = orc.refine_pivot(A64, it, v, s, c)
                outcomes.append((k_c, e_c, pl_c, sl_c, pls_c, en_c))
        ok = False
        used_bound = False
        why = ""
        for k_c, e_c, pl_c, sl_c, pls_c, en_c in outcomes:
            if k_g == k_c:
                if abs(P_g[g, 0] - pl_c[0]) <= DEPTH_REL * pl_c[0]:
                    if close(e_g, e_c):
                        ok = True
                        break
                    b = bound(pl_c)
                    if abs(e_g - e_c) <= REL * abs(e_c) + ABS + b:
                        ok = used_bound = True
                        break
                why = "slot %d: energy %.9g vs %.9g, depth %.7g vs %.7g" % (k_g, e_g, e_c, P_g[g, 0], pl_c[0])
                continue
            hit = np.nonzero(sl_c == k_g)[0]
            if len(hit) == 0:
                why = why or "GPU slot %d not among the oracle's candidates" % k_g
                continue
            e_at = en_c[hit[-1]]
            d_at = pls_c[hit[-1]][0]  # the oracle's plane for the GPU's slot: its depth must match too
            if abs(P_g[g, 0] - d_at) <= DEPTH_REL * d_at:
                if e_c - e_at <= MARGIN and close(e_g, e_at):
                    ok = True
                    break
                b_at, b_c = bound(pls_c[hit[-1]]), bound(pl_c)
                if e_c - e_at <= MARGIN + b_at + b_c and abs(e_g - e_at) <= REL * abs(e_at) + ABS + b_at:
                    ok = used_bound = True
                    break
            why = "slot %d (E %.9g, depth %.7g; oracle there E %.9g, depth %.7g) vs oracle slot %d (E %.9g)" % (
                k_g, e_g, P_g[g, 0], e_at, d_at, k_c, e_c)
        if ok:
            rep["near_tie_flips"] += 1
            rep["flip_bound_used"] += used_bound
        else:
            rep["bad"].append((v, s, why + " [final margin %.3g, pivot margin %.3g]" % (m_o, prop_margin)))
    return rep


def round_state(A):
    """State as the GPU holds it: FP32 values, back in FP64 for the oracle."""
    return np.asarray(A, np.float32).astype(np.float64)


def depth_mare(D_g, D_o):
    m = (D_o > 0) & (D_g > 0)
    rel = np.abs(D_g[m] - D_o[m]) / D_o[m]
    return float(rel.mean()) if rel.size else 0.0, rel
