"""Pins of the oracle's superpixel statistics and of the sweep-cost normalisation.

The superpixel centroid c_s (Sec. III-A: a plane is held as the depth at the
centroid plus a normal) enters every plane the refinement extrapolates to a
neighbour's centroid (Sec. III-C-1, eqs. 5-6), and the normalised sweep cost
divides eq. (2)'s sum over the neighbour views and the superpixel's pixels by
|Omega| |N(r)| T.  The expected values here never come from the oracle's own
statistics: centroids are pixel means taken with numpy from the label map, or
the analytic centre of a rectangle of pixels, and costs are closed forms.
"""
from __future__ import annotations

import numpy as np
import pytest

from lfsynth import config1
from oracle.oracle import Oracle
from tests.microrig import view, rig, params


def _rect_labels(W, H, xcuts, ycuts):
    """Label map of a grid of axis-aligned rectangles with the given column and
    row cut positions (cell k = (k mod gw, k div gw)); cells are unequal."""
    gx = np.searchsorted(np.asarray(xcuts[1:-1]), np.arange(W), side="right")
    gy = np.searchsorted(np.asarray(ycuts[1:-1]), np.arange(H), side="right")
    return (gy[:, None] * (len(xcuts) - 1) + gx[None, :]).astype(np.int32)


def test_centroids_of_rectangles_are_their_analytic_centres():
    """Pixel centres sit at integer coordinates, u = column, v = row: a cell
    covering columns x0..x1 and rows y0..y1 has centroid ((x0 + x1) / 2,
    (y0 + y1) / 2).  Cells are unequal and the image is not square, so swapping
    u and v or moving the pixel centres by half a pixel changes the result."""
    W, H = 37, 23
    xc, yc = [0, 5, 19, 37], [0, 9, 23]
    lab = _rect_labels(W, H, xc, yc)
    rng = np.random.default_rng(21)
    rgb = rng.integers(0, 256, size=(H, W, 3), dtype=np.uint8)
    orc = Oracle(rig([view(W, H, rgb=rgb, labels=lab, gw=3, gh=2), view(W, H, rgb=rgb, labels=lab, gw=3, gh=2)]),
                 params())
    area, cen, col = orc.sp_stats()
    for gy in range(2):
        for gx in range(3):
            k = gy * 3 + gx
            x0, x1 = xc[gx], xc[gx + 1] - 1
            y0, y1 = yc[gy], yc[gy + 1] - 1
            assert area[k] == (x1 - x0 + 1) * (y1 - y0 + 1)
            assert cen[k, 0] == pytest.approx((x0 + x1) / 2.0, abs=1e-12)
            assert cen[k, 1] == pytest.approx((y0 + y1) / 2.0, abs=1e-12)
            block = rgb[y0:y1 + 1, x0:x1 + 1].reshape(-1, 3).astype(np.float64)
            assert np.allclose(col[k], block.mean(0) / 255.0, atol=1e-12)


def test_centroids_of_irregular_labels_are_pixel_means():
    """Irregular cells (a staircase, a ring, scattered pixels, an empty cell):
    centroid = mean column and mean row of the cell's pixels, area = count,
    colour = mean of rgb / 255."""
    W, H = 29, 17
    u, v = np.meshgrid(np.arange(W), np.arange(H))
    lab = np.zeros((H, W), np.int32)
    lab[(u + 2 * v) % 7 == 0] = 1                  # scattered diagonal stripes
    lab[(u > 3 * v) & (lab == 0)] = 2              # staircase above a slanted line
    ring = (np.abs(u - 20) + np.abs(v - 10) <= 4) & (np.abs(u - 20) + np.abs(v - 10) >= 2)
    lab[ring] = 3                                   # a diamond ring
    # cell 4 stays empty; cell 5 is a single pixel
    lab[16, 0] = 5
    rng = np.random.default_rng(22)
    rgb = rng.integers(0, 256, size=(H, W, 3), dtype=np.uint8)
    vw = view(W, H, rgb=rgb, labels=lab, gw=3, gh=2)
    orc = Oracle(rig([vw, view(W, H, rgb=rgb, labels=lab, gw=3, gh=2)]), params())
    area, cen, col = orc.sp_stats()
    for k in range(6):
        ys, xs = np.nonzero(lab == k)
        assert area[k] == len(xs)
        if len(xs) == 0:
            continue
        assert cen[k, 0] == pytest.approx(xs.mean(), abs=1e-12)
        assert cen[k, 1] == pytest.approx(ys.mean(), abs=1e-12)
        assert np.allclose(col[k], rgb[ys, xs].astype(np.float64).mean(0) / 255.0, atol=1e-12)
    assert area[4] == 0 and area[5] == 1 and tuple(cen[5]) == (0.0, 16.0)


def test_centroids_of_slic_labels_are_pixel_means():
    """The same definition on every superpixel of the SLIC segmentation of the
    tiny 160 x 120 workload (all three views)."""
    w = config1()
    orc = Oracle(w.rig, w.params)
    area, cen, _ = orc.sp_stats()
    for vi, vw in enumerate(w.rig.views):
        sl = orc.view_slice(vi)
        a, c = area[sl], cen[sl]
        for k in range(vw.gw * vw.gh):
            ys, xs = np.nonzero(vw.labels == k)
            assert a[k] == len(xs)
            if len(xs):
                assert c[k, 0] == pytest.approx(xs.mean(), abs=1e-9)
                assert c[k, 1] == pytest.approx(ys.mean(), abs=1e-9)


def test_smoothness_extrapolates_at_analytic_centroids():
    """Eqs. (5)-(6) on a slanted plane: each neighbour's depth is set to the
    plane's depth along the ray of the analytic centre of its rectangle, so
    extrapolating the candidate plane to those centroids gives the same depths
    and E_s = 1 exactly.  A small sigma makes a centroid error of a fraction of
    a pixel visible: the same state built at centres moved by half a pixel, or
    with u and v exchanged, lowers E_s well below 1."""
    W, H, f = 41, 27, 90.0
    xc, yc = [0, 8, 21, 41], [0, 6, 17, 27]
    lab = _rect_labels(W, H, xc, yc)
    rgb = np.full((H, W, 3), 120, np.uint8)
    vs = [view(W, H, f=f, labels=lab, rgb=rgb, gw=3, gh=3) for _ in range(2)]
    sigma = 0.002
    orc = Oracle(rig(vs), params(term_mask=1, sigma=sigma))
    Kinv = np.linalg.inv(vs[0].K)
    n = np.array([0.45, -0.35, 1.0])
    n /= np.linalg.norm(n)
    delta = 3.0

    def state(shift=(0.0, 0.0), swap=False):
        A = np.zeros((orc.S, 4))
        for vi in range(2):
            for gy in range(3):
                for gx in range(3):
                    cu = (xc[gx] + xc[gx + 1] - 1) / 2.0 + shift[0]
                    cv = (yc[gy] + yc[gy + 1] - 1) / 2.0 + shift[1]
                    if swap:
                        cu, cv = cv, cu
                    ray = Kinv @ np.array([cu, cv, 1.0])
                    A[vi * 9 + gy * 3 + gx] = [delta / (n @ ray), *n]
        return A

    A = state()
    assert orc.energy(A, 0, 4, A[4]) == pytest.approx(1.0, abs=1e-12)
    for bad in (state(shift=(0.5, 0.5)), state(swap=True)):
        assert orc.energy(bad, 0, 4, bad[4]) < 1.0 - 1e-3


def _ramp_images(W, H):
    u = np.arange(W)[None, :]
    v = np.arange(H)[:, None]
    img = np.stack(np.broadcast_arrays(2 * u + v, u + 3 * v, 100 + u - v), axis=-1)
    return img.astype(np.uint8), np.array([[2, 1], [1, 3], [1, -1]], float)


def test_normalised_cost_of_a_three_view_rig_divides_by_both_neighbours():
    """Eq. (2) sums the truncated SSD over the N = |N(r)| neighbour views and
    the superpixel's pixels; normalised by |Omega| N T it is the mean per-sample
    cost over T.  A rectified 3-view rig on an affine image: neighbour 1 is
    shifted by s1 along x, neighbour 2 by s2 along y, so each sample's SSD is a
    closed form (bilinear interpolation reproduces an affine image), and the
    normalised cost is the mean of the two views' per-view means."""
    W, H, f, d = 40, 30, 100.0, 2.5
    img, slope = _ramp_images(W, H)
    s1, s2 = 1.25, 0.6
    vs = [view(W, H, f=f, rgb=img, gw=2, gh=2),
          view(W, H, f=f, centre=(-s1 * d / f, 0, 0), rgb=img, gw=2, gh=2),
          view(W, H, f=f, centre=(0, -s2 * d / f, 0), rgb=img, gw=2, gh=2)]
    T = 0.002
    orc = Oracle(rig(vs, neighbors=[[1, 2], [0, 2], [0, 1]]), params(tssd_T=T))
    ssd1 = min(T, float(np.sum((s1 * slope[:, 0] / 255.0) ** 2)))
    ssd2 = min(T, float(np.sum((s2 * slope[:, 1] / 255.0) ** 2)))
    assert ssd1 < T and ssd2 < T
    lab = vs[0].labels
    for s in range(4):
        ys, xs = np.nonzero(lab == s)
        in1 = xs + s1 <= W - 1
        in2 = ys + s2 <= H - 1
        total = in1.sum() * ssd1 + (~in1).sum() * T + in2.sum() * ssd2 + (~in2).sum() * T
        exp = total / (len(xs) * 2 * T)
        assert orc.sweep_cost(0, s, [d, 0, 0, 1.0]) == pytest.approx(exp, rel=1e-9, abs=1e-12)


@pytest.mark.parametrize("n_views", [2, 3, 4])
def test_normalised_cost_of_saturated_samples_is_one_for_any_neighbour_count(n_views):
    """Every sample costs T when it leaves the image (behind-camera and
    out-of-view samples cost T), so C = |Omega| N T and the normalised cost is
    exactly 1 whatever the number of neighbour views.  A plane at depth 1e-3
    shifts every sample by thousands of pixels in every neighbour."""
    W, H, f = 24, 18, 60.0
    rng = np.random.default_rng(5)
    vs = [view(W, H, f=f, centre=(0.4 * j, 0.0, 0.0), rgb=rng.integers(0, 256, (H, W, 3), dtype=np.uint8),
               gw=2, gh=2) for j in range(n_views)]
    orc = Oracle(rig(vs), params(tssd_T=0.04))
    for vi in range(n_views):
        for s in range(4):
            assert orc.sweep_cost(vi, s, [1e-3, 0, 0, 1.0]) == pytest.approx(1.0, rel=1e-12)
