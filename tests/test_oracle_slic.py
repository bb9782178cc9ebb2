"""Pins of the oracle's grid-seeded SLIC segmentation (Sec. III-A: SLIC
superpixels read as a regular grid of cells).  Expected values come from the
geometry of the grid (uniform images), numpy means, label maps built by hand
for the connectivity rule, and properties that hold on any image (every label
one 4-connected region, boundary adherence at low compactness)."""
from __future__ import annotations

from collections import deque

import numpy as np
import pytest

from lfsynth import config1
from lfsynth.scene import grid_labels
from oracle import oracle


def _components(mask):
    """4-connected components of a boolean mask (list of pixel-index arrays)."""
    H, W = mask.shape
    seen = np.zeros_like(mask, bool)
    out = []
    for s in zip(*np.nonzero(mask)):
        if seen[s]:
            continue
        q = deque([s])
        seen[s] = True
        comp = []
        while q:
            y, x = q.popleft()
            comp.append((y, x))
            for dy, dx in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                ny, nx = y + dy, x + dx
                if 0 <= ny < H and 0 <= nx < W and mask[ny, nx] and not seen[ny, nx]:
                    seen[ny, nx] = True
                    q.append((ny, nx))
        out.append(comp)
    return out


@pytest.mark.parametrize("gw, gh, cell_w, cell_h", [(4, 3, 8, 8), (5, 2, 6, 10), (3, 4, 7, 5)])
def test_uniform_image_keeps_the_seed_grid(gw, gh, cell_w, cell_h):
    """With one colour everywhere only the spatial term counts; cells of
    cell_w x cell_h pixels have their centres in the middle of each cell, so
    every pixel is closest to its own cell's centre (midpoints between centres
    fall between pixels), the centres do not move, and the labels are the
    seed grid.  A non-square grid and cells fails an exchange of u and v."""
    W, H = gw * cell_w, gh * cell_h
    rgb = np.full((H, W, 3), 90, np.uint8)
    cen = oracle.slic_centres_init(rgb, gw, gh)
    k = np.arange(gw * gh)
    assert np.allclose(cen[:, 0], (k % gw + 0.5) * cell_w - 0.5)
    assert np.allclose(cen[:, 1], (k // gw + 0.5) * cell_h - 0.5)
    assert np.all(cen[:, 2:] == 90)
    lab = oracle.slic(rgb, gw, gh, iterations=5, compactness=10.0)
    assert np.array_equal(lab, grid_labels(W, H, gw, gh))


def test_seed_colour_is_the_nearest_pixel_of_the_cell_centre():
    """Cells of 5 x 3 pixels: centre (2, 1) + cell offset, an exact pixel."""
    gw, gh = 4, 3
    W, H = 20, 9
    rng = np.random.default_rng(3)
    rgb = rng.integers(0, 256, size=(H, W, 3), dtype=np.uint8)
    cen = oracle.slic_centres_init(rgb, gw, gh)
    for k in range(gw * gh):
        u, v = (k % gw) * 5 + 2, (k // gw) * 3 + 1
        assert tuple(cen[k, :2]) == (u, v)
        assert np.array_equal(cen[k, 2:], rgb[v, u].astype(np.float32))


def test_update_is_the_mean_of_each_label():
    """Centres after an update: mean column, row and colour of each label's
    pixels (numpy, rounded to FP32); a label without pixels keeps its centre."""
    gw, gh = 3, 2
    W, H = 17, 11
    rng = np.random.default_rng(4)
    rgb = rng.integers(0, 256, size=(H, W, 3), dtype=np.uint8)
    lab = rng.integers(0, gw * gh - 1, size=(H, W)).astype(np.int32)   # the last label stays empty
    cen0 = oracle.slic_centres_init(rgb, gw, gh)
    cen = oracle.slic_update(rgb, gw, gh, lab, cen0)
    v, u = np.mgrid[0:H, 0:W]
    for k in range(gw * gh - 1):
        m = lab == k
        exp = [u[m].mean(), v[m].mean(), rgb[..., 0][m].mean(), rgb[..., 1][m].mean(), rgb[..., 2][m].mean()]
        assert np.allclose(cen[k], np.float32(exp), rtol=0, atol=1e-5)
    assert np.array_equal(cen[-1], cen0[-1])


def test_connectivity_rule_on_hand_made_labels():
    """Label 1 has components of 4 (kept) and 2 pixels: the 2-pixel fragment
    takes the label left of its first pixel (0).  Label 2 has two components of
    3 pixels: the one whose first pixel comes first in raster order keeps the
    label, the other takes the label above its first pixel (first column: no
    left pixel)."""
    lab = np.array([[1, 1, 0, 0, 2],
                    [1, 1, 0, 1, 2],
                    [0, 0, 0, 1, 2],
                    [2, 0, 0, 0, 0],
                    [2, 2, 0, 0, 0]], np.int32)
    out = oracle.slic_connectivity(lab, 3, 1)
    exp = lab.copy()
    exp[1:3, 3] = 0          # fragment of label 1 -> left of (1, 3) is label 0
    exp[3:5, 0] = 0          # second component of label 2 (first pixel (3, 0)) -> above is label 0
    exp[4, 1] = 0
    assert np.array_equal(out, exp)


def test_connectivity_chains_and_the_first_pixel():
    """A fragment whose left neighbour is itself a fragment follows it to its
    final label; a fragment holding the image's first pixel keeps its label."""
    lab = np.array([[0, 1, 1, 1, 1],
                    [1, 1, 2, 0, 1],
                    [1, 1, 1, 1, 1],
                    [0, 0, 0, 0, 0]], np.int32)
    out = oracle.slic_connectivity(lab, 3, 1)
    exp = lab.copy()
    # label 0: components {(0,0)} size 1, {(1,3)} size 1, row 3 size 5 (kept); (0,0) is the first pixel: kept
    # (1,3) -> left is (1,2) of label 2 (its only component, kept) -> 2
    exp[1, 3] = 2
    assert np.array_equal(out, exp)
    lab2 = np.array([[3, 3, 0, 1, 1, 1],
                     [0, 0, 0, 1, 2, 1],
                     [0, 1, 1, 1, 1, 1]], np.int32)
    # label 0 (5 px) kept; 3 at (0,0) single component kept; 2 single kept; 1: components
    # {(0,3),(0,4),(0,5),(1,3),(1,5),(2,1..5)} connected? (0,3)-(1,3)-(2,3) yes: one component
    out2 = oracle.slic_connectivity(lab2, 4, 1)
    assert np.array_equal(out2, lab2)


def test_full_segmentation_gives_connected_labels_and_adheres_to_edges():
    """On the tiny workload's first view every label is a single 4-connected
    region (or empty); on a two-colour image with a vertical edge off the cell
    boundaries, low compactness puts no superpixel across the edge."""
    v = config1().rig.views[0]
    lab = oracle.slic(v.rgb, 20, 15, iterations=10, compactness=20.0)
    assert lab.min() >= 0 and lab.max() < 300
    for k in np.unique(lab):
        if k == lab[0, 0]:
            continue      # the first pixel's fragment may keep its label
        assert len(_components(lab == k)) == 1, k
    W, H = 64, 40
    rgb = np.zeros((H, W, 3), np.uint8)
    rgb[:, :37] = [200, 40, 40]
    rgb[:, 37:] = [30, 160, 220]
    lab = oracle.slic(rgb, 8, 5, iterations=10, compactness=1.0)
    left, right = set(np.unique(lab[:, :37])), set(np.unique(lab[:, 37:]))
    assert not (left & right)


def test_ties_go_to_the_first_centre_in_scan_order():
    """Colour only (compactness 0), two cells on one row: centre 0 holds grey
    100, centre 1 grey 120, every other pixel grey 110, equally far from both.
    The scan visits the left cell first (dx = -1 before dx = 0 in cell 1, dx = 0
    before dx = +1 in cell 0), so every tie goes to label 0."""
    rgb = np.full((1, 10, 3), 110, np.uint8)
    rgb[0, 2] = 100
    rgb[0, 7] = 120
    lab = oracle.slic(rgb, 2, 1, iterations=1, compactness=0.0, connectivity=False)
    assert lab[0].tolist() == [0, 0, 0, 0, 0, 0, 0, 1, 0, 0]
    # with connectivity the fragment {8, 9} of label 0 joins label 1 (left of pixel 8)
    lab = oracle.slic(rgb, 2, 1, iterations=1, compactness=0.0, connectivity=True)
    assert lab[0].tolist() == [0, 0, 0, 0, 0, 0, 0, 1, 1, 1]


def test_pixel_cells_and_seed_pixels_on_a_ragged_grid():
    """W = 10, gw = 4: cell widths 2.5 px.  Pixel u lies in cell floor((u + 0.5)
    0.4) = 0,0,1,1,1,2,2,3,3,3; centre k starts at (k + 0.5) 2.5 - 0.5 = 0.75,
    3.25, 5.75, 8.25 with the colour of pixels 1, 3, 6, 8 (nearest, round half
    up).  With colour-only distance, pixel 2 (in cell 1) sees centres 0..2 and
    takes centre 2 whose colour it shares; from cell 0 it could not."""
    rgb = np.zeros((1, 10, 3), np.uint8)
    cols = {1: 10, 3: 60, 6: 200, 8: 250}
    for u, c in cols.items():
        rgb[0, u] = c
    rgb[0, 2] = 200
    cen = oracle.slic_centres_init(rgb, 4, 1)
    assert np.allclose(cen[:, 0], [0.75, 3.25, 5.75, 8.25])
    assert cen[:, 2].tolist() == [10, 60, 200, 250]
    lab = oracle.slic(rgb, 4, 1, iterations=1, compactness=0.0, connectivity=False)
    assert lab[0, 2] == 2
    # half-pixel centres round up: W = 6, gw = 3 -> centres 0.5, 2.5, 4.5 -> pixels 1, 3, 5
    rgb6 = np.arange(18, dtype=np.uint8).reshape(1, 6, 3) * 10
    cen6 = oracle.slic_centres_init(rgb6, 3, 1)
    assert np.array_equal(cen6[:, 2:], rgb6[0, [1, 3, 5]].astype(np.float32))
