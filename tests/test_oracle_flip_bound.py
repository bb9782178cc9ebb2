"""Pins of the oracle's parity instrument Oracle.energy_flip_bound: an upper
bound of how much the energy (eq. 3) can change when the per-sample discrete
decisions of the consistency term (the nearest pixel of eq. 9, the visible /
occluded split of eqs. 10-11) that sit within a small distance of their
thresholds flip.  Each pin puts every sample exactly on a threshold, moves the
plane by 1e-9 to either side (which decides every flip one way or the other
while the continuous terms barely move) and checks that the bound covers the
energy change and is not zero; away from the thresholds the bound is 0."""
from __future__ import annotations

import numpy as np

from oracle.oracle import Oracle
from tests.microrig import block_rgb, fronto_state, params, rig, view


def _half_pixel_pair(shift):
    """A rectified pair whose disparity at depth 4 is `shift` px onto a view with
    labels alternating by column (two colours)."""
    W, H, f, d = 8, 2, 128.0, 4.0
    c0, c1 = np.array([100, 100, 100]), np.array([100, 160, 100])
    rgb_r = np.tile(c0.astype(np.uint8), (H, W, 1))
    lab_i = np.tile((np.arange(W) % 2).astype(np.int32), (H, 1))
    rgb_i = np.where(lab_i[..., None] == 0, c0, c1).astype(np.uint8)
    v0 = view(W, H, f=f, rgb=rgb_r, gw=1, gh=1)
    v1 = view(W, H, f=f, centre=(-shift * d / f, 0, 0), rgb=rgb_i, labels=lab_i, gw=2, gh=1)
    orc = Oracle(rig([v0, v1], neighbors=[[1], [0]]), params(term_mask=2 | 4, alpha=0.3))
    A = np.zeros((orc.S, 4))
    A[:, 0] = d
    A[:, 3] = 1.0
    return orc, A, d


def test_bound_covers_nearest_pixel_flips_at_half_pixel_disparity():
    orc, A, d = _half_pixel_pair(0.5)
    near = orc.energy_flip_bound(A, 0, 0, [d, 0, 0, 1])
    e_lo = orc.energy(A, 0, 0, [d * (1 + 1e-9), 0, 0, 1])   # disparity just below 0.5: rounds to column u
    e_hi = orc.energy(A, 0, 0, [d * (1 - 1e-9), 0, 0, 1])   # just above: rounds to column u + 1
    assert abs(e_hi - e_lo) > 1e-3                           # the labels alternate: the colour term changes
    assert near >= abs(e_hi - e_lo)
    assert orc.energy_flip_bound(A, 0, 0, [d * (1 + 1e-9), 0, 0, 1]) >= abs(e_hi - e_lo)
    # at 0.7 px no decision is near a threshold
    orc7, A7, _ = _half_pixel_pair(0.7)
    assert orc7.energy_flip_bound(A7, 0, 0, [d, 0, 0, 1]) == 0.0


def test_bound_covers_visibility_split_flips():
    """Identical cameras: z = d for the superpixel's plane.  The neighbour
    superpixel of view 1 under two of its pixels holds depth d / (1 + tau), so
    z sits exactly on the split z <= D (1 + tau); moving that depth by 1e-9
    moves both samples between X and Y (and toggles the occlusion term)."""
    sigma, alpha, eta, tau = 0.1, 0.15, 0.5, 1e-3
    cols0 = [[100, 100, 100], [150, 90, 100], [100, 100, 60], [90, 90, 90]]
    rgb0 = block_rgb(4, 4, 2, 2, cols0)
    lab1 = np.array([[0, 0, 1, 1], [2, 2, 3, 3], [2, 2, 3, 3], [2, 2, 3, 3]], np.int32)
    rgb1 = np.zeros((4, 4, 3), np.uint8)
    rgb1[lab1 == 0] = [110, 100, 100]
    rgb1[lab1 == 2] = [100, 130, 100]
    v0 = view(4, 4, f=128.0, rgb=rgb0, gw=2, gh=2)
    v1 = view(4, 4, f=128.0, rgb=rgb1, labels=lab1, gw=2, gh=2)
    orc = Oracle(rig([v0, v1]), params(term_mask=2 | 4, sigma=sigma, alpha=alpha, eta=eta, occ_tol=tau))
    d = 3.0
    A = fronto_state(orc.S, d)
    A[4 + 2, 0] = d / (1 + tau)
    b = orc.energy_flip_bound(A, 0, 0, [d, 0, 0, 1])
    Ap, Am = A.copy(), A.copy()
    Ap[4 + 2, 0] *= 1 + 1e-9    # visible
    Am[4 + 2, 0] *= 1 - 1e-9    # occluded
    e_vis = orc.energy(Ap, 0, 0, [d, 0, 0, 1])
    e_occ = orc.energy(Am, 0, 0, [d, 0, 0, 1])
    assert abs(e_vis - e_occ) > 1e-2
    assert b >= abs(e_vis - e_occ)
    # a clearly nearer neighbour: no sample near the split, no flip possible
    A[4 + 2, 0] = 2.5
    assert orc.energy_flip_bound(A, 0, 0, [d, 0, 0, 1]) == 0.0


def test_bound_is_zero_without_the_consistency_term():
    orc, A, d = _half_pixel_pair(0.5)
    orc.set_params(params(term_mask=1, alpha=0.3))
    assert orc.energy_flip_bound(A, 0, 0, [d, 0, 0, 1]) == 0.0
