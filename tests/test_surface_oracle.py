"""Pins of the surface-extraction oracle (smoothing, threshold, inner-voxel
removal; Sec. 2.2.2 last step, Sec. 3.3.3 steps d-e) against things other
than itself: hand-derived values, scipy's convolution, closed-form counts and
brute-force loops. No GPU."""
from fractions import Fraction
import itertools

import numpy as np
import pytest
from scipy import ndimage

from oracle import surface as SO


def test_hand_case_single_hot_voxel():
    # 3x3x3 grid, posterior 1 at the centre, 0 elsewhere. A voxel's in-grid
    # neighbourhood has 27 (centre), 18 (face), 12 (edge) or 8 (corner) cells,
    # and every one of them contains the centre.
    p = np.zeros((3, 3, 3))
    p[1, 1, 1] = 1.0
    sm = SO.smooth(p)
    want = {0: Fraction(1, 8), 1: Fraction(1, 12), 2: Fraction(1, 18), 3: Fraction(1, 27)}
    for k, j, i in itertools.product(range(3), repeat=3):
        centred = (k == 1) + (j == 1) + (i == 1)
        assert sm[k, j, i] == float(want[centred]), (k, j, i)


def test_smoothing_equals_ratio_of_zero_padded_convolutions():
    rng = np.random.default_rng(1)
    p = rng.random((7, 9, 11))
    ones = np.ones((3, 3, 3))
    num = ndimage.convolve(p, ones, mode="constant", cval=0.0)
    den = ndimage.convolve(np.ones_like(p), ones, mode="constant", cval=0.0)
    np.testing.assert_allclose(SO.smooth(p), num / den, rtol=1e-14, atol=1e-15)


def test_constant_field_is_kept():
    p = np.full((5, 4, 6), 0.375)
    assert np.array_equal(SO.smooth(p), p)
    assert SO.threshold(SO.smooth(p), 0.375).sum() == 0          # strict threshold
    assert SO.threshold(SO.smooth(p), 0.37).all()


def test_solid_block_surface_count():
    for m in (1, 2, 3, 5):
        occ = np.zeros((m + 4, m + 4, m + 4), np.uint8)
        occ[2:2 + m, 2:2 + m, 2:2 + m] = 1
        surf = SO.surface_mask(occ)
        assert surf.sum() == m ** 3 - max(m - 2, 0) ** 3
        assert not (surf & (occ == 0)).any()
    full = np.ones((6, 5, 4), np.uint8)                            # the grid border is exposed
    assert SO.surface_mask(full).sum() == 6 * 5 * 4 - 4 * 3 * 2


def test_brute_force_on_tiny_random_grids():
    rng = np.random.default_rng(7)
    for trial in range(6):
        shape = tuple(int(s) for s in rng.integers(1, 6, 3))
        p = rng.random(shape)
        tau = float(rng.uniform(0.3, 0.7))
        sm, occ, idx = SO.extract(p, tau)
        nz, ny, nx = shape
        want_sm = np.zeros(shape)
        for k, j, i in itertools.product(range(nz), range(ny), range(nx)):
            vals = [p[kk, jj, ii] for kk in range(k - 1, k + 2) for jj in range(j - 1, j + 2)
                    for ii in range(i - 1, i + 2) if 0 <= kk < nz and 0 <= jj < ny and 0 <= ii < nx]
            want_sm[k, j, i] = sum(vals) / len(vals)
        np.testing.assert_allclose(sm, want_sm, rtol=1e-14)
        want_idx = []
        for k, j, i in itertools.product(range(nz), range(ny), range(nx)):
            if not want_sm[k, j, i] > tau:
                continue
            exposed = False
            for dk, dj, di in ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)):
                kk, jj, ii = k + dk, j + dj, i + di
                if not (0 <= kk < nz and 0 <= jj < ny and 0 <= ii < nx) or not want_sm[kk, jj, ii] > tau:
                    exposed = True
            if exposed:
                want_idx.append((k * ny + j) * nx + i)
        assert idx.tolist() == want_idx


@pytest.mark.parametrize("tau", [0.25, 0.5])
def test_surface_is_occupied_and_ascending(tau):
    rng = np.random.default_rng(3)
    p = ndimage.gaussian_filter(rng.random((20, 18, 16)), 2.0)
    p = (p - p.min()) / (p.max() - p.min())
    sm, occ, idx = SO.extract(p, tau)
    assert np.all(np.diff(idx) > 0)
    assert occ.reshape(-1)[idx].all()
    # removing the surface leaves exactly the voxels whose 6 neighbours are all occupied
    interior = occ.astype(bool).copy()
    interior.reshape(-1)[idx] = False
    pad = np.pad(occ.astype(bool), 1)
    all6 = np.ones_like(interior)
    for d in ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)):
        all6 &= pad[1 + d[0]:pad.shape[0] - 1 + d[0], 1 + d[1]:pad.shape[1] - 1 + d[1], 1 + d[2]:pad.shape[2] - 1 + d[2]]
    assert np.array_equal(interior, occ.astype(bool) & all6)
