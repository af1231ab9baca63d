"""FP64 oracle of voxel colouring: the colour of each reconstructed (surface)
voxel from the views that see it.

TEST INFRASTRUCTURE ONLY: used by ``tests/`` and the benchmark's CPU baseline;
the product library never imports this package.

The paper colours the reconstructed voxels from the camera images (Sec. 3.1.1)
and splits the work into a step over voxel x camera pairs and two steps over
image pixels (Sec. 3.3.1, Sec. 3.3.3 "Voxel Projection and Color
Computation"); the colour rule and the visibility test are not given. The
readings taken here:

* a listed voxel's centre is projected into every view exactly as in the
  fusion (nearest pixel x = floor(u + 1/2), y = floor(v + 1/2); a view is
  skipped when the depth c <= 0 or the pixel is outside the image);
* visibility is a depth buffer over the listed voxels: at each pixel of each
  view the voxel with the smallest depth c wins (equal depths: the smaller
  position in the list);
* colour = the mean over the views in which the voxel wins its pixel of that
  pixel's RGB values; a voxel that wins in no view gets colour 0 and count 0.

For comparisons with FP32 arithmetic, ``ambiguous`` marks voxels whose result
could change under rounding: a projection within ``eps_px`` of a pixel
boundary (its own, or another listed voxel's that may land on its pixel), or
a depth within a relative ``eps_depth`` of another candidate at its pixel.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

EPS_PX = 1e-3
EPS_DEPTH = 1e-5


def voxel_centres(grid, indices: np.ndarray) -> np.ndarray:
    """FP64 centres of the voxels with linear indices (k*ny + j)*nx + i."""
    idx = np.asarray(indices, dtype=np.int64)
    nx, ny = int(grid.nx), int(grid.ny)
    i = idx % nx
    j = (idx // nx) % ny
    k = idx // (nx * ny)
    o = np.asarray(grid.origin, dtype=np.float64)
    h = float(grid.voxel)
    return np.stack([o[0] + h * (i + 0.5), o[1] + h * (j + 0.5), o[2] + h * (k + 0.5)], axis=1)


def project(cam, X: np.ndarray):
    """(pixel x, pixel y, depth c, in_view, ambiguous, u + 1/2, v + 1/2) of FP64 points X [n,3]."""
    P = np.asarray(cam.P, dtype=np.float64).reshape(3, 4)
    Xh = np.concatenate([X, np.ones((len(X), 1))], axis=1)
    a, b, c = (Xh @ P.T).T
    with np.errstate(divide="ignore", invalid="ignore"):
        u = a / c + 0.5
        v = b / c + 0.5
    fx, fy = np.floor(u), np.floor(v)
    ok = (c > 0) & (fx >= 0) & (fx < cam.width) & (fy >= 0) & (fy < cam.height)
    amb = ((u - fx) < EPS_PX) | ((fx + 1 - u) < EPS_PX) | ((v - fy) < EPS_PX) | ((fy + 1 - v) < EPS_PX)
    return fx.astype(np.int64), fy.astype(np.int64), c, ok, amb & (c > 0), u, v


def colour(cams: Sequence, grid, images: Sequence[np.ndarray], indices: np.ndarray):
    """(colour [n,3] FP64, views [n] int, ambiguous [n] bool) of the listed voxels."""
    idx = np.asarray(indices, dtype=np.int64)
    n = len(idx)
    X = voxel_centres(grid, idx)
    sums = np.zeros((n, 3))
    views = np.zeros(n, dtype=np.int64)
    ambiguous = np.zeros(n, dtype=bool)
    for cam, img in zip(cams, images):
        x, y, c, ok, amb, u, v = project(cam, X)
        W = int(cam.width)
        pix = y * W + x
        # winner per pixel: smallest depth, then smallest list position
        cand = np.flatnonzero(ok)
        order = np.lexsort((cand, c[cand], pix[cand]))
        cand = cand[order]
        first = np.ones(len(cand), dtype=bool)
        first[1:] = pix[cand[1:]] != pix[cand[:-1]]
        winners = cand[first]
        for w in winners:
            sums[w] += img[y[w], x[w]].astype(np.float64)
            views[w] += 1
        # rounding-sensitive voxels: a projection near a pixel boundary, and
        # every candidate at a pixel such a projection may leave or reach
        # (floor(u +- eps) x floor(v +- eps)); a depth near-tie at a pixel
        ambiguous |= amb
        unsafe = set()
        for q in np.flatnonzero(amb):
            for px in {int(np.floor(u[q] - EPS_PX)), int(np.floor(u[q] + EPS_PX))}:
                for py in {int(np.floor(v[q] - EPS_PX)), int(np.floor(v[q] + EPS_PX))}:
                    if 0 <= px < W and 0 <= py < cam.height:
                        unsafe.add(py * W + px)
        for q in cand:
            if int(pix[q]) in unsafe:
                ambiguous[q] = True
        same = pix[cand[1:]] == pix[cand[:-1]]
        close = np.abs(c[cand[1:]] - c[cand[:-1]]) <= EPS_DEPTH * np.abs(c[cand[:-1]])
        for t in np.flatnonzero(same & close):
            ambiguous[cand[t]] = ambiguous[cand[t + 1]] = True
    col = np.where(views[:, None] > 0, sums / np.maximum(views, 1)[:, None], 0.0)
    return col, views, ambiguous
