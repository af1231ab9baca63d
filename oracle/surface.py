"""FP64 oracle of the step after the posterior: smoothing, thresholding and
inner-voxel removal (surface extraction).

TEST INFRASTRUCTURE ONLY: used by ``tests/`` and the benchmark's CPU baseline;
the product library never imports this package.

The paper (Sec. 2.2.2, last paragraph) filters the voxel occupancy
probabilities, thresholds them, and removes the voxels inside the body so
that only surface voxels remain; its GPU version merges the smoothing with the
voxel generation in one traversal and keeps the inner-voxel removal on the CPU
(Sec. 3.3.1, Sec. 3.3.3 steps d and e). The filter, its size and the surface
neighbourhood are not stated; the readings taken here:

* smoothing: the mean of the posterior over the 3x3x3 block of voxels centred
  on each voxel, counting only the voxels inside the grid (so a constant field
  stays constant up to the border);
* thresholding: occupied = smoothed > tau (strict, like the unfiltered
  threshold);
* surface voxel: an occupied voxel with at least one of its 6 face neighbours
  unoccupied or outside the grid; the output lists the linear indices
  ``(k*ny + j)*nx + i`` of the surface voxels in increasing order.
"""
from __future__ import annotations

import numpy as np

OFFSETS_27 = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
FACES_6 = [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]


def _shifted(shape, d):
    """Slices (dst, src) such that dst[v] = src[v + d] for every v with v + d in the grid."""
    dst, src = [], []
    for n, o in zip(shape, d):
        if o >= 0:
            dst.append(slice(0, n - o))
            src.append(slice(o, n))
        else:
            dst.append(slice(-o, n))
            src.append(slice(0, n + o))
    return tuple(dst), tuple(src)


def smooth(post: np.ndarray) -> np.ndarray:
    """Mean of the posterior over each voxel's in-grid 3x3x3 neighbourhood (FP64)."""
    p = np.asarray(post, dtype=np.float64)
    total = np.zeros_like(p)
    count = np.zeros_like(p)
    for d in OFFSETS_27:
        dst, src = _shifted(p.shape, d)
        total[dst] += p[src]
        count[dst] += 1.0
    return total / np.where(count > 0, count, 1.0)


def threshold(smoothed: np.ndarray, tau: float = 0.5) -> np.ndarray:
    return (np.asarray(smoothed) > tau).astype(np.uint8)


def surface_mask(occ: np.ndarray) -> np.ndarray:
    """Occupied voxels with an unoccupied or out-of-grid face neighbour."""
    o = np.asarray(occ).astype(bool)
    exposed = np.zeros_like(o)
    for d in FACES_6:
        inside = np.zeros_like(o)           # neighbour v + d inside the grid and occupied
        dst, src = _shifted(o.shape, d)
        inside[dst] = o[src]
        exposed |= ~inside
    return o & exposed


def extract(post: np.ndarray, tau: float = 0.5):
    """(smoothed posterior, occupancy, ascending int64 linear indices of the surface voxels)."""
    sm = smooth(post)
    occ = threshold(sm, tau)
    idx = np.flatnonzero(surface_mask(occ).reshape(-1)).astype(np.int64)
    return sm, occ, idx
