"""FP64 oracle of the annealed particle filter's particle weights (Eq. 10,
14-16): how well each particle's body model matches the silhouette and edge
maps of every view.

TEST INFRASTRUCTURE ONLY: used by ``tests/`` and the benchmark's CPU baseline;
the product library never imports this package.

Eq. 14 and 15 average 1 - p over the N sample points of the model in one
camera, p being the edge-map value (Eq. 14) or the silhouette-map value
(Eq. 15) at the point's image; Eq. 16 takes w = exp(-(sum over cameras of the
two averages)) and Eq. 10 normalises the weights over the particles. The paper
computes the model's ten cylinders from 31 pose parameters (a step outside
this pass) and does not say which points are sampled. The reading taken here,
per particle, camera (centre C) and cylinder (end points A, B, radii rA, rB):

* M = 8 cross-sections at t = (m + 1/2) / M: centre X = A + t (B - A), radius
  r = rA + t (rB - rA), unit axis a = (B - A) / |B - A|;
* w = (X - C) minus its component along a, rho = |w|, u = w / rho, e = a x u:
  u points away from the camera across the axis, e across the cylinder's image;
* edge points (Eq. 14): the two points of the cross-section circle where the
  viewing ray touches the circle, X - (r^2 / rho) u +- r sqrt(1 - r^2 / rho^2) e
  (the cylinder's two outlines);
* silhouette points (Eq. 15): X and X +- (r / 2) e, inside the cylinder's image;
* a point is projected with the nearest-pixel rule of the occupancy pass
  (Eq. 3-9): pixel (floor(x / z + 1/2), floor(y / z + 1/2)) of (x, y, z) = P [X; 1];
  p is the map value there, and p = 0 when z <= 0, when the pixel lies outside
  the image, and for all five points of a cross-section whose circle contains
  the camera centre (rho <= r), where no outline exists, or whose geometry is
  not finite (A = B, or a non-finite coordinate or radius);
* per camera: Sigma_e = mean over the 10 * 8 * 2 edge points of 1 - p,
  Sigma_r = mean over the 10 * 8 * 3 silhouette points of 1 - p;
  log w = -sum over cameras of (Sigma_e + Sigma_r);
* the annealing layer's weighting function is w^beta (beta = 1 by default):
  normalised weights pi = exp(beta log w) / sum over particles of the same.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

NCYL = 10
M = 8
N_EDGE = NCYL * M * 2
N_REGION = NCYL * M * 3


def camera_centre(P) -> np.ndarray:
    """C with P [C; 1] = 0, by an FP64 linear solve."""
    P = np.asarray(P, np.float64).reshape(3, 4)
    return -np.linalg.solve(P[:, :3], P[:, 3])


# Geometry that is not finite (A = B, NaN or infinite inputs) propagates NaN,
# which the rho > r test and the image-bounds tests turn into p = 0; numpy's
# warnings about it are silenced where it is computed.
_quiet = np.errstate(invalid="ignore", divide="ignore", over="ignore")


@_quiet
def cross_sections(cyl: np.ndarray):
    """Centres X [..., 10, M, 3], radii r [..., 10, M] and unit axes a [..., 10, 1, 3]
    of the M cross-sections of each cylinder (A, B, rA, rB) in cyl [..., 10, 8]."""
    cyl = np.asarray(cyl, np.float64)
    A, B = cyl[..., 0:3], cyl[..., 3:6]
    rA, rB = cyl[..., 6], cyl[..., 7]
    t = (np.arange(M) + 0.5) / M
    d = B - A
    X = A[..., None, :] + t[:, None] * d[..., None, :]
    r = rA[..., None] + t * (rB - rA)[..., None]
    a = d / np.linalg.norm(d, axis=-1, keepdims=True)
    return X, r, a[..., None, :]


@_quiet
def sample_points(cyl: np.ndarray, C: np.ndarray):
    """Edge points [..., 10, M, 2, 3], silhouette points [..., 10, M, 3, 3] and the
    mask [..., 10, M] of cross-sections that have outlines (rho > r), seen from C."""
    X, r, a = cross_sections(cyl)
    w = X - np.asarray(C, np.float64)
    w = w - np.sum(w * a, axis=-1, keepdims=True) * a
    rho = np.linalg.norm(w, axis=-1)
    valid = rho > r                                         # False for NaN geometry
    safe = np.where(valid, rho, 1.0)
    u = w / safe[..., None]
    e = np.cross(np.broadcast_to(a, u.shape), u)
    q = np.where(valid, r / safe, 0.0)
    back = (r * q)[..., None] * u                                   # (r^2 / rho) u
    side = (r * np.sqrt(1.0 - q * q))[..., None] * e                # r sqrt(1 - r^2/rho^2) e
    edge = np.stack([X - back - side, X - back + side], axis=-2)
    half = (0.5 * r)[..., None] * e
    region = np.stack([X - half, X, X + half], axis=-2)
    return edge, region, valid


@_quiet
def image_coords(cam, pts: np.ndarray):
    """(x / z + 1/2, y / z + 1/2, z > 0) of (x, y, z) = P [pts; 1]: the nearest
    pixel is the floor of the first two."""
    P = np.asarray(cam.P, np.float64).reshape(3, 4)
    h = pts @ P[:, :3].T + P[:, 3]
    z = h[..., 2]
    front = z > 0
    zs = np.where(front, z, 1.0)
    return h[..., 0] / zs + 0.5, h[..., 1] / zs + 0.5, front


@_quiet
def sample_map(cam, image_map: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """Map value at the nearest pixel of each point [..., 3] (0 behind or outside)."""
    xs, ys, front = image_coords(cam, pts)
    x, y = np.floor(xs), np.floor(ys)
    ok = front & (x >= 0) & (x < cam.width) & (y >= 0) & (y < cam.height)
    xi = np.where(ok, x, 0).astype(np.int64)
    yi = np.where(ok, y, 0).astype(np.int64)
    return np.where(ok, np.asarray(image_map, np.float64)[yi, xi], 0.0)


def camera_terms(cam, cylinders: np.ndarray, silhouette: np.ndarray, edge_map: np.ndarray):
    """(Sigma_e, Sigma_r) of Eq. 14 and 15 for every particle in one camera, [np] each."""
    cyl = np.asarray(cylinders, np.float64)
    edge, region, valid = sample_points(cyl, camera_centre(cam.P))
    pe = np.where(valid[..., None], sample_map(cam, edge_map, edge), 0.0)
    pr = np.where(valid[..., None], sample_map(cam, silhouette, region), 0.0)
    n = cyl.shape[0]
    return (1.0 - pe).reshape(n, -1).mean(axis=1), (1.0 - pr).reshape(n, -1).mean(axis=1)


def log_weights(cams: Sequence, cylinders: np.ndarray, silhouettes: Sequence[np.ndarray],
                edges: Sequence[np.ndarray]) -> np.ndarray:
    """log w of Eq. 16 for every particle (cylinders [np, 10, 8])."""
    cyl = np.asarray(cylinders, np.float64)
    total = np.zeros(cyl.shape[0])
    for cam, S, E in zip(cams, silhouettes, edges):
        se, sr = camera_terms(cam, cyl, S, E)
        total += se + sr
    return -total


def normalised(logw: np.ndarray, beta: float = 1.0) -> np.ndarray:
    """Eq. 10: weights w^beta scaled to sum to 1."""
    z = beta * np.asarray(logw, np.float64)
    e = np.exp(z - z.max())
    return e / e.sum()
