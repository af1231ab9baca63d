"""Literal, brute-force evaluation of Eq. 3-9 (Sec. 2.2.2) for tiny scenes.

TEST INFRASTRUCTURE ONLY. Pure Python on Python floats (IEEE FP64):

* the pixel a voxel projects to is found by scanning every pixel for the unit
  square ``[x-1/2, x+1/2) x [y-1/2, y+1/2)`` that contains the projected
  centre (no rounding formula);
* ``P(S_k | V)`` is the sum over the occluder variable O of the sensor-model
  table of Eq. 6-9 times ``P(O) = 1/2`` (Eq. 5);
* the views are multiplied (Eq. 4) and Bayes' rule over ``V in {0, 1}`` gives
  the posterior (Eq. 3).

It exists to pin the C oracle on tiny inputs; it shares no code with it.
"""
from __future__ import annotations

from typing import Sequence

# Eq. 6-9: P(S | O, V) as a function of the SLM value s, keyed by (O, V).
SENSOR_MODEL = {
    (0, 0): lambda s: 1.0 - s,      # Eq. 6: no voxel, no occluder
    (1, 0): lambda s: s,            # Eq. 7
    (0, 1): lambda s: s,            # Eq. 8
    (1, 1): lambda s: s,            # Eq. 9
}
P_OCCLUDER = {0: 0.5, 1: 0.5}       # P(O), no preference


def pixel_by_containment(u: float, v: float, W: int, H: int):
    for y in range(H):
        if not (y - 0.5 <= v < y + 0.5):
            continue
        for x in range(W):
            if x - 0.5 <= u < x + 0.5:
                return x, y
    return None


def view_term(s: float, V: int) -> float:
    return sum(SENSOR_MODEL[(O, V)](s) * P_OCCLUDER[O] for O in (0, 1))


def posterior_from_slm_values(values: Sequence[float], prior: float) -> float:
    like = {}
    for V in (0, 1):
        prod = 1.0
        for s in values:
            prod *= view_term(s, V)
        like[V] = prod
    joint = {1: like[1] * prior, 0: like[0] * (1.0 - prior)}
    return joint[1] / (joint[0] + joint[1])


def posterior_grid(cams, grid, slm_maps, prior: float = 0.5):
    """Nested-list posterior [nz][ny][nx] of a tiny scene."""
    o = [float(x) for x in grid.origin]
    h = float(grid.voxel)
    out = []
    for k in range(grid.nz):
        plane = []
        for j in range(grid.ny):
            row = []
            for i in range(grid.nx):
                X = (o[0] + h * (i + 0.5), o[1] + h * (j + 0.5), o[2] + h * (k + 0.5), 1.0)
                values = []
                for cam, smap in zip(cams, slm_maps):
                    P = [[float(cam.P[r][c]) for c in range(4)] for r in range(3)]
                    a, b, c = (sum(P[r][q] * X[q] for q in range(4)) for r in range(3))
                    if not c > 0.0:
                        continue
                    pix = pixel_by_containment(a / c, b / c, cam.width, cam.height)
                    if pix is None:
                        continue
                    values.append(float(smap[pix[1]][pix[0]]))
                row.append(posterior_from_slm_values(values, prior))
            plane.append(row)
        out.append(plane)
    return out
