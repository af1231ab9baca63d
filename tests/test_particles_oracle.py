"""Pins of the FP64 particle-weight oracle (Sec. 2.3.2, Eq. 14-16, normalised
as in Eq. 10) against facts that do not come from the oracle itself: a
hand-computed scene, the tangency that defines an outline (found by brute
force), closed forms for constant maps, degenerate cases, and invariances of
the projection (rigid motion and scale of the world, order of cameras and
particles)."""
import json
import os
from dataclasses import dataclass

import numpy as np
import pytest

from oracle import particles as PT
from synth import scene as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "particle_hand_case.json")
# camera at the origin looking along +z, f = 10 px, principal point (32, 24)
HAND_P = np.array([[10.0, 0, 32, 0], [0, 10, 24, 0], [0, 0, 1, 0]])


@dataclass
class Cam:
    width: int
    height: int
    P: np.ndarray


def _hand_case():
    with open(GOLDEN) as fh:
        g = json.load(fh)
    W, H = g["image"]["width"], g["image"]["height"]
    cams = [Cam(W, H, np.asarray(P, np.float64)) for P in g["cameras_P"]]
    vis, hid = np.asarray(g["visible_cylinder"]), np.asarray(g["hidden_cylinder"])
    parts = np.stack([np.stack([vis] + [hid] * 9), np.stack([hid] * 10)])
    maps = {}
    for key, entries in g["maps_nonzero"].items():
        m = np.zeros((H, W))
        for r, c, v in entries:
            m[r, c] = v
        maps[key] = m
    Sm = [maps["silhouette_cam0"], maps["silhouette_cam1"]]
    Em = [maps["edge_cam0"], maps["edge_cam1"]]
    return g, cams, parts, Sm, Em


def test_hand_case():
    g, cams, parts, Sm, Em = _hand_case()
    lw = PT.log_weights(cams, parts, Sm, Em)
    np.testing.assert_allclose(lw, g["log_w"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(PT.normalised(lw), g["weights_beta_1"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(PT.normalised(lw, 0.5), g["weights_beta_0.5"], rtol=0, atol=1e-12)


def _random_cylinders(rng, n):
    A = rng.uniform(-0.5, 0.5, (n, 10, 3))
    d = rng.normal(size=(n, 10, 3))
    d *= rng.uniform(0.1, 0.5, (n, 10, 1)) / np.linalg.norm(d, axis=-1, keepdims=True)
    r = rng.uniform(0.03, 0.15, (n, 10, 2))
    return np.concatenate([A, A + d, r], axis=-1)


def test_outline_points_touch_the_viewing_cone():
    """Brute force: walk each cross-section circle in 20000 steps and find where
    the ray from the camera centre stops crossing into the circle (the sign of
    (P - C) . (P - X) changes); those two angles are the oracle's outline points."""
    rng = np.random.default_rng(11)
    cyl = _random_cylinders(rng, 1)[0]
    C = np.array([3.1, -2.2, 1.4])
    edge, region, valid = PT.sample_points(cyl, C)
    assert valid.all()
    X, r, a = PT.cross_sections(cyl)
    th = np.linspace(0.0, 2.0 * np.pi, 20000, endpoint=False)
    for c in range(10):
        ax = a[c, 0]
        b1 = np.cross(ax, [1.0, 0.0, 0.0] if abs(ax[0]) < 0.9 else [0.0, 1.0, 0.0])
        b1 /= np.linalg.norm(b1)
        b2 = np.cross(ax, b1)
        for m in range(PT.M):
            ring = X[c, m] + r[c, m] * (np.cos(th)[:, None] * b1 + np.sin(th)[:, None] * b2)
            g = np.einsum("ij,ij->i", ring - C, ring - X[c, m])
            flips = np.nonzero(np.sign(g) != np.sign(np.roll(g, -1)))[0]
            assert len(flips) == 2
            found = ring[flips]
            for p in edge[c, m]:
                assert np.min(np.linalg.norm(found - p, axis=1)) < 2 * np.pi * r[c, m] / 20000 * 1.01


def test_sample_point_geometry():
    rng = np.random.default_rng(12)
    cyl = _random_cylinders(rng, 3)
    C = np.array([-2.5, 3.0, 0.7])
    edge, region, valid = PT.sample_points(cyl, C)
    X, r, a = PT.cross_sections(cyl)
    for k in range(2):
        off = edge[..., k, :] - X
        np.testing.assert_allclose(np.linalg.norm(off, axis=-1), r, rtol=1e-12)
        np.testing.assert_allclose(np.sum(off * a, axis=-1), 0.0, atol=1e-12)
    np.testing.assert_array_equal(region[..., 1, :], X)
    for k in (0, 2):
        off = region[..., k, :] - X
        np.testing.assert_allclose(np.linalg.norm(off, axis=-1), 0.5 * r, rtol=1e-12)
        np.testing.assert_allclose(np.sum(off * a, axis=-1), 0.0, atol=1e-12)
        np.testing.assert_allclose(np.sum(off * (X - C), axis=-1), 0.0, atol=1e-12)
    # the cross-sections sit at the centres of M equal slices of the axis
    A, B = cyl[..., 0:3], cyl[..., 3:6]
    np.testing.assert_allclose(X[..., 0, :], A + (B - A) / (2 * PT.M), atol=1e-15)
    np.testing.assert_allclose(X[..., -1, :], B - (B - A) / (2 * PT.M), atol=1e-15)
    np.testing.assert_allclose(r[..., 0], cyl[..., 6] + (cyl[..., 7] - cyl[..., 6]) / (2 * PT.M), atol=1e-15)


def test_camera_centre_of_generated_rig():
    for cam in S.ring_rig(8, 600.0, 640, 480):
        np.testing.assert_allclose(PT.camera_centre(cam.P), cam.C, atol=2e-5)


def _visible_scene():
    fr_cams = S.ring_rig(4, 300.0, 320, 240)
    body = S.make_body(S.rng_for(0, 0, S.STREAM_BODY))
    parts = S.make_particles(np.random.default_rng(5), S.body_cylinders(body), 6)
    return fr_cams, parts


def test_constant_maps_closed_form():
    cams, parts = _visible_scene()
    for cam in cams:          # every sample point is in front and inside the image
        edge, region, valid = PT.sample_points(parts.astype(np.float64), PT.camera_centre(cam.P))
        assert valid.all()
        for pts in (edge, region):
            x, y, front = PT.image_coords(cam, pts)
            assert front.all() and (x >= 0).all() and (x < cam.width).all() and (y >= 0).all() and (y < cam.height).all()
    a, b = 0.3, 0.8
    Sm = [np.full((c.height, c.width), a) for c in cams]
    Em = [np.full((c.height, c.width), b) for c in cams]
    lw = PT.log_weights(cams, parts, Sm, Em)
    np.testing.assert_allclose(lw, -len(cams) * ((1 - a) + (1 - b)), rtol=1e-14)
    for cam, s, e in zip(cams, Sm, Em):
        se, sr = PT.camera_terms(cam, parts, s, e)
        np.testing.assert_allclose(se, 1 - b, rtol=1e-14)
        np.testing.assert_allclose(sr, 1 - a, rtol=1e-14)


def test_hidden_particles_score_two_per_camera():
    cams, parts = _visible_scene()
    behind = parts.astype(np.float64).copy()
    ones = [np.ones((c.height, c.width)) for c in cams]
    # move every cylinder 20 m up: above every camera's field of view
    behind[..., 2] += 20.0
    behind[..., 5] += 20.0
    np.testing.assert_allclose(PT.log_weights(cams, behind, ones, ones), -2.0 * len(cams), rtol=0, atol=0)
    zeros = [np.zeros((c.height, c.width)) for c in cams]
    np.testing.assert_allclose(PT.log_weights(cams, parts, zeros, zeros), -2.0 * len(cams), rtol=0, atol=0)


def test_camera_inside_a_cylinder():
    """Cross-sections whose circle holds the camera centre have no outline: all
    five of their points count p = 0 (here 16 outline and 24 silhouette points)."""
    cam = Cam(64, 48, HAND_P)
    small = [-0.2, 0.0, 10.0, 0.2, 0.0, 10.0, 0.01, 0.01]
    # a tube of radius 1 along the optical axis, 5 cm off it: the camera sits
    # inside every cross-section, whose middle silhouette points would be seen
    tube = [0.05, 0.0, -1.0, 0.05, 0.0, 3.0, 1.0, 1.0]
    parts = np.array([[tube] + [small] * 9])
    ones = np.ones((48, 64))
    se, sr = PT.camera_terms(cam, parts, ones, ones)
    np.testing.assert_allclose(se, 16 / 160, rtol=1e-14)
    np.testing.assert_allclose(sr, 24 / 240, rtol=1e-14)


def test_degenerate_geometry_counts_as_unmatched():
    """A cylinder with A = B, a NaN radius or an infinite end point has no
    outline: its 16 outline and 24 silhouette points count p = 0 in every view
    (here every other point reads 1)."""
    cams, parts = _visible_scene()
    parts = parts[:3].astype(np.float64).copy()
    parts[0, 2, 3:6] = parts[0, 2, 0:3]
    parts[1, 7, 7] = np.nan
    parts[2, 4, 1] = np.inf
    for cam in cams:
        ones = np.ones((cam.height, cam.width))
        se, sr = PT.camera_terms(cam, parts, ones, ones)
        np.testing.assert_allclose(se, 16 / 160, rtol=1e-14)
        np.testing.assert_allclose(sr, 24 / 240, rtol=1e-14)


def test_image_borders():
    """Cylinders leaving the image across each of its four borders:
    4 of their 8 cross-sections land on pixels inside (map value 1), the other
    4 on the first pixels outside (value 0)."""
    cam = Cam(64, 48, HAND_P)
    hid = [-1.0, 0.0, -5.0, 1.0, 0.0, -5.0, 0.1, 0.1]
    right = [27.2, 0.0, 10.0, 35.2, 0.0, 10.0, 0.01, 0.01]     # columns 60..67
    bottom = [0.0, 19.2, 10.0, 0.0, 27.2, 10.0, 0.01, 0.01]    # rows 44..51
    left = [-36.8, 0.0, 10.0, -28.8, 0.0, 10.0, 0.01, 0.01]    # columns -4..3
    top = [0.0, -28.2, 10.0, 0.0, -20.2, 10.0, 0.01, 0.01]     # rows -4..3
    parts = np.array([[c] + [hid] * 9 for c in (right, bottom, left, top)])
    ones = np.ones((48, 64))
    se, sr = PT.camera_terms(cam, parts, ones, ones)
    np.testing.assert_allclose(se, 1 - 8 / 160, rtol=1e-14)
    np.testing.assert_allclose(sr, 1 - 12 / 240, rtol=1e-14)


def _ambiguous(cams, parts, tol=1e-7):
    """Particles with a sample point within tol of a pixel boundary in some view."""
    bad = np.zeros(parts.shape[0], bool)
    for cam in cams:
        edge, region, valid = PT.sample_points(np.asarray(parts, np.float64), PT.camera_centre(cam.P))
        for pts in (edge, region):
            x, y, _ = PT.image_coords(cam, pts)
            near = (np.abs(x - np.round(x)) < tol) | (np.abs(y - np.round(y)) < tol)
            bad |= near.reshape(parts.shape[0], -1).any(axis=1)
    return bad


def _random_maps(cams, seed):
    rng = np.random.default_rng(seed)
    return ([rng.random((c.height, c.width)) for c in cams], [rng.random((c.height, c.width)) for c in cams])


def test_rigid_motion_and_scale_invariance():
    """Moving and scaling the whole world (cylinders and cameras together) leaves
    every image point, hence every weight, unchanged."""
    cams, parts = _visible_scene()
    parts = parts.astype(np.float64)
    Sm, Em = _random_maps(cams, 3)
    lw = PT.log_weights(cams, parts, Sm, Em)
    rng = np.random.default_rng(9)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    Q *= np.sign(np.linalg.det(Q))
    t = rng.normal(size=3)
    s = 2.5
    T = np.eye(4)
    T[:3, :3], T[:3, 3] = s * Q, t                       # world -> new world
    Tinv = np.linalg.inv(T)
    cams2 = [Cam(c.width, c.height, np.asarray(c.P, np.float64).reshape(3, 4) @ Tinv) for c in cams]
    parts2 = parts.copy()
    for o in (0, 3):
        parts2[..., o:o + 3] = parts[..., o:o + 3] @ (s * Q).T + t
    parts2[..., 6:8] *= s
    ok = ~(_ambiguous(cams, parts) | _ambiguous(cams2, parts2))
    assert ok.sum() >= parts.shape[0] - 1
    lw2 = PT.log_weights(cams2, parts2, Sm, Em)
    np.testing.assert_allclose(lw2[ok], lw[ok], rtol=0, atol=1e-12)


def test_order_of_cameras_and_particles():
    cams, parts = _visible_scene()
    Sm, Em = _random_maps(cams, 4)
    lw = PT.log_weights(cams, parts, Sm, Em)
    perm = [2, 0, 3, 1]
    lw_c = PT.log_weights([cams[k] for k in perm], parts, [Sm[k] for k in perm], [Em[k] for k in perm])
    np.testing.assert_allclose(lw_c, lw, rtol=0, atol=1e-13)
    pp = np.random.default_rng(1).permutation(parts.shape[0])
    np.testing.assert_allclose(PT.log_weights(cams, parts[pp], Sm, Em), lw[pp], rtol=0, atol=0)
    # distinct maps give distinct weights: a swapped map pair is noticed
    lw_swap = PT.log_weights(cams, parts, Em, Sm)
    assert np.max(np.abs(lw_swap - lw)) > 1e-3


def test_normalised_weights():
    lw = np.array([-3.0, -1.0, -2.5, -1.0, -40.0])
    w = PT.normalised(lw)
    assert abs(w.sum() - 1.0) < 1e-15
    np.testing.assert_allclose(w[1] / w[0], np.exp(2.0), rtol=1e-14)
    np.testing.assert_allclose(PT.normalised(lw, 0.0), np.full(5, 0.2), rtol=1e-15)
    np.testing.assert_allclose(PT.normalised(lw, 2.0), PT.normalised(2.0 * lw), rtol=1e-15)
    # shifting every log weight does not change the normalised weights, even far out
    np.testing.assert_allclose(PT.normalised(lw - 1e4), w, rtol=1e-12)
    assert PT.normalised(np.array([-5.0]))[0] == 1.0
