"""Pins of the oracle's nearest-pixel rule near rounding boundaries, and of
its per-pixel likelihood and pixel chain at hand-computed points.

No GPU. The candidate pixels the oracle admits when a projected voxel centre
lies within eps of a rounding boundary decide every GPU validity check on
ambiguous voxels; these tests fix the exact candidate sets, the number of
choice combinations, the bounds and every combination's posterior from
hand-derived fractions (tests/golden/ambiguity_cases.json), so that taking the
neighbour on the wrong side, dropping it, or widening the band fails here.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O
from synth import scene as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


AMB = _load("ambiguity_cases.json")


def _scene(case):
    sc = AMB["scene"]
    g = sc["grid"]
    grid = S.Grid(g["nx"], g["ny"], g["nz"], np.array(g["origin"], np.float32), np.float32(g["voxel"]))
    W, H = sc["image"]["width"], sc["image"]["height"]
    cams = []
    for bx, by in case["views"]:
        P = np.array([[1, 0, 0, float(bx)], [0, 1, 0, float(by)], [0, 0, 0, 1]], np.float32)
        cams.append(S.Camera(W, H, P))
    k = np.arange(W * H, dtype=np.float64).reshape(H, W)
    smap = (k + 1.0) / 32.0
    return cams, grid, [smap] * len(cams)


def _f(s):
    return float(Fraction(s))


@pytest.mark.parametrize("case", AMB["cases"], ids=[c["name"] for c in AMB["cases"]])
def test_ambiguity_candidates(case):
    cams, grid, maps = _scene(case)
    eps = AMB["scene"]["eps_px"]
    post = O.posterior(cams, grid, maps, prior=AMB["scene"]["prior"], eps_px=eps)
    want_all = sorted(_f(p) for p in case["p_all"])
    ncand = int(np.prod([len(c) for c in case["candidates"]]))
    assert ncand == len(want_all)
    # canonical posterior, number of combinations, bounds
    assert post.post.reshape(-1)[0] == pytest.approx(_f(case["p_canonical"]), rel=1e-14)
    assert int(post.ncombo.reshape(-1)[0]) == ncand
    assert post.lo.reshape(-1)[0] == pytest.approx(want_all[0], rel=1e-14)
    assert post.hi.reshape(-1)[0] == pytest.approx(want_all[-1], rel=1e-14)
    # every combination, the canonical one first
    vals = O.voxel_combos(cams, grid, maps, 0, prior=AMB["scene"]["prior"], eps_px=eps)
    assert len(vals) == ncand
    assert vals[0] == pytest.approx(_f(case["p_canonical"]), rel=1e-14)
    np.testing.assert_allclose(np.sort(vals), want_all, rtol=1e-14)


def test_ambiguity_band_closed_at_zero_eps():
    # with eps = 0 only the canonical pixel is admissible, even on a tie
    for case in AMB["cases"]:
        cams, grid, maps = _scene(case)
        post = O.posterior(cams, grid, maps, eps_px=0.0)
        assert int(post.ncombo.reshape(-1)[0]) == 1
        assert post.post.reshape(-1)[0] == pytest.approx(_f(case["p_canonical"]), rel=1e-14)
        assert post.lo.reshape(-1)[0] == post.hi.reshape(-1)[0] == post.post.reshape(-1)[0]


def test_ambiguity_on_a_grid_of_voxels():
    # a 4 x 3 x 2 grid seen by one affine camera whose voxel centres land
    # 1e-4 px past a boundary in x (every voxel ambiguous in x only); the
    # neighbour is the pixel to the left; the last column and row project
    # outside the image
    grid = S.Grid(4, 3, 2, np.array([0.0, 0.0, 0.0], np.float32), np.float32(1.0))
    P = np.array([[1, 0, 0, 0.0001], [0, 1, 0, 0.5], [0, 0, 0, 1]], np.float32)
    cam = S.Camera(4, 3, P)
    k = np.arange(12, dtype=np.float64).reshape(3, 4)
    smap = (k + 1.0) / 32.0
    post = O.posterior([cam], grid, [smap], eps_px=1e-3)
    for z in range(2):
        for j in range(3):
            for i in range(4):
                # u + 1/2 = i + 1 + 1e-4: x = i + 1, neighbour x = i; v + 1/2 = j + 1.5: y = j + 1
                y = j + 1
                def p_of(x):
                    if not (0 <= x < 4 and 0 <= y < 3):
                        return 0.5
                    kk = 4 * y + x
                    return (kk + 1) / (kk + 17)
                want = sorted([p_of(i + 1), p_of(i)])
                assert post.post[z, j, i] == pytest.approx(p_of(i + 1), rel=1e-14)
                assert post.lo[z, j, i] == pytest.approx(want[0], rel=1e-14)
                assert post.hi[z, j, i] == pytest.approx(want[1], rel=1e-14)
                assert post.ncombo[z, j, i] == 2


# ----------------------------------------------- Eq. 1-2 and the pixel chain

SLM = _load("slm_hand_cases.json")


@pytest.mark.parametrize("case", SLM["cases"], ids=["equal-25", "equal-225", "offset"])
def test_log2slm_hand_values(case):
    img = np.array([case["I"]], np.uint8)
    mean = np.array([case["mean"]], np.float32)
    var = np.array([case["var"]], np.float32)
    got = O.log2slm(img, mean, var, -3 * math.log(256.0))[0]
    assert got == pytest.approx(case["log2slm"], rel=1e-13)
    s = O.slm(img, mean, var, -3 * math.log(256.0))[0]
    # SLM = sigmoid(-d)
    assert s == pytest.approx(1.0 / (1.0 + math.exp(case["d"])), rel=1e-12)


def test_pixel_chain_hand_values():
    # one pixel seen by one voxel whose centre projects exactly onto it
    # (bilinear weight 1): the logit is log(2 SLM) of the pixel (prior 1/2),
    # and with label 0 the adjoint of that pixel is sigmoid(logit); the
    # oracle's mean / variance gradients divided by it are the pixel chain
    case = SLM["cases"][2]
    img = np.array(case["I"], np.uint8).reshape(1, 1, 3)
    mean = np.array(case["mean"], np.float32).reshape(1, 1, 3)
    var = np.array(case["var"], np.float32).reshape(1, 1, 3)
    grid = S.Grid(1, 1, 1, np.array([0.0, 0.0, 0.0], np.float32), np.float32(1.0))
    P = np.array([[1, 0, 0, -0.5], [0, 1, 0, -0.5], [0, 0, 0, 1]], np.float32)
    cam = S.Camera(1, 1, P)
    L = O.bilinear_logits([cam], grid, [O.log2slm(img, mean, var)])
    assert L.reshape(-1)[0] == pytest.approx(case["log2slm"], rel=1e-13)
    labels = np.zeros((1, 1, 1), np.uint8)
    gm, gv, gP = O.grad([cam], grid, [img], [mean], [var], labels)
    adj = 1.0 / (1.0 + math.exp(-case["log2slm"]))
    np.testing.assert_allclose(gm[0].reshape(3) / adj, case["dl_dmean"], rtol=1e-12)
    np.testing.assert_allclose(gv[0].reshape(3) / adj, case["dl_dvar"], rtol=1e-12)
