"""Pins of the FP64 oracle against what the paper and the mathematics fix.

No GPU. Each test pins a part of the oracle to something other than itself:
hand-derived exact values, closed forms, a library Gaussian density, a literal
brute-force evaluation of Eq. 3-9 with pixel search by containment, the
classical visual hull (Sec. 2.2.1), invariants, and finite differences.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.stats
import torch

from oracle import literal
from oracle import oracle as O
from synth import scene as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# ------------------------------------------------------------- Eq. 3-9 values

def test_fuse_views_hand_cases():
    g = _load("fuse_hand_cases.json")
    for case in g["cases"]:
        want = float(Fraction(case["p"]))
        got = O.fuse_views(case["s"], case["prior"])
        assert got == pytest.approx(want, rel=1e-14, abs=1e-300), case


def test_fuse_views_closed_form_random():
    # Closed form of Eq. 5-9: each seeing view multiplies the odds by 2*SLM,
    # p = prior*prod(s) / (prior*prod(s) + (1-prior)*2^-m), evaluated exactly.
    rng = np.random.default_rng(7)
    for _ in range(400):
        m = int(rng.integers(0, 9))
        s = rng.uniform(0.0, 1.0, m)
        prior = float(rng.choice([0.2, 0.5, 0.8]))
        num = Fraction(prior)
        for v in s:
            num *= Fraction(float(v))
        den = num + (1 - Fraction(prior)) * Fraction(1, 2 ** m)
        want = float(num / den)
        assert O.fuse_views(s, prior) == pytest.approx(want, rel=1e-13)


def test_literal_view_terms_reduce_to_slm_and_half():
    # Eq. 5 with Eq. 6-9 and P(O)=1/2: P(S|V=1) = s and P(S|V=0) = 1/2.
    for s in (0.0, 0.1, 0.5, 0.93, 1.0):
        assert literal.view_term(s, 1) == pytest.approx(s, abs=1e-16)
        assert literal.view_term(s, 0) == pytest.approx(0.5, abs=1e-16)


# ------------------------------------------------------------------- Eq. 1-2

def test_slm_against_library_gaussian():
    rng = np.random.default_rng(3)
    img = rng.integers(0, 256, (50, 3)).astype(np.uint8)
    mean = rng.uniform(0, 255, (50, 3)).astype(np.float32)
    var = rng.uniform(4, 400, (50, 3)).astype(np.float32)
    log_u = -3 * math.log(256.0)
    got = O.slm(img, mean, var, log_u)
    for p in range(50):
        dens = scipy.stats.multivariate_normal.pdf(img[p].astype(np.float64), mean[p].astype(np.float64),
                                                   np.diag(var[p].astype(np.float64)))
        u = math.exp(log_u)
        # Eq. 1 with P(F=1) = P(F=0): the priors cancel
        assert got[p] == pytest.approx(u / (u + dens), rel=1e-12)


def test_slm_special_cases():
    # I = mu: the density is (2 pi v)^(-3/2) for equal channel variances.
    log_u = -3 * math.log(256.0)
    for v in (25.0, 225.0):
        img = np.array([[10, 200, 77]], np.uint8)
        got = O.slm(img, img.astype(np.float32), np.full((1, 3), v, np.float32), log_u)[0]
        want = 1.0 / (1.0 + (2 * math.pi * v) ** -1.5 * 256.0 ** 3)
        assert got == pytest.approx(want, rel=1e-13)
    # the variance at which the background density at I = mu equals the
    # uniform density makes the SLM exactly 1/2
    v = np.float32(256.0 ** 2 / (2 * math.pi))
    img = np.array([[128, 128, 128]], np.uint8)
    got = O.slm(img, img.astype(np.float32), np.full((1, 3), v, np.float32), log_u)[0]
    assert got == pytest.approx(0.5, abs=1e-6)
    # far from the mean (outlier) the pixel is foreground with certainty
    got = O.slm(np.array([[255, 255, 255]], np.uint8), np.zeros((1, 3), np.float32),
                np.full((1, 3), 25.0, np.float32), log_u)[0]
    assert got == 1.0


def test_slm_rejects_bad_variance():
    img = np.zeros((2, 3), np.uint8)
    with pytest.raises(ValueError):
        O.slm(img, np.zeros((2, 3), np.float32), np.array([[1, 1, 1], [1, 0, 1]], np.float32))
    with pytest.raises(ValueError):
        O.slm(img, np.zeros((2, 3), np.float32), np.array([[1, 1, 1], [1, np.nan, 1]], np.float32))


def test_slm_monotone_in_distance():
    mean = np.full((1, 3), 100.0, np.float32)
    var = np.full((1, 3), 50.0, np.float32)
    vals = [O.slm(np.array([[100 + d, 100, 100]], np.uint8), mean, var)[0] for d in range(0, 60, 3)]
    assert all(b >= a for a, b in zip(vals, vals[1:]))


# ---------------------------------------------------- tiny scenes, brute force

def _tiny_scene(seed, affine_ties=False):
    rng = np.random.default_rng(seed)
    grid = S.Grid(6, 5, 4, np.array([-0.6, -0.5, -0.4], np.float32), np.float32(0.2))
    cams = []
    for k in range(3):
        th = rng.uniform(0, 2 * np.pi)
        cams.append(S.look_at_camera((3 * np.cos(th), 3 * np.sin(th), rng.uniform(-1, 2)),
                                     f=rng.uniform(6, 14), W=int(rng.integers(8, 14)), H=int(rng.integers(6, 12))))
    if affine_ties:
        # affine camera: voxel centres land exactly on half-integer coordinates
        h = 0.25
        grid = S.Grid(5, 4, 3, np.array([-1.0, -1.0, -1.0], np.float32), np.float32(h))
        P = np.array([[1 / h, 0, 0, 1 / h], [0, 1 / h, 0, 1 / h], [0, 0, 0, 1]], np.float32)
        cams.append(S.Camera(5, 4, P))
    maps = [rng.uniform(0.0, 1.0, (c.height, c.width)) for c in cams]
    return cams, grid, maps


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_oracle_matches_literal_bruteforce(seed):
    cams, grid, maps = _tiny_scene(seed)
    got = O.posterior(cams, grid, maps, prior=0.4)
    want = np.array(literal.posterior_grid(cams, grid, maps, prior=0.4))
    np.testing.assert_allclose(got.post, want, rtol=1e-12, atol=1e-300)
    assert np.any(got.post != 0.4)      # not vacuous: some voxels are seen


def test_oracle_matches_literal_voxels_behind_camera():
    # a camera inside the grid: voxels behind it would project (point-reflected)
    # into the image if the depth test were missing
    rng = np.random.default_rng(21)
    grid = S.Grid(6, 5, 4, np.array([-0.6, -0.5, -0.4], np.float32), np.float32(0.2))
    cam = S.look_at_camera((0.05, 0.02, 0.01), f=4.0, W=12, H=10, target=(3.0, 0.3, 0.2))
    smap = rng.uniform(0.0, 1.0, (10, 12))
    got = O.posterior([cam], grid, [smap], prior=0.5).post
    want = np.array(literal.posterior_grid([cam], grid, [smap], prior=0.5))
    np.testing.assert_allclose(got, want, rtol=1e-12)
    xs, ys, zs = grid.centres64()
    behind_in_image = 0
    for z in zs:
        for y in ys:
            for x in xs:
                xc = cam.R @ (np.array([x, y, z]) - cam.C)
                if xc[2] < 0:
                    u = 4.0 * xc[0] / xc[2] + 6.0
                    v = 4.0 * xc[1] / xc[2] + 5.0
                    behind_in_image += (0 <= math.floor(u + 0.5) < 12) and (0 <= math.floor(v + 0.5) < 10)
    assert behind_in_image > 0
    assert np.any(got != 0.5) and np.any(got == 0.5)


def test_oracle_half_pixel_ties_round_up():
    cams, grid, maps = _tiny_scene(5, affine_ties=True)
    aff = cams[-1:]
    amap = maps[-1:]
    got = O.posterior(aff, grid, amap, prior=0.5)
    want = np.array(literal.posterior_grid(aff, grid, amap, prior=0.5))
    np.testing.assert_allclose(got.post, want, rtol=1e-14)
    # every projection sits on a tie, so every seen voxel is flagged ambiguous
    seen = got.post != 0.5
    assert np.all(got.ncombo[seen] >= 2)
    # voxel (i, j) projects to (i + 1/2, j + 1/2) -> pixel (i + 1, j + 1)
    s = amap[0]
    for j in range(3):
        for i in range(4):
            p = got.post[0, j, i]
            assert p == pytest.approx(s[j + 1, i + 1] / (s[j + 1, i + 1] + 0.5), rel=1e-14)


def test_ambiguity_combos_contain_canonical():
    cams, grid, maps = _tiny_scene(5, affine_ties=True)
    post = O.posterior(cams, grid, maps)
    flat = post.post.reshape(-1)
    for v in np.flatnonzero(post.ambiguous.reshape(-1))[:20]:
        vals = O.voxel_combos(cams, grid, maps, int(v))
        assert len(vals) == post.ncombo.reshape(-1)[v]
        assert np.min(np.abs(vals - flat[v])) == 0.0
        assert post.lo.reshape(-1)[v] == pytest.approx(vals.min(), rel=1e-14)
        assert post.hi.reshape(-1)[v] == pytest.approx(vals.max(), rel=1e-14)


def test_closed_form_log_domain_on_scene():
    # logit p = logit prior + sum over seeing views of log(2*SLM) (Eq. 3-9 closed form)
    cams, grid, maps = _tiny_scene(11)
    prior = 0.3
    got = O.posterior(cams, grid, maps, prior=prior).post
    # independent per-voxel projection through K, R, C rather than the 3x4 matrix
    xs, ys, zs = grid.centres64()
    for k in range(grid.nz):
        for j in range(grid.ny):
            for i in range(grid.nx):
                X = np.array([xs[i], ys[j], zs[k]])
                L = math.log(prior / (1 - prior))
                for cam, m in zip(cams, maps):
                    xc = cam.R @ (X - cam.C)
                    if xc[2] <= 0:
                        continue
                    u = cam.K[0, 0] * xc[0] / xc[2] + cam.K[0, 2]
                    v = cam.K[1, 1] * xc[1] / xc[2] + cam.K[1, 2]
                    x, y = math.floor(u + 0.5), math.floor(v + 0.5)
                    if 0 <= x < cam.width and 0 <= y < cam.height:
                        L += math.log(2 * m[y, x])
                want = 1 / (1 + math.exp(-L))
                # K,R,C differ from the FP32-rounded P by ~1e-6 px: compare where unambiguous
                assert got[k, j, i] == pytest.approx(want, rel=1e-9, abs=1e-12)


# ------------------------------------------------------------------ invariants

@pytest.fixture(scope="module")
def c0():
    return S.config_frame(0, 0)


def test_invariants_bounds_and_unseen(c0):
    maps, post, occ = O.reconstruct(c0.cams, c0.grid, c0.images, c0.mean, c0.var)
    n = c0.n
    upper = 2 ** n * 0.5 / (2 ** n * 0.5 + 0.5)
    assert post.post.min() >= 0.0 and post.post.max() <= upper + 1e-15
    # a grid far outside every frustum keeps the prior
    far = S.Grid(4, 4, 4, np.array([50.0, 50.0, 50.0], np.float32), np.float32(0.1))
    p = O.posterior(c0.cams, far, maps, prior=0.37).post
    assert np.all(p == 0.37)
    # occupancy is a superset of nothing: the body is reconstructed
    gt = S.gt_occupancy(c0.grid, c0.body)
    assert occ[gt == 1].mean() > 0.9


def test_invariant_camera_permutation(c0):
    maps, post, _ = O.reconstruct(c0.cams, c0.grid, c0.images, c0.mean, c0.var)
    perm = [2, 0, 3, 1]
    p2 = O.posterior([c0.cams[i] for i in perm], c0.grid, [maps[i] for i in perm]).post
    np.testing.assert_allclose(p2, post.post, rtol=1e-12, atol=1e-300)


def test_invariant_all_background_gives_empty_grid(c0):
    # images equal to an integer-valued background mean: every seeing view has SLM < 1/2
    rng = np.random.default_rng(1)
    imgs, means = [], []
    for c in c0.cams:
        im = rng.integers(0, 256, (c.height, c.width, 3)).astype(np.uint8)
        imgs.append(im)
        means.append(im.astype(np.float32))
    vars_ = [np.full(m.shape, 225.0, np.float32) for m in means]
    _, post, occ = O.reconstruct(c0.cams, c0.grid, imgs, means, vars_)
    assert occ.sum() == 0
    assert post.post.max() <= 0.5


def test_invariant_uninformative_camera(c0):
    maps, post, _ = O.reconstruct(c0.cams, c0.grid, c0.images, c0.mean, c0.var)
    half = [np.full_like(maps[0], 0.5)]
    p = O.posterior(c0.cams + [c0.cams[0]], c0.grid, maps + half).post
    np.testing.assert_allclose(p, post.post, rtol=1e-12, atol=1e-300)


def test_invariant_monotone_in_slm(c0):
    maps, post, _ = O.reconstruct(c0.cams, c0.grid, c0.images, c0.mean, c0.var)
    up = [m.copy() for m in maps]
    up[1] = np.minimum(1.0, up[1] * 1.5)
    p = O.posterior(c0.cams, c0.grid, up).post
    assert np.all(p >= post.post - 1e-15)


# --------------------------------------------------------- visual-hull limit

def test_visual_hull_limit():
    """Near-binary silhouettes reduce the method to classical shape from silhouette
    (Sec. 2.2.1): a voxel seen by >= 1 view is occupied iff every seeing view's
    pixel is foreground (here n*log 2 < log(1/(2 SLM_bg)) with SLM_bg from v = 25)."""
    fr = S.config_frame(0, 3)
    rng = np.random.default_rng(9)
    imgs, means, vars_ = [], [], []
    for cam, mask in zip(fr.cams, fr.masks):
        mu = rng.integers(70, 186, (cam.height, cam.width, 3)).astype(np.float32)
        im = mu.copy()
        im[mask, 0] = np.where(mu[mask, 0] > 127, mu[mask, 0] - 65, mu[mask, 0] + 65)
        imgs.append(im.astype(np.uint8))
        means.append(mu)
        vars_.append(np.full(mu.shape, 25.0, np.float32))
    _, post, occ = O.reconstruct(fr.cams, fr.grid, imgs, means, vars_)
    # brute-force cone intersection with the textbook projection x = K R (X - C)
    xs, ys, zs = fr.grid.centres64()
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    pts = np.stack([X, Y, Z], -1).reshape(-1, 3)
    inside = np.ones(len(pts), bool)
    seen = np.zeros(len(pts), bool)
    ambiguous = np.zeros(len(pts), bool)
    for cam, mask in zip(fr.cams, fr.masks):
        xc = (pts - cam.C) @ cam.R.T
        u = cam.K[0, 0] * xc[:, 0] / xc[:, 2] + cam.K[0, 2]
        v = cam.K[1, 1] * xc[:, 1] / xc[:, 2] + cam.K[1, 2]
        x, y = np.floor(u + 0.5).astype(int), np.floor(v + 0.5).astype(int)
        ok = (xc[:, 2] > 0) & (x >= 0) & (x < cam.width) & (y >= 0) & (y < cam.height)
        fg = np.zeros(len(pts), bool)
        fg[ok] = mask[y[ok], x[ok]]
        inside &= ~ok | fg
        seen |= ok
        ru, rv = u + 0.5 - np.floor(u + 0.5), v + 0.5 - np.floor(v + 0.5)
        ambiguous |= (np.minimum(ru, 1 - ru) < 1e-6) | (np.minimum(rv, 1 - rv) < 1e-6)
    hull = (inside & seen).reshape(occ.shape)
    keep = ~ambiguous.reshape(occ.shape)
    assert hull.sum() > 100
    assert np.array_equal(occ.astype(bool)[keep], hull[keep])


# ------------------------------------------------------ differentiable variant

def test_bilinear_hand_case():
    g = _load("bilinear_hand_case.json")
    # one voxel, one affine camera placing the centre at (2 + fx, 1 + fy)
    grid = S.Grid(1, 1, 1, np.array([0.0, 0.0, 0.0], np.float32), np.float32(1.0))
    P = np.array([[1, 0, 0, 2 + g["fx"] - 0.5], [0, 1, 0, 1 + g["fy"] - 0.5], [0, 0, 0, 1]], np.float32)
    cam = S.Camera(5, 4, P)
    l2s = np.zeros((4, 5))
    t = g["taps"]
    l2s[1, 2], l2s[1, 3], l2s[2, 2], l2s[2, 3] = t["l00"], t["l10"], t["l01"], t["l11"]
    L = O.bilinear_logits([cam], grid, [l2s], prior=0.5)
    assert L[0, 0, 0] == pytest.approx(g["value"], abs=1e-15)
    # the u and v slopes by central differences of the oracle (linear in u inside a cell)
    for key, col in (("d_du", 0), ("d_dv", 1)):
        Pp, Pm = P.astype(np.float64).copy(), P.astype(np.float64).copy()
        Pp[col, 3] += 1e-3
        Pm[col, 3] -= 1e-3
        Lp = O.bilinear_logits([S.Camera(5, 4, Pp)], grid, [l2s])[0, 0, 0]
        Lm = O.bilinear_logits([S.Camera(5, 4, Pm)], grid, [l2s])[0, 0, 0]
        assert (Lp - Lm) / 2e-3 == pytest.approx(g[key], rel=1e-9)


def test_bilinear_equals_nearest_on_integer_projections():
    # affine camera with unit pixel pitch per voxel: every centre lands on an
    # integer pixel, so the bilinear weights are (1, 0, 0, 0)
    h = 0.125
    grid = S.Grid(7, 6, 3, np.array([0.0, 0.0, 0.0], np.float32), np.float32(h))
    P = np.array([[1 / h, 0, 0, -0.5], [0, 1 / h, 0, -0.5], [0, 0, 0, 1]], np.float32)
    rng = np.random.default_rng(2)
    cams = [S.Camera(7, 6, P), S.Camera(7, 6, P)]
    maps = [rng.uniform(0.01, 1.0, (6, 7)) for _ in cams]
    near = O.posterior(cams, grid, maps, prior=0.5).post
    L = O.bilinear_logits(cams, grid, [np.log(2 * m) for m in maps], prior=0.5)
    np.testing.assert_allclose(1 / (1 + np.exp(-L)), near, rtol=1e-13)


def test_bce_against_torch():
    rng = np.random.default_rng(4)
    L = rng.normal(0, 5, (5, 6, 7))
    y = (rng.random((5, 6, 7)) < 0.3).astype(np.uint8)
    sub = [1, 5, 0, 4, 2, 5]
    got = O.bce_loss(L, y, sub)
    Lt = torch.from_numpy(L[2:5, 0:4, 1:5].copy())
    yt = torch.from_numpy(y[2:5, 0:4, 1:5].astype(np.float64))
    want = torch.nn.functional.binary_cross_entropy_with_logits(Lt, yt).item()
    assert got == pytest.approx(want, rel=1e-14)
    assert O.bce_loss(L, y) == pytest.approx(
        torch.nn.functional.binary_cross_entropy_with_logits(torch.from_numpy(L), torch.from_numpy(y.astype(np.float64))).item(),
        rel=1e-14)


def _fd_scene():
    fr = S.config_frame(0, 1)
    grid = S.Grid(24, 24, 24, np.array([-0.375, -0.375, -0.5], np.float32), np.float32(2.0 / 64))
    cams = S.perturb_cameras(fr.cams[:3], seed=(40, 0))
    labels = S.gt_occupancy(grid, fr.body)
    sub = [4, 20, 4, 20, 4, 20]
    return fr, grid, cams, labels, sub


def test_gradient_matches_finite_differences():
    fr, grid, cams, labels, sub = _fd_scene()
    cams64 = [S.Camera(c.width, c.height, c.P.astype(np.float64)) for c in cams]
    imgs, means, vars_ = fr.images[:3], fr.mean[:3], fr.var[:3]
    gm, gv, gP = O.grad(cams64, grid, imgs, means, vars_, labels, sub, grad_loss=1.0)

    def loss(cs=cams64, ms=means, vs=vars_):
        return O.loss(cs, grid, imgs, ms, vs, labels, sub)

    # background means and variances: steps exactly representable in FP32
    rng = np.random.default_rng(0)
    adj_pix = np.argwhere(np.abs(gm[0]).sum(-1) > 0)
    assert len(adj_pix) > 50
    for y, x in adj_pix[rng.choice(len(adj_pix), 12, replace=False)]:
        c = int(rng.integers(0, 3))
        for arr, g, hstep in ((means, gm, 2.0 ** -8), (vars_, gv, 2.0 ** -8)):
            p, m = [a.copy() for a in arr], [a.copy() for a in arr]
            p[0][y, x, c] += np.float32(hstep)
            m[0][y, x, c] -= np.float32(hstep)
            d = float(p[0][y, x, c]) - float(m[0][y, x, c])
            fd = (loss(ms=p) if arr is means else loss(vs=p)) - (loss(ms=m) if arr is means else loss(vs=m))
            fd /= d
            assert fd == pytest.approx(g[0][y, x, c], rel=2e-5, abs=1e-12 + 1e-6 * np.abs(g[0]).max())

    # camera matrices (FP64 perturbation; a small step keeps taps in their cells)
    for k in range(3):
        for e in range(12):
            r, q = divmod(e, 4)
            base = cams64[k].P[r, q]
            hstep = 1e-7 * max(1.0, abs(base))
            cp = [S.Camera(c.width, c.height, c.P.copy()) for c in cams64]
            cm = [S.Camera(c.width, c.height, c.P.copy()) for c in cams64]
            cp[k].P[r, q] += hstep
            cm[k].P[r, q] -= hstep
            fd = (loss(cs=cp) - loss(cs=cm)) / (2 * hstep)
            scale = np.abs(gP[k]).max()
            assert fd == pytest.approx(gP[k, r, q], rel=1e-4, abs=1e-5 * scale), (k, r, q)


def test_gradient_zero_outside_loss_region():
    fr, grid, cams, labels, sub = _fd_scene()
    tiny = [0, 1, 0, 1, 0, 1]   # one voxel
    gm, gv, gP = O.grad(cams, grid, fr.images[:3], fr.mean[:3], fr.var[:3], labels, tiny)
    touched = sum(int((np.abs(g).sum(-1) > 0).sum()) for g in gm)
    assert touched <= 3 * 4       # at most 4 taps in each of 3 views
