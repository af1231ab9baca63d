"""GPU particle weights (Sec. 2.3.2, Eq. 14-16, normalised as in Eq. 10)
against the FP64 oracle (oracle/particles.py), through the C ABI.

Both sides compute the sample points and their projections in FP64 from the
same FP32 inputs; they differ only in rounding order (~1e-13 px), so a
particle is compared only if none of its sample points lies within 1e-7 px of
a pixel boundary in any view (at most a few in a thousand do). Log weights and
per-view terms then agree to 1e-12 (sums of at most 400 values in [0, 1] per
view, FP64), normalised weights to a relative 1e-12."""
import sys
from dataclasses import dataclass

import numpy as np
import pytest
import torch

import paper_1311_6811_amd as psfs
from oracle import particles as PT
from synth import scene as S

pytestmark = pytest.mark.gpu

LOGW_ATOL = 1e-12
W_RTOL = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@dataclass
class Cam:
    width: int
    height: int
    P: np.ndarray


def ambiguous(cams, parts, tol=1e-7):
    bad = np.zeros(parts.shape[0], bool)
    for cam in cams:
        edge, region, _ = PT.sample_points(np.asarray(parts, np.float64), PT.camera_centre(cam.P))
        for pts in (edge, region):
            x, y, _ = PT.image_coords(cam, pts)
            near = (np.abs(x - np.round(x)) < tol) | (np.abs(y - np.round(y)) < tol)
            bad |= near.reshape(parts.shape[0], -1).any(axis=1)
    return bad


def to_dev(arrs):
    return [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda() for a in arrs]


def run(cams, parts, Sm, Em, beta=1.0):
    plan = psfs.Plan(cams)
    cyl = torch.from_numpy(np.ascontiguousarray(parts, dtype=np.float32)).cuda()
    lw, w, t = plan.particle_weights(cyl, to_dev(Sm), to_dev(Em), beta=beta, weights=True, terms=True)
    torch.cuda.synchronize()
    return lw.cpu().numpy(), w.cpu().numpy(), t.cpu().numpy()


def check(cams, parts, Sm, Em, beta=1.0):
    parts = np.asarray(parts, np.float32)
    lw, w, t = run(cams, parts, Sm, Em, beta)
    keep = ~ambiguous(cams, parts)
    assert keep.mean() >= 0.95, f"{(~keep).sum()} particles have a sample point on a pixel boundary"
    want = PT.log_weights(cams, parts, Sm, Em)
    np.testing.assert_allclose(lw[keep], want[keep], rtol=0, atol=LOGW_ATOL)
    for k, (cam, s, e) in enumerate(zip(cams, Sm, Em)):
        se, sr = PT.camera_terms(cam, parts, s, e)
        np.testing.assert_allclose(t[keep, k, 0], se[keep], rtol=0, atol=1e-13)
        np.testing.assert_allclose(t[keep, k, 1], sr[keep], rtol=0, atol=1e-13)
    # the per-view terms add up to the log weight in view order
    np.testing.assert_array_equal(lw, -np.sum(t, axis=2).cumsum(axis=1)[:, -1])
    # normalisation of the GPU's own log weights (defined for every particle)
    np.testing.assert_allclose(w, PT.normalised(lw, beta), rtol=W_RTOL, atol=0)
    if keep.all():
        np.testing.assert_allclose(w, PT.normalised(want, beta), rtol=W_RTOL, atol=0)
    return lw


@pytest.mark.parametrize("cfg,n_particles", [(0, 64), (1, 200)])
def test_parity_on_tracking_scenes(cfg, n_particles):
    say(f"particle weights, config {cfg}, {n_particles} particles, silhouette/edge maps of the frame")
    cams, parts, Sm, Em = S.tracking_inputs(cfg, 0, n_particles)
    lw = check(cams, parts, Sm, Em)
    assert np.ptp(lw) > 0.1               # the particles are told apart


def test_parity_random_maps_and_beta():
    """Uniform random maps: every pixel holds a distinct value, so reading a
    neighbouring pixel or the other map shows."""
    say("particle weights, random maps, beta 0.3")
    cams, parts, _, _ = S.tracking_inputs(0, 1, 96)
    rng = np.random.default_rng(21)
    Sm = [rng.random((c.height, c.width), dtype=np.float32) for c in cams]
    Em = [rng.random((c.height, c.width), dtype=np.float32) for c in cams]
    check(cams, parts, Sm, Em, beta=0.3)


@pytest.mark.parametrize("n_particles", [1, 1024, 1025])
def test_normalisation_at_the_thread_count(n_particles):
    """Up to 1024 particles the normalisation keeps one particle per thread;
    beyond, each thread loops over several: both sides of the boundary, and a
    single particle (weight exactly 1)."""
    say(f"particle weights, {n_particles} particles, normalisation")
    cams, parts, Sm, Em = S.tracking_inputs(0, 4, n_particles)
    plan = psfs.Plan(cams)
    cyl = torch.from_numpy(np.ascontiguousarray(parts, dtype=np.float32)).cuda()
    lw, w, _ = plan.particle_weights(cyl, to_dev(Sm), to_dev(Em), beta=0.6)
    torch.cuda.synchronize()
    lw, w = lw.cpu().numpy(), w.cpu().numpy()
    np.testing.assert_allclose(w, PT.normalised(lw, 0.6), rtol=W_RTOL, atol=0)
    if n_particles == 1:
        assert w[0] == 1.0


@pytest.mark.parametrize("nviews", [1, 3, 5, 12, 16])
def test_view_counts(nviews):
    """Each view count splits the 80 (cylinder, cross-section) pairs over its
    own number of waves per view (16 // n): one to sixteen."""
    say(f"particle weights, {nviews} views")
    if nviews == 12:
        cams, parts, Sm, Em = S.tracking_inputs(2, 0, 48)
    else:
        cams, parts, Sm, Em = S.tracking_inputs(1, 3, 48)
        idx = [k % len(cams) for k in range(nviews)] if nviews > len(cams) else list(range(0, 8, 8 // nviews))[:nviews]
        cams, Sm, Em = [cams[k] for k in idx], [Sm[k] for k in idx], [Em[k] for k in idx]
    assert len(cams) == nviews
    check(cams, parts, Sm, Em, beta=1.5)


def test_hand_case():
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "particle_hand_case.json")) as fh:
        g = json.load(fh)
    W, H = g["image"]["width"], g["image"]["height"]
    cams = [Cam(W, H, np.asarray(P, np.float32)) for P in g["cameras_P"]]
    vis, hid = g["visible_cylinder"], g["hidden_cylinder"]
    parts = np.array([[vis] + [hid] * 9, [hid] * 10], np.float32)
    maps = {}
    for key, entries in g["maps_nonzero"].items():
        m = np.zeros((H, W), np.float32)
        for r, c, v in entries:
            m[r, c] = v
        maps[key] = m
    lw, w, _ = run(cams, parts, [maps["silhouette_cam0"], maps["silhouette_cam1"]],
                   [maps["edge_cam0"], maps["edge_cam1"]], beta=0.5)
    np.testing.assert_allclose(lw, g["log_w"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(w, g["weights_beta_0.5"], rtol=1e-12)


def test_many_particles_and_reproducible():
    say("particle weights, 3000 particles, twice")
    cams, parts, Sm, Em = S.tracking_inputs(0, 2, 3000)
    lw = check(cams, parts, Sm, Em, beta=2.0)
    lw2, _, _ = run(cams, parts, Sm, Em, beta=2.0)
    assert np.array_equal(lw.view(np.uint64), lw2.view(np.uint64))


def test_degenerate_cases():
    cams, parts, Sm, Em = S.tracking_inputs(0, 0, 8)
    # every cylinder far above the cameras: nothing seen, -2 per view
    up = parts.copy()
    up[..., 2] += 20.0
    up[..., 5] += 20.0
    lw, w, t = run(cams, up, Sm, Em)
    assert np.all(lw == -2.0 * len(cams))
    np.testing.assert_allclose(w, np.full(8, 1 / 8), rtol=1e-15)
    # beta = 0: uniform weights whatever the scores
    lw, w, _ = run(cams, parts, Sm, Em, beta=0.0)
    np.testing.assert_allclose(w, np.full(8, 1 / 8), rtol=1e-15)
    # degenerate cylinders (A = B, NaN radius, infinite end point): unmatched
    bad = parts.copy()
    bad[0, 2, 3:6] = bad[0, 2, 0:3]
    bad[1, 7, 7] = np.nan
    bad[2, 4, 1] = np.inf
    ones = [np.ones((c.height, c.width), np.float32) for c in cams]
    lw, w, t = run(cams, bad, ones, ones)
    want = PT.log_weights(cams, bad, ones, ones)
    np.testing.assert_allclose(lw, want, rtol=0, atol=LOGW_ATOL)
    for k in range(len(cams)):
        se, sr = PT.camera_terms(cams[k], bad, ones[k], ones[k])
        np.testing.assert_allclose(t[:, k, 0], se, rtol=0, atol=1e-13)
        np.testing.assert_allclose(t[:, k, 1], sr, rtol=0, atol=1e-13)
    # no views: log w = 0
    plan = psfs.Plan([])
    cyl = torch.from_numpy(parts).cuda()
    lw, w, t = plan.particle_weights(cyl, [], [], terms=True)
    torch.cuda.synchronize()
    assert np.all(lw.cpu().numpy() == 0.0)
    np.testing.assert_allclose(w.cpu().numpy(), np.full(8, 1 / 8), rtol=1e-15)
    assert t.numel() == 0
    # no particles: a no-op
    plan = psfs.Plan(cams)
    lw, w, t = plan.particle_weights(torch.empty((0, 10, 8), dtype=torch.float32, device="cuda"), to_dev(Sm), to_dev(Em))
    torch.cuda.synchronize()
    assert lw.numel() == 0 and w.numel() == 0


def test_graph_replays_match_eager():
    """Captured once into a HIP graph and replayed three times, with eager
    launches and synchronisations between the replays: every replay gives the
    eager bits."""
    say("particle weights, graph replays")
    cams, parts, Sm, Em = S.tracking_inputs(0, 4, 128)
    plan = psfs.Plan(cams)
    cyl = torch.from_numpy(parts).cuda()
    sil, edg = to_dev(Sm), to_dev(Em)
    out = {"log_w": torch.empty(128, dtype=torch.float64, device="cuda"),
           "weights": torch.empty(128, dtype=torch.float64, device="cuda")}
    lw0, w0, _ = plan.particle_weights(cyl, sil, edg, beta=0.7)
    torch.cuda.synchronize()
    lw0, w0 = lw0.clone(), w0.clone()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan.particle_weights(cyl, sil, edg, beta=0.7, out=out)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            plan.particle_weights(cyl, sil, edg, beta=0.7, out=out)
    for r in range(3):
        out["log_w"].fill_(float("nan"))
        out["weights"].fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out["log_w"], lw0), r
        assert torch.equal(out["weights"], w0), r
        plan.particle_weights(cyl, sil, edg, beta=0.7)      # eager work between replays
        torch.cuda.synchronize()
