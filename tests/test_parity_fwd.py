"""GPU forward path (likelihood maps, fusion, threshold) against the FP64 oracle.

Posterior: within 1e-5 absolute; where a voxel's projection lies within 1e-3 px
of a pixel-rounding boundary in some view, any admissible pixel choice is
correct, so the GPU value must match one of them. Occupancy: bit-exact where
the oracle's posterior is more than 1e-4 from the threshold.
"""
import sys

import numpy as np
import pytest
import torch

import paper_1311_6811_amd as psfs
from oracle import oracle as O
from synth import scene as S
from tests.gpu_util import (assert_occupancy_parity, assert_posterior_parity, plan_for, upload)

pytestmark = pytest.mark.gpu

LMAP_RTOL, LMAP_ATOL = 2e-6, 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_forward(frame, **kw):
    ims, mus, vs = upload(frame)
    plan = plan_for(frame, mus, vs, **kw)
    lmap = plan.likelihood(ims)
    post, occ = plan.fuse(lmap)
    post2, occ2 = plan.reconstruct(ims)
    torch.cuda.synchronize()
    assert torch.equal(post, post2) and torch.equal(occ, occ2)
    return plan, lmap, post, occ


def check_lmaps(plan, lmap, frame, log_u=O.LOG_U_DEFAULT):
    worst = 0.0
    for k in range(frame.n):
        want = O.log2slm(frame.images[k], frame.mean[k], frame.var[k], log_u)
        got = plan.lmap_view(lmap, k).cpu().numpy().astype(np.float64)
        err = np.abs(got - want) - LMAP_RTOL * np.abs(want)
        assert err.max() <= LMAP_ATOL, f"view {k}: lmap error {err.max():.3e}"
        worst = max(worst, float(np.abs(got - want).max()))
    return worst


def oracle_forward(frame, prior=0.5, log_u=O.LOG_U_DEFAULT):
    maps = [O.slm(i, m, v, log_u) for i, m, v in zip(frame.images, frame.mean, frame.var)]
    ref = O.posterior(frame.cams, frame.grid, maps, prior)
    combos = lambda v: O.voxel_combos(frame.cams, frame.grid, maps, v, prior)  # noqa: E731
    return ref, combos


@pytest.mark.parametrize("cfg", [0, 1])
def test_forward_parity_named_workloads(cfg):
    say(f"forward parity config {cfg}")
    fr = S.config_frame(cfg, 0)
    plan, lmap, post, occ = run_forward(fr)
    check_lmaps(plan, lmap, fr)
    ref, combos = oracle_forward(fr)
    worst = assert_posterior_parity(post, ref, combos=combos)
    assert_occupancy_parity(occ, ref)
    say(f"  max posterior error {worst:.2e}, ambiguous {ref.ambiguous.mean():.4f}")


def test_forward_parity_large_grid_12_views():
    say("forward parity 256^3 x 12 views 1280x720")
    fr = S.config_frame(2, 5)
    plan, lmap, post, occ = run_forward(fr)
    check_lmaps(plan, lmap, fr)
    ref, combos = oracle_forward(fr)
    assert_posterior_parity(post, ref, combos=combos, n_enum=100)
    assert_occupancy_parity(occ, ref)


def test_largest_grid_index_range():
    """A 1290^3 grid (2,146,689,000 voxels, just under the 2^31 limit the header
    states) seen by 4 views: the first and last voxels, the ends of rows and
    planes, and random voxels inside and around the body, each within 1e-5 of
    one of the posteriors the per-voxel oracle admits; occupancy consistent; the
    block tile gives the same bits at those voxels."""
    say("forward at 1290^3 voxels x 4 views (sampled)")
    f, W, H = S.IMAGE_CLASSES[0]
    cams = S.ring_rig(4, f, W, H)
    grid = S.cube_grid(1290, 2.0)
    V = grid.nvox
    assert V < 2 ** 31
    rng = np.random.default_rng(77)
    body = S.make_body(rng)
    fr = S.render_frame(13, 0, cams, grid, body, (13, 0))
    ims, mus, vs = upload(fr)
    plan = plan_for(fr, mus, vs)
    post, occ = plan.reconstruct(ims)
    torch.cuda.synchronize()
    nx, ny = grid.nx, grid.ny
    ends = [0, 1, nx - 1, nx, nx * ny - 1, nx * ny, V // 2, V - nx * ny, V - nx, V - 2, V - 1]
    h, o = float(grid.voxel), float(grid.origin[0])
    c = body[0].centre
    near = [((int((c[2] - o) / h) + dk) * ny + int((c[1] - o) / h) + dj) * nx + int((c[0] - o) / h) + di
            for di, dj, dk in rng.integers(-20, 21, (300, 3))]
    idx = np.array(ends + near + list(rng.integers(0, V, 300)), np.int64)
    t = torch.from_numpy(idx).cuda()
    gp = post.view(-1)[t].cpu().numpy().astype(np.float64)
    go = occ.view(-1)[t].cpu().numpy()
    # the block tile (16 x 16 x 8 blocks staged in LDS) over the same index range: same bits
    block = [k for k, shape in enumerate(psfs.tiles()) if shape == (16, 16, 8)][0]
    plan.set_tile(block)
    plan.reconstruct(ims, post, occ)
    torch.cuda.synchronize()
    assert np.array_equal(post.view(-1)[t].cpu().numpy().astype(np.float64), gp)
    assert np.array_equal(occ.view(-1)[t].cpu().numpy(), go)
    del post, occ
    torch.cuda.empty_cache()
    maps = [O.slm(i, m, v) for i, m, v in zip(fr.images, fr.mean, fr.var)]
    occupied = 0
    for v, p, oc in zip(idx, gp, go):
        combos = O.voxel_combos(cams, grid, maps, int(v))
        assert len(combos) > 0
        assert np.min(np.abs(combos - p)) <= 1e-5, f"voxel {v}: {p} vs {combos[:4]}"
        assert oc == (1 if p > 0.5 else 0)
        occupied += int(oc)
    assert occupied > 20
    say(f"  {len(idx)} voxels checked, {occupied} occupied")


def test_ragged_grid_odd_images_mixed_sizes():
    say("ragged grid 37x29x23, odd image sizes")
    rng = np.random.default_rng(5)
    cams = [S.look_at_camera((4 * np.cos(t), 4 * np.sin(t), 1.2), f, W, H)
            for t, (f, W, H) in zip((0.3, 1.9, 3.7, 5.1), ((300, 321, 241), (250, 160, 117), (400, 401, 303), (90, 97, 61)))]
    grid = S.Grid(37, 29, 23, np.array([-0.9, -0.8, -1.05], np.float32), np.float32(0.047))
    body = S.make_body(rng)
    fr = S.render_frame(10, 0, cams, grid, body, (10, 0))
    plan, lmap, post, occ = run_forward(fr, prior=0.35, threshold=0.6)
    check_lmaps(plan, lmap, fr)
    ref, combos = oracle_forward(fr, prior=0.35)
    assert_posterior_parity(post, ref, combos=combos)
    assert_occupancy_parity(occ, ref, tau=0.6)


@pytest.mark.parametrize("n", [1, 16])
def test_view_count_extremes(n):
    say(f"view count {n}")
    f, W, H = S.IMAGE_CLASSES[0]
    cams = S.ring_rig(n, f, W, H, phase=0.1)
    grid = S.cube_grid(40, 2.0)
    body = S.make_body(np.random.default_rng(n))
    fr = S.render_frame(11, n, cams, grid, body, (11, n))
    plan, lmap, post, occ = run_forward(fr)
    ref, combos = oracle_forward(fr)
    assert_posterior_parity(post, ref, combos=combos)
    assert_occupancy_parity(occ, ref)


def test_zero_views_gives_prior_and_empty_grid_is_noop():
    grid = S.cube_grid(17, 2.0)
    plan = psfs.Plan([], grid, prior=0.3, threshold=0.25)
    post, occ = plan.reconstruct([])
    torch.cuda.synchronize()
    assert float((post - 0.3).abs().max()) < 1e-6
    assert bool(torch.all(occ == 1))
    empty = S.Grid(0, 5, 5, np.zeros(3, np.float32), np.float32(0.1))
    plan = psfs.Plan([], empty)
    post, occ = plan.reconstruct([])
    torch.cuda.synchronize()
    assert post.numel() == 0


def test_camera_inside_grid_voxels_behind():
    say("camera inside the grid")
    cam = S.look_at_camera((0.05, 0.02, 0.01), f=150.0, W=160, H=120, target=(3.0, 0.3, 0.2))
    grid = S.cube_grid(48, 2.0)
    body = S.make_body(np.random.default_rng(3), shift=(0.6, 0.0, 0.0))
    fr = S.render_frame(12, 0, [cam] + S.ring_rig(3, 300, 320, 240), grid, body, (12, 0))
    plan, lmap, post, occ = run_forward(fr)
    ref, combos = oracle_forward(fr)
    assert_posterior_parity(post, ref, combos=combos)
    assert_occupancy_parity(occ, ref)


def test_every_tile_gives_identical_bits():
    fr = S.config_frame(1, 0)
    ims, mus, vs = upload(fr)
    plan = plan_for(fr, mus, vs)
    lmap = plan.likelihood(ims)
    outs = []
    for t in range(len(psfs.tiles())):
        plan.set_tile(t)
        post, occ = plan.fuse(lmap)
        outs.append((post, occ))
    torch.cuda.synchronize()
    for post, occ in outs[1:]:
        assert torch.equal(post, outs[0][0]) and torch.equal(occ, outs[0][1])


def test_block_tile_views_that_cannot_be_staged():
    """The block tile's LDS-staged fusion beside views it must gather directly
    or skip: a camera inside the grid (block corners behind it), a close
    camera with a long focal length (boxes larger than the staging arena) and
    a camera looking past the grid (boxes that miss the image), on a grid
    that is ragged for the 16 x 16 x 8 blocks. Bit-identical to the column
    tiles, and within the oracle's bounds."""
    say("block tile: cameras inside, close to and looking past the grid")
    cams = [S.look_at_camera((0.05, -0.1, 0.02), 300.0, 200, 150, target=(1.0, 0.3, 0.1)),
            S.look_at_camera((1.4, 0.2, 0.3), 700.0, 640, 480),
            S.look_at_camera((-4.0, 0.5, 1.5), 150.0, 320, 240, target=(-1.0, 3.5, 1.0)),
            S.look_at_camera((3.5, -2.0, 1.0), 150.0, 320, 240)]
    grid = S.Grid(50, 41, 27, np.array([-1.0, -0.82, -0.54], np.float32), np.float32(0.04))
    body = S.make_body(np.random.default_rng(44))
    fr = S.render_frame(15, 0, cams, grid, body, (15, 0))
    ims, mus, vs = upload(fr)
    plan = plan_for(fr, mus, vs)
    lmap = plan.likelihood(ims)
    block = [t for t, (tx, ty, kz) in enumerate(psfs.tiles()) if (tx, ty, kz) == (16, 16, 8)]
    assert block, "no 16 x 16 x 8 tile"
    plan.set_tile(0)
    p0, o0 = plan.fuse(lmap)
    plan.set_tile(block[0])
    p1, o1 = plan.fuse(lmap)
    p2, o2 = plan.reconstruct(ims)
    # the pipelined form: maps of the frame, then its fusion beside the maps again
    m0, m1 = plan.new_lmap(), plan.new_lmap()
    plan.pipeline_step(ims, m0)
    p3, o3 = torch.full_like(p0, -1.0), torch.full_like(o0, 7)
    plan.pipeline_step(ims, m1, m0, p3, o3)
    torch.cuda.synchronize()
    assert torch.equal(p0, p1) and torch.equal(o0, o1)
    assert torch.equal(p0, p2) and torch.equal(o0, o2)
    assert torch.equal(p0, p3) and torch.equal(o0, o3)
    for k in range(len(cams)):        # each view's map (the padding between views is not written)
        assert torch.equal(plan.lmap_view(m0, k), plan.lmap_view(lmap, k))
        assert torch.equal(plan.lmap_view(m1, k), plan.lmap_view(lmap, k))
    ref, combos = oracle_forward(fr)
    assert_posterior_parity(p1, ref, combos=combos)
    assert_occupancy_parity(o1, ref)


def test_bilinear_every_tile_gives_identical_bits():
    fr = S.config_frame(0, 1)
    ims, mus, vs = upload(fr)
    plan = plan_for(fr, mus, vs, sampling=psfs.BILINEAR)
    lmap = plan.likelihood(ims)
    outs = []
    for t in range(len(psfs.tiles())):
        plan.set_tile(t)
        outs.append(plan.fuse(lmap))
    torch.cuda.synchronize()
    for t, (post, occ) in enumerate(outs[1:], 1):
        assert torch.equal(post, outs[0][0]) and torch.equal(occ, outs[0][1]), f"tile {t}"


def test_bilinear_posterior_parity():
    say("bilinear posterior")
    fr = S.config_frame(0, 2)
    ims, mus, vs = upload(fr)
    plan = plan_for(fr, mus, vs, sampling=psfs.BILINEAR)
    post, occ = plan.reconstruct(ims)
    torch.cuda.synchronize()
    l2s = [O.log2slm(i, m, v) for i, m, v in zip(fr.images, fr.mean, fr.var)]
    L = O.bilinear_logits(fr.cams, fr.grid, l2s)
    want = 1.0 / (1.0 + np.exp(-L))
    err = np.abs(post.cpu().numpy().astype(np.float64) - want)
    assert err.max() <= 1e-5, err.max()
    decided = np.abs(want - 0.5) > 1e-4
    assert np.array_equal(occ.cpu().numpy()[decided], (want > 0.5).astype(np.uint8)[decided])


def test_all_background_views_give_empty_grid():
    fr = S.config_frame(0, 4)
    rng = np.random.default_rng(8)
    fr.images = [rng.integers(0, 256, (c.height, c.width, 3)).astype(np.uint8) for c in fr.cams]
    fr.mean = [im.astype(np.float32) for im in fr.images]
    plan, lmap, post, occ = run_forward(fr)
    assert int(occ.sum()) == 0
    assert float(post.max()) <= 0.5


def test_threshold_entry_point():
    torch.manual_seed(0)
    post = torch.rand(1000003, device="cuda")
    post[:5] = torch.tensor([0.0, 0.25, 0.5, 0.75, 1.0], device="cuda")
    for tau in (0.0, 0.25, 0.5, 1.0):
        occ = psfs.threshold(post, tau)
        torch.cuda.synchronize()
        assert torch.equal(occ, (post > tau).to(torch.uint8))
