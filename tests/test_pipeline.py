"""Pipelined frame sequence: one launch per frame computes the next frame's
likelihood maps beside the current frame's fusion.

Each frame's posterior and occupancy must be bit-identical to reconstructing
that frame alone (same per-pixel and per-column code), and one frame of a
ragged sequence is also checked against the FP64 oracle.
"""
import sys

import numpy as np
import pytest
import torch

import paper_1311_6811_amd as psfs
from oracle import oracle as O
from synth import scene as S
from tests.gpu_util import assert_occupancy_parity, assert_posterior_parity, plan_for, upload

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def sequence(frames, **kw):
    """Plan over the first frame's rig and background; every frame's images."""
    ims0, mus, vs = upload(frames[0])
    plan = plan_for(frames[0], mus, vs, **kw)
    images = [ims0] + [upload(fr)[0] for fr in frames[1:]]
    return plan, images


def run_pipeline(plan, images):
    pipe = psfs.Pipeline(plan)
    outs = []
    for ims in images:
        o = pipe.push(ims)
        if o is not None:
            outs.append(o)
    outs.append(pipe.flush())
    torch.cuda.synchronize()
    return outs


def assert_matches_single(plan, images, outs):
    assert len(outs) == len(images)
    for k, (ims, (post, occ)) in enumerate(zip(images, outs)):
        p1, o1 = plan.reconstruct(ims)
        torch.cuda.synchronize()
        assert torch.equal(p1, post), f"frame {k}: posterior differs"
        assert torch.equal(o1, occ), f"frame {k}: occupancy differs"


def test_sequence_bitwise_equals_single_frames():
    say("pipelined 128^3 x 8 views, 4 frames")
    frames = [S.config_frame(1, f) for f in range(4)]
    plan, images = sequence(frames)
    outs = run_pipeline(plan, images)
    assert_matches_single(plan, images, outs)


def test_largest_workload_sequence():
    """The 12-view 1280x720 rig over a 256^3 grid, 3 frames moving 2 cm per
    frame: every pipelined frame bit-identical to the frame alone, the last
    one within the posterior tolerance of the FP64 oracle."""
    say("pipelined 256^3 x 12 views, 3 frames")
    frames = [S.config_frame(2, f) for f in range(3)]
    plan, images = sequence(frames)
    outs = run_pipeline(plan, images)
    assert_matches_single(plan, images, outs)
    fr = frames[-1]
    maps = [O.slm(i, m, v) for i, m, v in zip(fr.images, fr.mean, fr.var)]
    ref = O.posterior(fr.cams, fr.grid, maps)
    post, occ = outs[-1]
    worst = assert_posterior_parity(post, ref, combos=lambda v: O.voxel_combos(fr.cams, fr.grid, maps, v))
    assert_occupancy_parity(occ, ref)
    say(f"  max posterior error {worst:.2e}")


def test_ragged_sequence_and_oracle_parity():
    say("pipelined ragged grid, odd image sizes")
    rng = np.random.default_rng(21)
    cams = [S.look_at_camera((4 * np.cos(t), 4 * np.sin(t), 1.2), f, W, H)
            for t, (f, W, H) in zip((0.3, 1.9, 3.7), ((300, 321, 241), (250, 163, 117), (90, 97, 61)))]
    grid = S.Grid(37, 29, 23, np.array([-0.9, -0.8, -1.05], np.float32), np.float32(0.047))
    # one rig and one background model (same background key), a new body per frame
    frames = [S.render_frame(13, f, cams, grid, S.make_body(rng), (13, 0)) for f in range(3)]
    plan, images = sequence(frames, prior=0.4, threshold=0.55)
    outs = run_pipeline(plan, images)
    assert_matches_single(plan, images, outs)
    fr = frames[2]
    maps = [O.slm(i, m, v) for i, m, v in zip(fr.images, fr.mean, fr.var)]
    ref = O.posterior(fr.cams, fr.grid, maps, 0.4)
    assert_posterior_parity(outs[2][0], ref, combos=lambda v: O.voxel_combos(fr.cams, fr.grid, maps, v, 0.4))
    assert_occupancy_parity(outs[2][1], ref, tau=0.55)


def test_bilinear_sequence():
    frames = [S.config_frame(0, f) for f in range(3)]
    plan, images = sequence(frames, sampling=psfs.BILINEAR)
    outs = run_pipeline(plan, images)
    assert_matches_single(plan, images, outs)


def test_one_sided_steps_equal_likelihood_and_fuse():
    fr = S.config_frame(0, 1)
    ims, mus, vs = upload(fr)
    plan = plan_for(fr, mus, vs)
    a = plan.new_lmap()
    plan.pipeline_step(ims, a)                                 # likelihood only
    post = torch.empty((fr.grid.nz, fr.grid.ny, fr.grid.nx), dtype=torch.float32, device="cuda")
    occ = torch.empty_like(post, dtype=torch.uint8)
    plan.pipeline_step(None, None, a, post, occ)               # fusion only
    lmap = plan.likelihood(ims)
    p1, o1 = plan.fuse(lmap)
    torch.cuda.synchronize()
    assert torch.equal(a[:plan.lmap_floats()], lmap[:plan.lmap_floats()])
    assert torch.equal(post, p1) and torch.equal(occ, o1)


def test_every_tile_gives_identical_bits():
    frames = [S.config_frame(1, f) for f in range(2)]
    plan, images = sequence(frames)
    ref = None
    for t in range(len(psfs.tiles())):
        plan.set_tile(t)
        outs = run_pipeline(plan, images)
        if ref is None:
            ref = outs
            continue
        for (p0, o0), (p1, o1) in zip(ref, outs):
            assert torch.equal(p0, p1) and torch.equal(o0, o1), f"tile {t}"


def test_zero_views_and_empty_grid():
    grid = S.cube_grid(17, 2.0)
    plan = psfs.Plan([], grid, prior=0.3, threshold=0.25)
    outs = run_pipeline(plan, [[], []])
    for post, occ in outs:
        assert float((post - 0.3).abs().max()) < 1e-6 and bool(torch.all(occ == 1))
    fr = S.config_frame(0, 0)
    ims, mus, vs = upload(fr)
    empty = S.Grid(0, 5, 5, np.zeros(3, np.float32), np.float32(0.1))
    plan = psfs.Plan(fr.cams, empty)
    plan.set_backgrounds(mus, vs)
    outs = run_pipeline(plan, [ims, ims])
    assert all(p.numel() == 0 for p, _ in outs)


def test_largest_grid_sequence_bitwise():
    """Two frames over a 1290^3 grid (just under the 2^31-voxel limit) seen by
    4 views: the pipelined frames are bit-identical to the frames alone."""
    say("pipelined 1290^3 x 4 views, 2 frames")
    f, W, H = S.IMAGE_CLASSES[0]
    cams = S.ring_rig(4, f, W, H)
    grid = S.cube_grid(1290, 2.0)
    rng = np.random.default_rng(91)
    frames = [S.render_frame(14, k, cams, grid, S.make_body(rng, shift=(0.03 * k, 0.0, 0.0)), (14, 0)) for k in range(2)]
    plan, images = sequence(frames)
    outs = run_pipeline(plan, images)
    assert_matches_single(plan, images, outs)
