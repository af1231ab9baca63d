"""Two frames of one rig per launch (psfs_pipeline_step_pair): the pair maps
interleave the two frames' likelihood maps, and every frame's maps, posterior
and occupancy must be bit-identical to computing that frame alone."""
import sys

import numpy as np
import pytest
import torch

from synth import scene as S
from tests.gpu_util import plan_for, upload

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def sequence(frames, **kw):
    ims0, mus, vs = upload(frames[0])
    plan = plan_for(frames[0], mus, vs, **kw)
    return plan, [ims0] + [upload(fr)[0] for fr in frames[1:]]


def interleave(a, b):
    return torch.stack([a, b], dim=1).reshape(-1)


def run_pairs(plan, images):
    """A sequence of an even number of frames, two per launch (maps of pair k
    beside the fusion of pair k - 1); returns every frame's (posterior,
    occupancy)."""
    g = plan.grid
    shape = (g.nz, g.ny, g.nx)
    maps = [plan.new_lmap_pair(), plan.new_lmap_pair()]
    outs = []
    npairs = len(images) // 2
    for k in range(npairs + 1):
        nxt = (images[2 * k], images[2 * k + 1]) if k < npairs else (None, None)
        if k > 0:
            post = [torch.empty(shape, dtype=torch.float32, device="cuda") for _ in range(2)]
            occ = [torch.empty(shape, dtype=torch.uint8, device="cuda") for _ in range(2)]
            plan.pipeline_step_pair(nxt[0], nxt[1], maps[k % 2] if nxt[0] is not None else None, maps[(k - 1) % 2],
                                    post[0], occ[0], post[1], occ[1])
            outs += [(post[0], occ[0]), (post[1], occ[1])]
        else:
            plan.pipeline_step_pair(nxt[0], nxt[1], maps[0])
    torch.cuda.synchronize()
    return outs


def assert_frames_match(plan, images, outs):
    assert len(outs) == len(images)
    for k, (ims, (post, occ)) in enumerate(zip(images, outs)):
        p1, o1 = plan.reconstruct(ims)
        torch.cuda.synchronize()
        assert torch.equal(p1, post), f"frame {k}: posterior differs"
        assert torch.equal(o1, occ), f"frame {k}: occupancy differs"


def test_pair_maps_and_fusion_equal_single_frames():
    say("two-frame step, 128^3 x 8 views")
    frames = [S.config_frame(1, f) for f in range(2)]
    plan, images = sequence(frames)
    lm2 = plan.new_lmap_pair()
    plan.pipeline_step_pair(images[0], images[1], lm2)
    la, lb = plan.likelihood(images[0]), plan.likelihood(images[1])
    torch.cuda.synchronize()
    assert torch.equal(lm2, interleave(la, lb))
    shape = (plan.grid.nz, plan.grid.ny, plan.grid.nx)
    pa, pb = torch.empty(shape, device="cuda"), torch.empty(shape, device="cuda")
    oa, ob = (torch.empty(shape, dtype=torch.uint8, device="cuda") for _ in range(2))
    plan.pipeline_step_pair(None, None, None, lm2, pa, oa, pb, ob)
    ra, rb = plan.fuse(la), plan.fuse(lb)
    torch.cuda.synchronize()
    assert torch.equal(pa, ra[0]) and torch.equal(oa, ra[1])
    assert torch.equal(pb, rb[0]) and torch.equal(ob, rb[1])
    # without occupancy outputs
    qa, qb = torch.empty_like(pa), torch.empty_like(pb)
    plan.pipeline_step_pair(None, None, None, lm2, qa, None, qb, None)
    torch.cuda.synchronize()
    assert torch.equal(qa, pa) and torch.equal(qb, pb)


def test_pair_sequence_bitwise_equals_single_frames():
    say("two-frame sequence, 6 frames, 64^3 x 4 views")
    frames = [S.config_frame(0, f) for f in range(6)]
    plan, images = sequence(frames)
    outs = run_pairs(plan, images)
    assert_frames_match(plan, images, outs)


def test_pair_ragged_sequence_and_foreground():
    """Ragged grid and odd image sizes (tail waves of the likelihood), then the
    same with a learned foreground model."""
    say("two-frame sequence, ragged grid, odd image sizes, foreground model")
    rng = np.random.default_rng(31)
    cams = [S.look_at_camera((4 * np.cos(t), 4 * np.sin(t), 1.2), f, W, H)
            for t, (f, W, H) in zip((0.3, 1.9, 3.7), ((300, 321, 241), (250, 163, 117), (90, 97, 61)))]
    grid = S.Grid(37, 29, 23, np.array([-0.9, -0.8, -1.05], np.float32), np.float32(0.047))
    frames = [S.render_frame(13, f, cams, grid, S.make_body(rng), (13, 0)) for f in range(4)]
    plan, images = sequence(frames, prior=0.4, threshold=0.55)
    outs = run_pairs(plan, images)
    assert_frames_match(plan, images, outs)
    logd = plan.foreground_model(images[0], lmap=plan.likelihood(images[0]))
    plan.set_foreground(logd)
    outs = run_pairs(plan, images)
    assert_frames_match(plan, images, outs)
    plan.set_foreground(None)


def test_pair_grid_with_whole_and_partial_32_column_waves():
    """A grid whose rows are a multiple of 16 voxels but not of 32, with
    ragged y and z edges: waves that lie inside the grid store their outputs
    as regrouped row pieces, the others voxel by voxel, in the same launch;
    every frame bit-identical to the frame alone."""
    say("two-frame sequence, 48 x 41 x 22 grid")
    rng = np.random.default_rng(45)
    cams = S.ring_rig(4, 300.0, 320, 240)
    grid = S.Grid(48, 41, 22, np.array([-0.96, -0.82, -0.44], np.float32), np.float32(0.04))
    frames = [S.render_frame(16, f, cams, grid, S.make_body(rng), (16, 0)) for f in range(4)]
    plan, images = sequence(frames)
    outs = run_pairs(plan, images)
    assert_frames_match(plan, images, outs)


def test_zero_views_give_the_prior():
    say("two-frame step, no views")
    fr = S.config_frame(0, 0)
    plan, images = sequence([fr])
    plan.set_cameras([])
    shape = (plan.grid.nz, plan.grid.ny, plan.grid.nx)
    pa, pb = torch.empty(shape, device="cuda"), torch.empty(shape, device="cuda")
    plan.pipeline_step_pair([], [], plan.new_lmap_pair(), plan.new_lmap_pair(), pa, None, pb, None)
    torch.cuda.synchronize()
    prior = torch.full(shape, 0.5, device="cuda")
    assert torch.allclose(pa, prior) and torch.allclose(pb, prior)
