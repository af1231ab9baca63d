"""Four frames of one rig per launch (psfs_pipeline_step_quad): the quad maps
interleave the four frames' likelihood maps, and every frame's maps, posterior
and occupancy must be bit-identical to computing that frame alone; one frame
of the ragged sequence is also checked against the FP64 oracle."""
import sys

import numpy as np
import pytest
import torch

from oracle import oracle as O
from synth import scene as S
from tests.gpu_util import assert_occupancy_parity, assert_posterior_parity, plan_for, upload

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def sequence(frames, **kw):
    ims0, mus, vs = upload(frames[0])
    plan = plan_for(frames[0], mus, vs, **kw)
    return plan, [ims0] + [upload(fr)[0] for fr in frames[1:]]


def outputs(plan, k=4):
    g = plan.grid
    shape = (g.nz, g.ny, g.nx)
    posts = [torch.full(shape, -1.0, dtype=torch.float32, device="cuda") for _ in range(k)]
    occs = [torch.full(shape, 7, dtype=torch.uint8, device="cuda") for _ in range(k)]
    return posts, occs


def run_quads(plan, images):
    """A sequence of a multiple of four frames, four per launch (maps of group
    k beside the fusion of group k - 1); returns every frame's (posterior,
    occupancy)."""
    maps = [plan.new_lmap_quad(), plan.new_lmap_quad()]
    outs = []
    ngroups = len(images) // 4
    for k in range(ngroups + 1):
        nxt = images[4 * k:4 * k + 4] if k < ngroups else None
        if k > 0:
            posts, occs = outputs(plan)
            plan.pipeline_step_quad(nxt, maps[k % 2] if nxt is not None else None, maps[(k - 1) % 2], posts, occs)
            outs += list(zip(posts, occs))
        else:
            plan.pipeline_step_quad(nxt, maps[0])
    torch.cuda.synchronize()
    return outs


def assert_frames_match(plan, images, outs):
    assert len(outs) == len(images)
    for k, (ims, (post, occ)) in enumerate(zip(images, outs)):
        p1, o1 = plan.reconstruct(ims)
        torch.cuda.synchronize()
        assert torch.equal(p1, post), f"frame {k}: posterior differs"
        assert torch.equal(o1, occ), f"frame {k}: occupancy differs"


def test_quad_maps_and_fusion_equal_single_frames():
    say("four-frame step, 128^3 x 8 views")
    frames = [S.config_frame(1, f) for f in range(4)]
    plan, images = sequence(frames)
    lm4 = plan.new_lmap_quad()
    plan.pipeline_step_quad(images, lm4)
    singles = [plan.likelihood(ims) for ims in images]
    torch.cuda.synchronize()
    assert torch.equal(lm4, torch.stack(singles, dim=1).reshape(-1))
    posts, occs = outputs(plan)
    plan.pipeline_step_quad(None, None, lm4, posts, occs)
    refs = [plan.fuse(m) for m in singles]
    torch.cuda.synchronize()
    for f in range(4):
        assert torch.equal(posts[f], refs[f][0]), f"frame {f}: posterior"
        assert torch.equal(occs[f], refs[f][1]), f"frame {f}: occupancy"
    # without occupancy outputs, and with only some of them
    q, _ = outputs(plan)
    plan.pipeline_step_quad(None, None, lm4, q, None)
    q2, o2 = outputs(plan)
    plan.pipeline_step_quad(None, None, lm4, q2, [None, o2[1], None, o2[3]])
    torch.cuda.synchronize()
    for f in range(4):
        assert torch.equal(q[f], posts[f]) and torch.equal(q2[f], posts[f])
    assert torch.equal(o2[1], occs[1]) and torch.equal(o2[3], occs[3])
    assert bool((o2[0] == 7).all()) and bool((o2[2] == 7).all())      # untouched


def test_quad_sequence_bitwise_equals_single_frames():
    say("four-frame sequence, 8 frames, 64^3 x 4 views")
    frames = [S.config_frame(0, f) for f in range(8)]
    plan, images = sequence(frames)
    outs = run_quads(plan, images)
    assert_frames_match(plan, images, outs)


def test_quad_ragged_sequence_foreground_and_oracle():
    """Ragged grid and odd image sizes (tail waves of the likelihood, partial
    tiles of the fusion), one frame against the FP64 oracle, then the same
    sequence with a learned foreground model."""
    say("four-frame sequence, ragged grid, odd image sizes, oracle, foreground model")
    rng = np.random.default_rng(41)
    cams = [S.look_at_camera((4 * np.cos(t), 4 * np.sin(t), 1.2), f, W, H)
            for t, (f, W, H) in zip((0.3, 1.9, 3.7), ((300, 321, 241), (250, 163, 117), (90, 97, 61)))]
    grid = S.Grid(37, 29, 23, np.array([-0.9, -0.8, -1.05], np.float32), np.float32(0.047))
    frames = [S.render_frame(13, f, cams, grid, S.make_body(rng), (13, 0)) for f in range(4)]
    plan, images = sequence(frames, prior=0.4, threshold=0.55)
    outs = run_quads(plan, images)
    assert_frames_match(plan, images, outs)
    fr = frames[3]
    maps = [O.slm(i, m, v) for i, m, v in zip(fr.images, fr.mean, fr.var)]
    ref = O.posterior(fr.cams, fr.grid, maps, 0.4)
    assert_posterior_parity(outs[3][0], ref, combos=lambda v: O.voxel_combos(fr.cams, fr.grid, maps, v, 0.4))
    assert_occupancy_parity(outs[3][1], ref, tau=0.55)
    logd = plan.foreground_model(images[0], lmap=plan.likelihood(images[0]))
    plan.set_foreground(logd)
    outs = run_quads(plan, images)
    assert_frames_match(plan, images, outs)
    plan.set_foreground(None)


def test_quad_grid_with_whole_and_partial_32_column_waves():
    """A grid whose rows are a multiple of 16 voxels but not of 32, with
    ragged y and z edges: waves that lie inside the grid store their outputs
    as regrouped row pieces, the others voxel by voxel, in the same launch;
    every frame bit-identical to the frame alone."""
    say("four-frame sequence, 48 x 41 x 22 grid")
    rng = np.random.default_rng(45)
    cams = S.ring_rig(4, 300.0, 320, 240)
    grid = S.Grid(48, 41, 22, np.array([-0.96, -0.82, -0.44], np.float32), np.float32(0.04))
    frames = [S.render_frame(16, f, cams, grid, S.make_body(rng), (16, 0)) for f in range(8)]
    plan, images = sequence(frames)
    outs = run_quads(plan, images)
    assert_frames_match(plan, images, outs)


def test_quad_cameras_inside_and_close_to_the_grid():
    """Views whose pixel box cannot be staged: a camera inside the grid (block
    corners behind it), a close camera with a long focal length (boxes larger
    than the staging buffer) and a camera looking past the grid (boxes that
    miss the image), beside an ordinary view, on a grid that is ragged for
    every block shape: every frame bit-identical to the frame alone."""
    say("four-frame sequence, cameras inside, close to and looking past the grid")
    rng = np.random.default_rng(43)
    cams = [S.look_at_camera((0.05, -0.1, 0.02), 300.0, 200, 150, target=(1.0, 0.3, 0.1)),
            S.look_at_camera((1.4, 0.2, 0.3), 700.0, 640, 480),
            S.look_at_camera((-4.0, 0.5, 1.5), 150.0, 320, 240, target=(-1.0, 3.5, 1.0)),
            S.look_at_camera((3.5, -2.0, 1.0), 150.0, 320, 240)]
    grid = S.Grid(50, 41, 27, np.array([-1.0, -0.82, -0.54], np.float32), np.float32(0.04))
    frames = [S.render_frame(14, f, cams, grid, S.make_body(rng), (14, 0)) for f in range(4)]
    plan, images = sequence(frames)
    outs = run_quads(plan, images)
    assert_frames_match(plan, images, outs)


def test_quad_zero_views_give_the_prior():
    say("four-frame step, no views")
    fr = S.config_frame(0, 0)
    plan, _ = sequence([fr])
    plan.set_cameras([])
    posts, _ = outputs(plan)
    plan.pipeline_step_quad([[], [], [], []], plan.new_lmap_quad(), plan.new_lmap_quad(), posts, None)
    torch.cuda.synchronize()
    prior = torch.full_like(posts[0], 0.5)
    for p in posts:
        assert torch.allclose(p, prior)


def test_quad_largest_workload():
    """The 12-view 1280x720 rig over a 256^3 grid, four frames in one group:
    every frame bit-identical to the frame alone."""
    say("four-frame step, 256^3 x 12 views of 1280x720")
    frames = [S.config_frame(2, f) for f in range(4)]
    plan, images = sequence(frames)
    outs = run_quads(plan, images)
    assert_frames_match(plan, images, outs)


def test_quad_whole_256cube_sequence_and_oracle():
    """The whole 16-frame sequence of the 256^3-voxel, 12-view, 1280x720
    workload (one rig and background model, the body moving 2 cm per frame)
    as four quad groups through five launches: every frame bit-identical to
    that frame reconstructed alone, and the last frame against the FP64
    oracle (unambiguous voxels within 1e-5, ambiguous ones within their
    admissible range, decided occupancy exact)."""
    from concurrent.futures import ThreadPoolExecutor
    say("four-frame steps, whole 16-frame sequence at 256^3 x 12 views of 1280x720")
    with ThreadPoolExecutor(8) as ex:
        frames = list(ex.map(lambda t: S.config_frame(2, t), range(16)))
    last = frames[15]
    for fr in frames[1:15]:
        fr.mean, fr.var = None, None                  # one background model for the rig: frame 0's
    ims0, mus, vs = upload(frames[0])
    plan = plan_for(frames[0], mus, vs)
    images = [ims0] + [[torch.from_numpy(i).cuda() for i in fr.images] for fr in frames[1:]]
    outs = run_quads(plan, images)
    assert_frames_match(plan, images, outs)
    say("  frames bit-identical; oracle on frame 15")
    maps = [O.slm(i, m, v) for i, m, v in zip(last.images, last.mean, last.var)]
    ref = O.posterior(last.cams, last.grid, maps)
    assert_posterior_parity(outs[15][0], ref, combos=lambda v: O.voxel_combos(last.cams, last.grid, maps, v),
                            n_enum=100)
    assert_occupancy_parity(outs[15][1], ref)
