"""GPU learned foreground model (after the first frame) against the FP64
oracle (oracle/foreground.py): the histogram density learned from a frame's
foreground pixels, then the next frame's likelihood maps and posterior with
that density in place of the uniform one."""
import sys

import numpy as np
import pytest
import torch

import paper_1311_6811_amd as psfs
from oracle import foreground as FG
from oracle import oracle as O
from synth import scene as S
from tests.gpu_util import assert_occupancy_parity, assert_posterior_parity, plan_for, upload

pytestmark = pytest.mark.gpu

LMAP_RTOL, LMAP_ATOL = 2e-6, 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def two_frames(cfg):
    """Two frames from one rig and one background model, the body moved."""
    base = S.config_frame(cfg, 0)
    rng = np.random.default_rng(40 + cfg)
    body0 = S.make_body(rng)
    body1 = S.make_body(rng, shift=(0.04, 0.02, 0.0))
    f0 = S.render_frame(50 + cfg, 0, base.cams, base.grid, body0, (50 + cfg, 0))
    f1 = S.render_frame(50 + cfg, 1, base.cams, base.grid, body1, (50 + cfg, 0))
    return f0, f1


@pytest.mark.parametrize("cfg", [0, 1, 2])
def test_learned_model_density_maps_and_posterior(cfg):
    say(f"foreground model, rig of config {cfg}")
    f0, f1 = two_frames(cfg)
    ims0, mus, vs = upload(f0)
    ims1 = upload(f1)[0]
    plan = plan_for(f0, mus, vs)
    # training pixels of frame 0: SLM > 1/2 by the oracle, given to both sides
    l0 = [O.log2slm(i, m, v) for i, m, v in zip(f0.images, f0.mean, f0.var)]
    masks = [(l > 0).astype(np.uint8) for l in l0]
    want_logd = FG.log_density(FG.histogram(f0.images, masks))
    logd = plan.foreground_model(ims0, masks=[torch.from_numpy(m).cuda() for m in masks])
    torch.cuda.synchronize()
    got = logd.cpu().numpy().astype(np.float64)
    assert np.abs(got - want_logd).max() <= 2e-6 * np.abs(want_logd).max()
    # frame 1 with the learned density
    plan.set_foreground(logd)
    lmap = plan.likelihood(ims1)
    post, occ = plan.fuse(lmap)
    torch.cuda.synchronize()
    l1 = [FG.log2slm(i, m, v, want_logd) for i, m, v in zip(f1.images, f1.mean, f1.var)]
    for k in range(f1.n):
        g = plan.lmap_view(lmap, k).cpu().numpy().astype(np.float64)
        err = np.abs(g - l1[k]) - LMAP_RTOL * np.abs(l1[k])
        assert err.max() <= LMAP_ATOL, f"view {k}: {err.max():.3e}"
    maps = [FG.slm(i, m, v, want_logd) for i, m, v in zip(f1.images, f1.mean, f1.var)]
    ref = O.posterior(f1.cams, f1.grid, maps)
    worst = assert_posterior_parity(post, ref, combos=lambda v: O.voxel_combos(f1.cams, f1.grid, maps, v))
    assert_occupancy_parity(occ, ref)
    say(f"  max posterior error {worst:.2e}")


def test_masks_from_maps_and_uniform_restore():
    f0, f1 = two_frames(0)
    ims0, mus, vs = upload(f0)
    ims1 = upload(f1)[0]
    plan = plan_for(f0, mus, vs)
    lmap0 = plan.likelihood(ims0)
    a = plan.foreground_model(ims0, lmap=lmap0)
    masks = [(plan.lmap_view(lmap0, k) > 0).to(torch.uint8).contiguous() for k in range(plan.n)]
    b = plan.foreground_model(ims0, masks=masks)
    mixed = plan.foreground_model(ims0, masks=[masks[0]] + [None] * (plan.n - 1), lmap=lmap0)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(a, mixed)
    plain = plan.likelihood(ims1).clone()
    plan.set_foreground(a)
    learned = plan.likelihood(ims1).clone()
    pipe_maps = plan.new_lmap()
    plan.pipeline_step(ims1, pipe_maps)                        # the pipelined step uses the model too
    plan.set_foreground(None)
    again = plan.likelihood(ims1)
    torch.cuda.synchronize()
    n = plan.lmap_floats()
    assert torch.equal(plain[:n], again[:n]) and not torch.equal(plain[:n], learned[:n])
    assert torch.equal(pipe_maps[:n], learned[:n])
