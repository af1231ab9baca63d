"""Optional device check of the background model (PSFS_E_INPUT): Eq. 1 is
defined only for positive finite variances and finite means. With the check
on, every likelihood pass of a plan flags the views whose model holds an
invalid value; the values written are then meaningless, but nothing faults.
The bad values are planted in the inputs on the host (NaN, infinities, zero
and negative variances) and the flags read back after a synchronisation."""
import sys

import numpy as np
import pytest
import torch

import paper_1311_6811_amd as psfs
from paper_1311_6811_amd import _lib as L
from synth import scene as S
from tests.gpu_util import plan_for, upload

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def ragged_frame():
    # odd image sizes: the likelihood's tail waves see the last pixels
    cams = [S.look_at_camera((4 * np.cos(t), 4 * np.sin(t), 1.2), f, W, H)
            for t, (f, W, H) in zip((0.3, 1.9, 3.7), ((300, 321, 241), (250, 163, 117), (90, 97, 61)))]
    grid = S.Grid(21, 17, 13, np.array([-0.9, -0.8, -1.05], np.float32), np.float32(0.08))
    return S.render_frame(13, 0, cams, grid, S.make_body(np.random.default_rng(5)), (13, 0))


def expect(plan, views):
    torch.cuda.synchronize()
    if not views:
        plan.input_status()
        return
    with pytest.raises(L.PsfsError) as e:
        plan.input_status()
    assert e.value.status == -8
    assert f"view(s) {', '.join(str(v) for v in views)} " in str(e.value)
    plan.input_status()                 # the flags were cleared


def test_valid_inputs_pass_and_check_off_by_default():
    say("input check: valid inputs")
    fr = S.config_frame(0, 0)
    ims, mus, vs = upload(fr)
    plan = plan_for(fr, mus, vs)
    with pytest.raises(L.PsfsError) as e:
        plan.input_status()             # no flags given
    assert e.value.status == -3
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    plan.set_input_check(flags)
    post, _ = plan.reconstruct(ims)
    expect(plan, [])
    assert bool(torch.isfinite(post).all())


@pytest.mark.parametrize("what,value", [("var", float("nan")), ("var", 0.0), ("var", -4.0), ("var", float("inf")),
                                        ("mean", float("nan")), ("mean", float("-inf"))])
def test_each_invalid_value_is_flagged(what, value):
    say(f"input check: {what} = {value}")
    fr = S.config_frame(0, 0)
    ims, mus, vs = upload(fr)
    t = (vs if what == "var" else mus)[2]
    t.view(-1)[3 * 1234 + 1] = value                 # pixel 1234 of view 2, green
    plan = plan_for(fr, mus, vs)
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    plan.set_input_check(flags)
    plan.reconstruct(ims)
    expect(plan, [2])
    plan.set_input_check(None)                       # off: nothing is recorded
    plan.reconstruct(ims)
    torch.cuda.synchronize()
    assert int(flags.item()) == 0


def test_every_checked_path_and_tail_pixels():
    """The likelihood, the one-, two- and four-frame steps and the
    differentiable forward each flag a bad value in the last pixel of a view
    whose pixel count is not a multiple of the wave's span, and a bad value
    in two views names both."""
    say("input check: every path, tail pixels")
    fr = ragged_frame()
    ims, mus, vs = upload(fr)
    vs[1].view(-1)[-1] = -1.0                         # last pixel of view 1 (163 x 117)
    mus[2].view(-1)[5] = float("nan")                 # an early pixel of view 2
    plan = plan_for(fr, mus, vs)
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    plan.set_input_check(flags)
    plan.likelihood(ims)
    expect(plan, [1, 2])
    plan.pipeline_step(ims, plan.new_lmap())
    expect(plan, [1, 2])
    plan.pipeline_step_pair(ims, ims, plan.new_lmap_pair())
    expect(plan, [1, 2])
    plan.pipeline_step_quad([ims] * 4, plan.new_lmap_quad())
    expect(plan, [1, 2])
    dplan = psfs.Plan(fr.cams, fr.grid, sampling=psfs.BILINEAR)
    dplan.set_backgrounds(mus, vs)
    dplan.set_input_check(flags)
    labels = torch.zeros((fr.grid.nz, fr.grid.ny, fr.grid.nx), dtype=torch.uint8, device="cuda")
    dplan.diff_forward(ims, labels)
    expect(dplan, [1, 2])
    vs[1].view(-1)[-1] = 30.0
    mus[2].view(-1)[5] = 100.0
    plan.pipeline_step_quad([ims] * 4, plan.new_lmap_quad())
    expect(plan, [])
