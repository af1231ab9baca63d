"""Stream semantics of the library: a plan keeps no device state of its own
(cameras, grid, parameters and buffer addresses travel in each launch's
arguments), so one plan can feed launches on several streams at once, and
changing its settings after a call does not change work already enqueued."""
import sys

import pytest
import torch

from synth import scene as S
from tests.gpu_util import plan_for, upload

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_one_plan_on_two_streams():
    say("one plan, two streams, 128^3 x 8 views")
    frames = [S.config_frame(1, f) for f in range(2)]
    up = [upload(fr) for fr in frames]
    plan = plan_for(frames[0], up[0][1], up[0][2])
    ims = [u[0] for u in up]
    ref = []
    for k in range(2):
        post, occ = plan.reconstruct(ims[k])
        torch.cuda.synchronize()
        ref.append((post.clone(), occ.clone()))
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    wss = [plan.new_workspace(), plan.new_workspace()]
    outs = []
    for rep in range(4):
        for k in range(2):
            with torch.cuda.stream(streams[k]):
                outs.append((k, plan.reconstruct(ims[k], workspace=wss[k])))
    torch.cuda.synchronize()
    for k, (post, occ) in outs:
        assert torch.equal(post, ref[k][0]) and torch.equal(occ, ref[k][1])


def test_settings_changed_after_a_call_leave_it_alone():
    say("settings changed after enqueueing, 128^3 x 8 views")
    fr = S.config_frame(1, 0)
    ims, mus, vs = upload(fr)
    plan = plan_for(fr, mus, vs)
    ref_a = plan.reconstruct(ims)
    plan.set_params(prior=0.3, threshold=0.8)
    ref_b = plan.reconstruct(ims)
    torch.cuda.synchronize()
    ref_a = [t.clone() for t in ref_a]
    ref_b = [t.clone() for t in ref_b]
    assert not torch.equal(ref_a[0], ref_b[0])
    plan.set_params()                                   # back to the defaults
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    with torch.cuda.stream(sa):
        got_a = plan.reconstruct(ims)
    plan.set_params(prior=0.3, threshold=0.8)           # while the first call may still run
    with torch.cuda.stream(sb):
        got_b = plan.reconstruct(ims)
    plan.set_params()
    torch.cuda.synchronize()
    assert torch.equal(got_a[0], ref_a[0]) and torch.equal(got_a[1], ref_a[1])
    assert torch.equal(got_b[0], ref_b[0]) and torch.equal(got_b[1], ref_b[1])
