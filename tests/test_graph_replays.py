"""Entry points captured into HIP graphs and replayed: every replay must give
the bits of the same calls made eagerly. Between replays the outputs are
overwritten and other eager work runs on the same workspaces, with
synchronisations, so a replay that leaned on state left by an earlier call (a
counter or buffer that a captured memset would have cleared only once) would
show up as a difference."""
import sys

import numpy as np
import pytest
import torch

import paper_1311_6811_amd as psfs
from synth import scene as S
from tests.gpu_util import plan_for, upload

pytestmark = pytest.mark.gpu

REPLAYS = 3


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def capture(fn, stream):
    """Runs fn once eagerly on `stream` (warm-up), then captures it."""
    with torch.cuda.stream(stream):
        fn()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            fn()
    torch.cuda.synchronize()
    return g


def scramble(tensors):
    for t in tensors:
        if t.dtype.is_floating_point:
            t.fill_(float("nan"))
        else:
            t.fill_(-7 if t.dtype != torch.uint8 else 7)


def same(a, b):
    return all(torch.equal(x, y) for x, y in zip(a, b))


def test_pipeline_step_and_reconstruct():
    say("graph replays: pipelined steps and reconstruct, 64^3 x 4 views")
    frames = [S.config_frame(0, f) for f in range(2)]
    up = [upload(fr) for fr in frames]
    plans = [plan_for(fr, mus, vs) for fr, (_, mus, vs) in zip(frames, up)]
    ims = [u[0] for u in up]
    shape = (frames[0].grid.nz, frames[0].grid.ny, frames[0].grid.nx)
    maps = [plans[0].new_lmap(), plans[0].new_lmap()]
    post = [torch.empty(shape, dtype=torch.float32, device="cuda") for _ in range(3)]
    occ = [torch.empty(shape, dtype=torch.uint8, device="cuda") for _ in range(3)]
    ws = plans[0].new_workspace()

    def calls():
        plans[1].pipeline_step(ims[1], maps[1], maps[0], post[0], occ[0])   # maps of frame 1, fusion of frame 0
        plans[0].pipeline_step(ims[0], maps[0], maps[1], post[1], occ[1])   # maps of frame 0, fusion of frame 1
        plans[0].reconstruct(ims[0], post[2], occ[2], ws)

    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plans[0].likelihood(ims[0], maps[0])
        calls()
        calls()                      # maps[0] now holds frame 0's maps, as before every replay
    torch.cuda.synchronize()
    ref = [t.clone() for t in post + occ + maps]
    g = capture(calls, stream)
    for rep in range(REPLAYS):
        scramble(post + occ)
        plans[1].reconstruct(ims[1], workspace=ws)            # eager work on the same workspace
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert same(post + occ + maps, ref), f"replay {rep}"


def test_two_and_four_frame_steps():
    say("graph replays: two- and four-frame steps, 64^3 x 4 views")
    frames = [S.config_frame(0, f) for f in range(4)]
    ims0, mus, vs = upload(frames[0])
    plan = plan_for(frames[0], mus, vs)
    ims = [ims0] + [upload(fr)[0] for fr in frames[1:]]
    shape = (frames[0].grid.nz, frames[0].grid.ny, frames[0].grid.nx)
    m2 = [plan.new_lmap_pair(), plan.new_lmap_pair()]
    m4 = [plan.new_lmap_quad(), plan.new_lmap_quad()]
    post = [torch.empty(shape, dtype=torch.float32, device="cuda") for _ in range(6)]
    occ = [torch.empty(shape, dtype=torch.uint8, device="cuda") for _ in range(6)]

    def calls():
        # maps of the later frames into one buffer beside the fusion of the other
        plan.pipeline_step_pair(ims[2], ims[3], m2[1], m2[0], post[0], occ[0], post[1], occ[1])
        plan.pipeline_step_pair(ims[0], ims[1], m2[0], m2[1], post[0], occ[0], post[1], occ[1])
        plan.pipeline_step_quad([ims[3], ims[2], ims[1], ims[0]], m4[1], m4[0], post[2:], occ[2:])
        plan.pipeline_step_quad(ims, m4[0], m4[1], post[2:], occ[2:])

    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan.pipeline_step_pair(ims[0], ims[1], m2[0])
        plan.pipeline_step_quad(ims, m4[0])
        calls()                      # m2[0] / m4[0] hold frames 0-1 / 0-3 again, as before every replay
    torch.cuda.synchronize()
    ref = [t.clone() for t in post + occ + m2 + m4]
    # the last fusion of each kind is of frames 2,3 (pair) and 3,2,1,0 (quad)
    singles = [plan.reconstruct(i) for i in ims]
    torch.cuda.synchronize()
    assert torch.equal(post[0], singles[2][0]) and torch.equal(post[1], singles[3][0])
    assert all(torch.equal(post[2 + f], singles[3 - f][0]) for f in range(4))
    g = capture(calls, stream)
    for rep in range(REPLAYS):
        scramble(post + occ)
        plan.reconstruct(ims[1])                              # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert same(post + occ + m2 + m4, ref), f"replay {rep}"


def test_surface_and_foreground_model():
    say("graph replays: surface list and foreground model, 64^3 x 4 views")
    fr = S.config_frame(0, 2)
    ims, mus, vs = upload(fr)
    plan = plan_for(fr, mus, vs)
    post, _ = plan.reconstruct(ims)
    lmap = plan.likelihood(ims)
    other = torch.rand_like(post)
    g_ = fr.grid
    V = g_.nx * g_.ny * g_.nz
    occ = torch.empty_like(post, dtype=torch.uint8)
    sm = torch.empty_like(post)
    out = torch.empty(V, dtype=torch.int32, device="cuda")
    count = torch.empty((), dtype=torch.int64, device="cuda")
    ws = torch.empty(max(plan.surface_workspace_bytes(), 4), dtype=torch.uint8, device="cuda")
    logd = torch.empty(psfs._lib.FG_BINS, dtype=torch.float32, device="cuda")
    fws = torch.empty(4 * psfs._lib.FG_BINS, dtype=torch.uint8, device="cuda")

    def calls():
        plan.surface(post, occ=occ, smoothed=sm, out=out, count=count, workspace=ws)
        plan.foreground_model(ims, lmap=lmap, out=logd, workspace=fws)

    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        calls()
    torch.cuda.synchronize()
    n = int(count.item())
    assert n > 100
    ref = [occ.clone(), sm.clone(), out[:n].clone(), count.clone(), logd.clone()]
    g = capture(calls, stream)
    for rep in range(REPLAYS):
        scramble([occ, sm, out, count, logd])
        plan.surface(other, workspace=ws)                     # eager work on the same workspaces
        plan.foreground_model(ims, masks=None, lmap=plan.likelihood(ims), workspace=fws)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert same([occ, sm, out[:n], count, logd], ref), f"replay {rep}"


def test_differentiable_forward_and_backward():
    say("graph replays: differentiable forward + backward, 64^3 x 4 views")
    fr = S.config_frame(0, 1)
    cams = S.perturb_cameras(fr.cams, seed=(0, 1))
    plan = psfs.Plan(cams, fr.grid, sampling=psfs.BILINEAR)
    ims, mus, vs = upload(fr)
    plan.set_backgrounds(mus, vs)
    lab = torch.from_numpy(S.gt_occupancy(fr.grid, fr.body)).cuda()
    lab2 = 1 - lab
    shape = tuple(lab.shape)
    ws = plan.new_diff_workspace()
    logits = torch.empty(shape, dtype=torch.float32, device="cuda")
    loss = torch.empty((), dtype=torch.float32, device="cuda")
    gl = torch.full((), 0.75, dtype=torch.float32, device="cuda")
    gm = [torch.empty_like(m) for m in mus]
    gv = [torch.empty_like(v) for v in vs]
    gP = torch.empty((len(cams), 3, 4), dtype=torch.float32, device="cuda")

    def calls():
        plan.diff_forward(ims, lab, None, logits, loss, ws)
        plan.diff_backward(ims, lab, logits, gl, ws, None, gm, gv, gP)

    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        calls()
    torch.cuda.synchronize()
    outs = [logits, loss, gP] + gm + gv
    ref = [t.clone() for t in outs]
    assert bool(torch.isfinite(loss).item()) and float(gP.abs().sum().item()) > 0.0
    g = capture(calls, stream)
    for rep in range(REPLAYS):
        scramble(outs)
        lg2, ls2, _ = plan.diff_forward(ims, lab2, workspace=ws)   # eager work on the same workspace
        plan.diff_backward(ims, lab2, lg2, gl, ws)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert same(outs, ref), f"replay {rep}"
