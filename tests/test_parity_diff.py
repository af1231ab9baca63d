"""GPU differentiable pass (bilinear logits, BCE loss, adjoint) against the FP64
oracle and its analytic gradient (itself pinned to finite differences in the
CPU tests).

Tolerances (FP32 evaluation with an FP64 projection):
  logits   |dL| <= 5e-5 (FP32 log(2*SLM) maps, errors ~2e-6 each, summed over
           4 taps x n views)
  loss     relative 1e-5
  grads    per tensor, max |gpu - oracle| <= 1e-4 * max |oracle| (the voxel
           adjoint sigmoid(L) - y inherits the logit error; adjoint terms are
           rounded to 2^-20 of their bound)
"""
import sys

import numpy as np
import pytest
import torch

import paper_1311_6811_amd as psfs
from oracle import oracle as O
from synth import scene as S
from tests.gpu_util import upload

pytestmark = pytest.mark.gpu

LOGIT_TOL = 5e-5
LOSS_RTOL = 1e-5
GRAD_RTOL = 1e-4


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def scene():
    fr = S.config_frame(4, 0)
    cams = S.perturb_cameras(fr.cams)
    labels = S.gt_occupancy(fr.grid, fr.body)
    return fr, cams, labels


def run_gpu(fr, cams, labels, sub=None, grad_loss=1.0):
    ims, mus, vs = upload(fr)
    plan = psfs.Plan(cams, fr.grid, sampling=psfs.BILINEAR)
    plan.set_backgrounds(mus, vs)
    lab = torch.from_numpy(labels).cuda()
    logits, loss, ws = plan.diff_forward(ims, lab, sub)
    gl = torch.full((), grad_loss, dtype=torch.float32, device="cuda")
    gm, gv, gP = plan.diff_backward(ims, lab, logits, gl, ws, sub)
    torch.cuda.synchronize()
    return (logits.cpu().numpy(), float(loss), [g.cpu().numpy() for g in gm], [g.cpu().numpy() for g in gv],
            gP.cpu().numpy())


def check_grads(gm, gv, gP, ref, label):
    rgm, rgv, rgP = ref
    worst = {}
    for name, got, want in (("mean", gm, rgm), ("var", gv, rgv)):
        scale = max(float(np.max(np.abs(w))) for w in want)
        err = max(float(np.max(np.abs(g.astype(np.float64) - w))) for g, w in zip(got, want))
        worst[name] = err / scale
        assert err <= GRAD_RTOL * scale, f"{label} d/d{name}: {err:.3e} vs scale {scale:.3e}"
    for k in range(len(gP)):
        scale = float(np.max(np.abs(rgP[k])))
        err = float(np.max(np.abs(gP[k].astype(np.float64) - rgP[k])))
        worst[f"P{k}"] = err / scale
        assert err <= GRAD_RTOL * scale, f"{label} dP[{k}]: {err:.3e} vs scale {scale:.3e}"
    say(f"  {label}: relative errors " + ", ".join(f"{k} {v:.1e}" for k, v in worst.items()))


def test_diff_forward_parity(scene):
    fr, cams, labels = scene
    logits, loss, *_ = run_gpu(fr, cams, labels)
    l2s = [O.log2slm(i, m, v) for i, m, v in zip(fr.images, fr.mean, fr.var)]
    L = O.bilinear_logits(cams, fr.grid, l2s)
    err = float(np.max(np.abs(logits.astype(np.float64) - L)))
    say(f"  logits max error {err:.2e}")
    assert err <= LOGIT_TOL
    want = O.bce_loss(L, labels)
    assert loss == pytest.approx(want, rel=LOSS_RTOL)


def test_diff_backward_parity_whole_grid(scene):
    fr, cams, labels = scene
    _, _, gm, gv, gP = run_gpu(fr, cams, labels)
    ref = O.grad(cams, fr.grid, fr.images, fr.mean, fr.var, labels)
    check_grads(gm, gv, gP, ref, "whole grid")


def test_diff_backward_parity_fd_region(scene):
    fr, cams, labels = scene
    sub = S.fd_subgrid(fr.grid, fr.body)
    logits, loss, gm, gv, gP = run_gpu(fr, cams, labels, sub=sub, grad_loss=0.75)
    l2s = [O.log2slm(i, m, v) for i, m, v in zip(fr.images, fr.mean, fr.var)]
    assert loss == pytest.approx(O.bce_loss(O.bilinear_logits(cams, fr.grid, l2s), labels, sub), rel=LOSS_RTOL)
    ref = O.grad(cams, fr.grid, fr.images, fr.mean, fr.var, labels, sub, grad_loss=0.75)
    check_grads(gm, gv, gP, ref, "16^3 region")
    # pixels outside every projected footprint of the region get exactly zero
    touched = np.abs(ref[0][0]).sum(-1) > 0
    assert np.all(gm[0][~touched] == 0.0)


def test_small_scene_ragged_and_edge_views():
    rng = np.random.default_rng(17)
    cams = [S.look_at_camera((3.5 * np.cos(t), 3.5 * np.sin(t), 1.0), 260.0, W, H)
            for t, (W, H) in zip((0.2, 2.3, 4.4), ((161, 119), (97, 75), (130, 101)))]
    grid = S.Grid(45, 38, 29, np.array([-1.0, -0.9, -1.1], np.float32), np.float32(0.051))
    body = S.make_body(rng)
    fr = S.render_frame(20, 0, cams, grid, body, (20, 0))
    labels = S.gt_occupancy(grid, body)
    logits, loss, gm, gv, gP = run_gpu(fr, cams, labels, sub=[3, 40, 0, 38, 5, 29])
    l2s = [O.log2slm(i, m, v) for i, m, v in zip(fr.images, fr.mean, fr.var)]
    L = O.bilinear_logits(cams, grid, l2s)
    assert float(np.max(np.abs(logits - L))) <= LOGIT_TOL
    ref = O.grad(cams, grid, fr.images, fr.mean, fr.var, labels, [3, 40, 0, 38, 5, 29])
    check_grads(gm, gv, gP, ref, "ragged")


def test_boxes_too_large_or_behind_a_camera_take_the_direct_path():
    """Workgroups whose pixel box exceeds the LDS cap (a close camera with a
    long focal length) or has a corner behind the camera (a camera inside
    the grid) sample the maps directly; logits and gradients still follow
    the oracle."""
    rng = np.random.default_rng(23)
    cams = [S.look_at_camera((1.6, 0.4, 0.3), 900.0, 320, 240),            # boxes of ~10^5 pixels
            S.look_at_camera((0.35, 0.25, 0.12), 150.0, 200, 150, target=(-1.0, -0.5, 0.0)),   # inside the grid
            S.look_at_camera((-3.0, 1.5, 1.0), 280.0, 180, 140)]           # an ordinary view
    grid = S.Grid(40, 36, 30, np.array([-1.0, -0.9, -0.75], np.float32), np.float32(0.05))
    body = S.make_body(rng)
    fr = S.render_frame(20, 1, cams, grid, body, (20, 1))
    labels = S.gt_occupancy(grid, body)
    logits, loss, gm, gv, gP = run_gpu(fr, cams, labels)
    l2s = [O.log2slm(i, m, v) for i, m, v in zip(fr.images, fr.mean, fr.var)]
    L = O.bilinear_logits(cams, grid, l2s)
    err = float(np.max(np.abs(logits - L)))
    say(f"  logits max error {err:.2e}")
    assert err <= LOGIT_TOL
    want = O.bce_loss(L, labels)
    assert abs(loss - want) <= LOSS_RTOL * abs(want)
    ref = O.grad(cams, grid, fr.images, fr.mean, fr.var, labels)
    check_grads(gm, gv, gP, ref, "direct path")


def test_every_output_bitwise_reproducible(scene):
    # fixed-order reductions and fixed-point (integer) adjoint accumulation
    fr, cams, labels = scene
    a = run_gpu(fr, cams, labels)
    b = run_gpu(fr, cams, labels)
    assert np.array_equal(a[0], b[0]) and a[1] == b[1] and np.array_equal(a[4], b[4])
    assert all(np.array_equal(x, y) for x, y in zip(a[2], b[2]))
    assert all(np.array_equal(x, y) for x, y in zip(a[3], b[3]))


def test_loss_of_each_forward_on_one_workspace(scene):
    """Forwards with alternating label sets on one plan and one workspace:
    each loss equals that label set's loss from a fresh plan and workspace,
    bit for bit (no partial of an earlier forward leaks into a later sum)."""
    fr, cams, labels = scene
    rng = np.random.default_rng(5)
    other = (rng.random(labels.shape) < 0.3).astype(np.uint8)
    fresh = [run_gpu(fr, cams, lab)[1] for lab in (labels, other)]
    assert fresh[0] != fresh[1]
    ims, mus, vs = upload(fr)
    plan = psfs.Plan(cams, fr.grid, sampling=psfs.BILINEAR)
    plan.set_backgrounds(mus, vs)
    labs = [torch.from_numpy(labels).cuda(), torch.from_numpy(other).cuda()]
    ws = plan.new_diff_workspace()
    logits = torch.empty((fr.grid.nz, fr.grid.ny, fr.grid.nx), dtype=torch.float32, device="cuda")
    losses = [torch.empty((), dtype=torch.float32, device="cuda") for _ in range(6)]
    for i in range(6):
        plan.diff_forward(ims, labs[i % 2], None, logits, losses[i], ws)
    torch.cuda.synchronize()
    got = [float(x) for x in losses]
    say(f"  losses {got}")
    assert got == [fresh[i % 2] for i in range(6)]


def test_backward_twice_after_one_forward(scene):
    """A second backward after the same forward (no forward in between to
    clear the adjoint maps) gives the bits of the first."""
    fr, cams, labels = scene
    ims, mus, vs = upload(fr)
    plan = psfs.Plan(cams, fr.grid, sampling=psfs.BILINEAR)
    plan.set_backgrounds(mus, vs)
    lab = torch.from_numpy(labels).cuda()
    logits, loss, ws = plan.diff_forward(ims, lab)
    gl = torch.ones((), dtype=torch.float32, device="cuda")
    first = plan.diff_backward(ims, lab, logits, gl, ws)
    first = [[g.clone() for g in first[0]], [g.clone() for g in first[1]], first[2].clone()]
    second = plan.diff_backward(ims, lab, logits, gl, ws)
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(first[0], second[0]))
    assert all(torch.equal(a, b) for a, b in zip(first[1], second[1]))
    assert torch.equal(first[2], second[2])


def test_empty_loss_region_gives_zero():
    fr = S.config_frame(0, 0)
    labels = S.gt_occupancy(fr.grid, fr.body)
    logits, loss, gm, gv, gP = run_gpu(fr, fr.cams, labels, sub=[5, 5, 0, 64, 0, 64])
    assert loss == 0.0
    assert all(np.all(g == 0) for g in gm) and all(np.all(g == 0) for g in gv) and np.all(gP == 0)


def test_autograd_function_matches_binding_and_oracle():
    fr = S.config_frame(0, 1)
    cams = S.perturb_cameras(fr.cams, seed=(4, 1))
    labels = S.gt_occupancy(fr.grid, fr.body)
    ims, mus, vs = upload(fr)
    mus = [m.clone().requires_grad_(True) for m in mus]
    vs = [v.clone().requires_grad_(True) for v in vs]
    P = torch.tensor(np.stack([c.P for c in cams]), dtype=torch.float32, requires_grad=True)
    plan = psfs.DiffPlan(cams, fr.grid)
    lab = torch.from_numpy(labels).cuda()
    loss = psfs.occupancy_loss(P, mus, vs, ims, lab, plan)
    (2.0 * loss).backward()
    torch.cuda.synchronize()
    assert P.grad is not None and P.grad.device.type == "cpu"
    ref = O.grad(cams, fr.grid, fr.images, fr.mean, fr.var, labels, grad_loss=2.0)
    check_grads([m.grad.cpu().numpy() for m in mus], [v.grad.cpu().numpy() for v in vs], P.grad.numpy(), ref,
                "autograd")
    assert float(loss.detach()) == pytest.approx(O.loss(cams, fr.grid, fr.images, fr.mean, fr.var, labels), rel=LOSS_RTOL)


def test_autograd_two_forwards_on_one_plan_before_backward():
    # two losses on one shared plan, with different cameras and backgrounds,
    # summed before one backward: each backward must use its own forward's
    # cameras and backgrounds, not whatever the plan holds last
    fr_a = S.config_frame(0, 1)
    fr_b = S.config_frame(0, 2)
    cams_a = S.perturb_cameras(fr_a.cams, seed=(4, 1))
    cams_b = S.perturb_cameras(fr_b.cams, seed=(4, 2))
    lab_a = S.gt_occupancy(fr_a.grid, fr_a.body)
    lab_b = S.gt_occupancy(fr_b.grid, fr_b.body)
    plan = psfs.DiffPlan(cams_a, fr_a.grid)
    leaves = []
    losses = []
    for fr, cams, lab in ((fr_a, cams_a, lab_a), (fr_b, cams_b, lab_b)):
        ims, mus, vs = upload(fr)
        mus = [m.clone().requires_grad_(True) for m in mus]
        vs = [v.clone().requires_grad_(True) for v in vs]
        P = torch.tensor(np.stack([c.P for c in cams]), dtype=torch.float32, requires_grad=True)
        losses.append(psfs.occupancy_loss(P, mus, vs, ims, torch.from_numpy(lab).cuda(), plan))
        leaves.append((mus, vs, P))
    (losses[0] + 3.0 * losses[1]).backward()
    torch.cuda.synchronize()
    for (fr, cams, lab, gl), (mus, vs, P), name in zip(((fr_a, cams_a, lab_a, 1.0), (fr_b, cams_b, lab_b, 3.0)),
                                                        leaves, ("first", "second")):
        ref = O.grad(cams, fr.grid, fr.images, fr.mean, fr.var, lab, grad_loss=gl)
        check_grads([m.grad.cpu().numpy() for m in mus], [v.grad.cpu().numpy() for v in vs], P.grad.numpy(), ref,
                    f"{name} of two forwards")
