"""GPU voxel colouring against the FP64 oracle (oracle/colour.py) on the
surface voxels of reconstructed frames. Voxels whose visibility could change
under FP32 rounding (flagged by the oracle) are left out; the rest must have
the same number of views and the same mean colour (integer sums divided once
in FP32: within 2e-5 of the FP64 mean)."""
import sys

import numpy as np
import pytest
import torch

import paper_1311_6811_amd as psfs
from oracle import colour as CO
from synth import scene as S
from tests.gpu_util import plan_for, upload

pytestmark = pytest.mark.gpu

COLOUR_ATOL = 2e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def check(fr, plan, ims, idx_t):
    col, views = plan.colour(ims, idx_t)
    torch.cuda.synchronize()
    idx = idx_t.cpu().numpy().astype(np.int64)
    want, wviews, amb = CO.colour(fr.cams, fr.grid, fr.images, idx)
    keep = ~amb
    # surface voxels sit ~2.3 px apart at 640x480, so an ambiguous projection
    # (~0.5 % of them) taints every candidate at the pixels it may reach:
    # ~13 % of the voxels at 128^3 x 8 views
    assert keep.mean() >= 0.8, f"only {keep.mean():.3f} of the voxels are unambiguous"
    got_v = views.cpu().numpy()
    got_c = col.cpu().numpy().astype(np.float64)
    assert np.array_equal(got_v[keep], wviews[keep])
    assert np.abs(got_c[keep] - want[keep]).max() <= COLOUR_ATOL
    return int(keep.sum()), len(idx)


@pytest.mark.parametrize("cfg", [0, 1, 2])
def test_surface_voxel_colours(cfg):
    say(f"colour of the surface voxels, config {cfg}")
    fr = S.config_frame(cfg, 0)
    ims, mus, vs = upload(fr)
    plan = plan_for(fr, mus, vs)
    post, _ = plan.reconstruct(ims)
    surf = plan.surface(post)
    idx = surf.indices()
    assert idx.numel() > 100
    kept, n = check(fr, plan, ims, idx.contiguous())
    say(f"  {kept} of {n} voxels compared")


def test_random_list_with_repeats_and_outside_entries():
    fr = S.config_frame(0, 3)
    ims, mus, vs = upload(fr)
    plan = plan_for(fr, mus, vs)
    rng = np.random.default_rng(9)
    idx = rng.choice(fr.grid.nvox, 5000, replace=False).astype(np.int32)
    idx[100:120] = idx[:20]                                  # repeats: the earlier entry wins its pixels
    check(fr, plan, ims, torch.from_numpy(idx).cuda())
    bad = torch.tensor([-1, fr.grid.nvox, 2 ** 31 - 1], dtype=torch.int32, device="cuda")
    col, views = plan.colour(ims, bad)
    torch.cuda.synchronize()
    assert int(views.abs().sum()) == 0 and float(col.abs().sum()) == 0.0


def test_empty_list_is_a_no_op():
    fr = S.config_frame(0, 0)
    ims, mus, vs = upload(fr)
    plan = plan_for(fr, mus, vs)
    col, views = plan.colour(ims, torch.empty(0, dtype=torch.int32, device="cuda"))
    torch.cuda.synchronize()
    assert col.shape == (0, 3) and views.shape == (0,)


def test_reused_workspace_and_graph_replays():
    """One workspace across calls with different lists (the depth buffer keeps
    entries of the earlier list that the later one never reaches), then the
    same call captured in a HIP graph and replayed with eager work between the
    replays: every result matches the oracle's."""
    fr = S.config_frame(0, 1)
    ims, mus, vs = upload(fr)
    plan = plan_for(fr, mus, vs)
    ws = torch.empty(max(plan.colour_workspace_bytes(), 8), dtype=torch.uint8, device="cuda")
    rng = np.random.default_rng(21)
    lists = [torch.from_numpy(rng.choice(fr.grid.nvox, m, replace=False).astype(np.int32)).cuda()
             for m in (6000, 1500)]
    for idx_t in lists:
        col, views = plan.colour(ims, idx_t, workspace=ws)
        torch.cuda.synchronize()
        idx = idx_t.cpu().numpy().astype(np.int64)
        want, wviews, amb = CO.colour(fr.cams, fr.grid, fr.images, idx)
        keep = ~amb
        assert np.array_equal(views.cpu().numpy()[keep], wviews[keep])
        assert np.abs(col.cpu().numpy().astype(np.float64)[keep] - want[keep]).max() <= COLOUR_ATOL

    idx_t = lists[0]
    idx = idx_t.cpu().numpy().astype(np.int64)
    want, wviews, amb = CO.colour(fr.cams, fr.grid, fr.images, idx)
    keep = ~amb
    col = torch.empty((idx_t.numel(), 3), dtype=torch.float32, device="cuda")
    views = torch.empty(idx_t.numel(), dtype=torch.int32, device="cuda")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan.colour(ims, idx_t, colour=col, views=views, workspace=ws)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            plan.colour(ims, idx_t, colour=col, views=views, workspace=ws)
    for rep in range(3):
        col.fill_(-1.0)
        views.fill_(-1)
        plan.colour(ims, lists[1], workspace=ws)              # eager work on the same depth buffer
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(views.cpu().numpy()[keep], wviews[keep]), rep
        assert np.abs(col.cpu().numpy().astype(np.float64)[keep] - want[keep]).max() <= COLOUR_ATOL, rep
