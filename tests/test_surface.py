"""GPU smoothing, threshold and surface extraction against the FP64 oracle
(oracle/surface.py). The smoothed posterior is a sum of 27 FP32 values, so it
matches to ~1e-6; thresholds are chosen away from every smoothed value by
more than that, so occupancy and the surface list must then match exactly."""
import sys

import numpy as np
import pytest
import torch
from scipy import ndimage

import paper_1311_6811_amd as psfs
from oracle import surface as SO
from synth import scene as S
from tests.gpu_util import plan_for, upload

pytestmark = pytest.mark.gpu

SMOOTH_TOL = 2e-6
BAND = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def field(shape, seed, sigma=1.5):
    rng = np.random.default_rng(seed)
    p = ndimage.gaussian_filter(rng.random(shape), sigma)
    p = (p - p.min()) / max(p.max() - p.min(), 1e-12)
    return p.astype(np.float32)


def clear_tau(sm, candidates=(0.5, 0.45, 0.55, 0.4, 0.6, 0.35, 0.65)):
    for t in candidates:
        if np.min(np.abs(sm - t)) > BAND:
            return t
    raise AssertionError("no threshold clear of the smoothed values")


def grid_of(shape):
    nz, ny, nx = shape
    return S.Grid(nx, ny, nz, np.zeros(3, np.float32), np.float32(0.01))


def run(post_np, tau, capacity=None, want_smoothed=True):
    nz, ny, nx = post_np.shape
    plan = psfs.Plan(None, grid_of(post_np.shape), threshold=tau)
    post = torch.from_numpy(np.ascontiguousarray(post_np)).cuda()
    res = plan.surface(post, capacity=capacity, want_smoothed=want_smoothed)
    torch.cuda.synchronize()
    return res


def check(post_np, tau=None):
    sm, _, _ = SO.extract(post_np.astype(np.float64))
    tau = clear_tau(sm) if tau is None else tau
    sm, occ, idx = SO.extract(post_np.astype(np.float64), tau)
    res = run(post_np, tau)
    got_sm = res.smoothed.cpu().numpy().astype(np.float64)
    assert np.abs(got_sm - sm).max() <= SMOOTH_TOL
    assert np.array_equal(res.occ.cpu().numpy(), occ)
    got = res.indices().cpu().numpy().astype(np.int64)
    assert int(res.count.item()) == len(idx)
    assert np.array_equal(got, idx)
    return len(idx)


# rows of a multiple of 4 voxels take the four-voxels-per-lane flag kernel,
# the others the one-voxel kernel
@pytest.mark.parametrize("shape", [(23, 29, 37), (16, 16, 16), (1, 1, 1), (7, 1, 5), (2, 33, 65), (40, 8, 130),
                                   (5, 7, 4), (1, 1, 8), (3, 9, 132), (13, 3, 64), (9, 1, 12)])
def test_random_fields_ragged_grids(shape):
    say(f"surface on {shape}")
    n = check(field(shape, sum(shape)))
    say(f"  {n} surface voxels")


def test_unaligned_occupancy_output():
    """Rows of whole 4-byte words but an occupancy array at an odd address: the
    one-voxel flag kernel runs and gives the same list as the oracle."""
    shape = (6, 9, 12)
    p = field(shape, 77)
    sm, _, _ = SO.extract(p.astype(np.float64))
    tau = clear_tau(sm)
    _, occ_ref, idx = SO.extract(p.astype(np.float64), tau)
    plan = psfs.Plan(None, grid_of(shape), threshold=tau)
    post = torch.from_numpy(np.ascontiguousarray(p)).cuda()
    raw = torch.empty(int(np.prod(shape)) + 1, dtype=torch.uint8, device="cuda")
    occ = raw[1:].view(shape)
    assert occ.data_ptr() % 4 == 1
    res = plan.surface(post, occ=occ)
    torch.cuda.synchronize()
    assert np.array_equal(occ.cpu().numpy(), occ_ref)
    assert int(res.count.item()) == len(idx)
    assert np.array_equal(res.indices().cpu().numpy().astype(np.int64), idx)


def test_posterior_of_the_headline_workload():
    say("surface of the 128^3 x 8-view posterior")
    fr = S.config_frame(1, 0)
    ims, mus, vs = upload(fr)
    plan = plan_for(fr, mus, vs)
    post, _ = plan.reconstruct(ims)
    torch.cuda.synchronize()
    p = post.cpu().numpy()
    n = check(p)
    say(f"  {n} surface voxels of {p.size}")
    assert n > 1000


def test_capacity_smaller_than_count():
    p = field((20, 24, 28), 5)
    sm, _, _ = SO.extract(p.astype(np.float64))
    tau = clear_tau(sm)
    _, _, idx = SO.extract(p.astype(np.float64), tau)
    assert len(idx) > 50
    cap = len(idx) // 3
    res = run(p, tau, capacity=cap, want_smoothed=False)
    assert int(res.count.item()) == len(idx)
    assert np.array_equal(res.out[:cap].cpu().numpy(), idx[:cap])
    assert res.smoothed is None


def test_solid_block_and_empty_grid():
    p = np.zeros((12, 12, 12), np.float32)
    p[2:10, 2:10, 2:10] = 1.0
    sm, occ, idx = SO.extract(p.astype(np.float64), 0.5)
    res = run(p, 0.5)
    assert np.array_equal(res.indices().cpu().numpy(), idx)
    plan = psfs.Plan(None, S.Grid(0, 4, 4, np.zeros(3, np.float32), np.float32(0.1)))
    res = plan.surface(torch.empty((4, 4, 0), device="cuda"))
    torch.cuda.synchronize()
    assert int(res.count.item()) == 0


def check_banded(p, tau=0.5):
    """Smoothed values within tolerance everywhere; occupancy where the
    oracle's smoothed value is clear of the threshold band; surface membership
    where the voxel and its six face neighbours all are. Returns (surface
    voxels, undecided voxels)."""
    sm, occ, idx = SO.extract(p.astype(np.float64), tau)
    res = run(p, tau)
    got_sm = res.smoothed.cpu().numpy().astype(np.float64)
    assert np.abs(got_sm - sm).max() <= SMOOTH_TOL
    clear = np.abs(sm - tau) > BAND
    got_occ = res.occ.cpu().numpy()
    assert np.array_equal(got_occ[clear], occ[clear])
    decided = clear.copy()
    pad = np.pad(clear, 1, constant_values=True)
    for axis in range(3):
        for d in (-1, 1):
            decided &= np.roll(pad, d, axis=axis)[1:-1, 1:-1, 1:-1]
    got = res.indices().cpu().numpy().astype(np.int64)
    assert int(res.count.item()) == len(got)
    assert np.all(np.diff(got) > 0)
    flat = decided.ravel()
    want_set = np.zeros(p.size, bool)
    want_set[idx] = True
    got_set = np.zeros(p.size, bool)
    got_set[got] = True
    assert np.array_equal(got_set[flat], want_set[flat])
    return len(got), int((~flat).sum())


def test_block_offsets_by_scan_kernel():
    """More than 4096 compaction blocks (17.0 M voxels): the block offsets come
    from the one-workgroup scan instead of each block's own sum."""
    shape = (260, 256, 256)
    say(f"surface on {shape} (scanned block offsets)")
    n, und = check_banded(field(shape, 31, sigma=3.0))
    say(f"  {n} surface voxels, {und} undecided")
    assert n > 10000 and und < 5e-3 * np.prod(shape)


def test_largest_workload_256cube_12_views():
    """The 256^3 posterior of the 12-view 1280x720 workload, threshold 1/2. At
    this size some smoothed values fall within the rounding band of the
    threshold, so occupancy is compared where the oracle's smoothed value is
    more than 1e-5 from it, and surface membership where the voxel and its six
    face neighbours all are."""
    say("surface of the 256^3 x 12-view posterior")
    fr = S.config_frame(2, 0)
    ims, mus, vs = upload(fr)
    plan = plan_for(fr, mus, vs)
    post, _ = plan.reconstruct(ims)
    torch.cuda.synchronize()
    p = post.cpu().numpy()
    n, und = check_banded(p)
    say(f"  {n} surface voxels, {und} undecided of {p.size}")
    assert n > 5000 and und < 1e-3 * p.size


@pytest.mark.parametrize("n", [1290, 1288])
def test_largest_grid_properties(n):
    """A 1290^3 grid (just under the 2^31-voxel limit, 524 k compaction blocks;
    rows of 1290 voxels take the one-voxel flag kernel, the 1288^3 grid the
    four-voxel one): a smooth ball-shaped posterior made on the GPU; checked by
    properties that hold at any size: the count equals the surface voxels of
    the returned occupancy (occupied with an unoccupied or out-of-grid face
    neighbour), the list is ascending and holds exactly those voxels, and
    sampled smoothed values are the 3x3x3 in-grid means of the posterior."""
    say(f"surface at {n}^3 (properties)")
    ax = torch.arange(n, device="cuda", dtype=torch.float32) / (n - 1) * 2.0 - 1.0
    r2 = ax.view(n, 1, 1) ** 2 + ax.view(1, n, 1) ** 2 + (1.3 * ax).view(1, 1, n) ** 2
    post = torch.sigmoid(40.0 * (0.6 - r2)).contiguous()
    del r2
    grid = S.Grid(n, n, n, np.zeros(3, np.float32), np.float32(0.01))
    plan = psfs.Plan(None, grid, threshold=0.5)
    res = plan.surface(post, want_smoothed=True)
    got = res.indices().to(torch.int64)
    occ = res.occ.bool()
    inner = torch.zeros_like(occ)
    inner[1:-1, 1:-1, 1:-1] = (occ[:-2, 1:-1, 1:-1] & occ[2:, 1:-1, 1:-1] & occ[1:-1, :-2, 1:-1] &
                               occ[1:-1, 2:, 1:-1] & occ[1:-1, 1:-1, :-2] & occ[1:-1, 1:-1, 2:])
    surf = (occ & ~inner).view(-1)
    del inner
    count = int(res.count.item())
    assert count == int(surf.sum().item()) == got.numel()
    assert bool((got[1:] > got[:-1]).all().item())
    assert bool(surf[got].all().item())
    assert count > 100000
    rng = np.random.default_rng(9)
    ks, js, is_ = (rng.integers(0, n, 200) for _ in range(3))
    ks[:4], js[:4], is_[:4] = [0, n - 1, 0, n - 1], [0, n - 1, n - 1, 0], [0, n - 1, 0, n - 1]
    for k, j, i in zip(ks, js, is_):
        lo = [max(c - 1, 0) for c in (k, j, i)]
        hi = [min(c + 2, n) for c in (k, j, i)]
        win = post[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]].double().cpu().numpy()
        m = win.mean()
        sm = float(res.smoothed[k, j, i].item())
        assert abs(sm - m) <= SMOOTH_TOL, (k, j, i, sm, m)
        assert int(res.occ[k, j, i].item()) == (1 if sm > 0.5 else 0)
    say(f"  {count} surface voxels")
