"""Batched pass over frames of uneven shape (a chain of pipelined launches), replayed from a HIP graph.

Every frame of a batch must be bit-identical to the same frame reconstructed
alone (same per-pixel and per-column code, fixed view order), and match the
FP64 oracle to the forward tolerances.
"""
import os
import sys

import numpy as np
import pytest
import torch

import paper_1311_6811_amd as psfs
from oracle import oracle as O
from synth import scene as S
from tests.gpu_util import assert_occupancy_parity, assert_posterior_parity, upload

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_batch_frame(fr, **kw):
    ims, mus, vs = upload(fr)
    return psfs.BatchFrame(fr.cams, fr.grid, ims, mus, vs, **kw)


@pytest.fixture(scope="module")
def mixed():
    say("generating 12 frames of the uneven-batch workload")
    frames = [S.config_frame(3, f) for f in range(12)]
    shapes = {(fr.grid.nx, fr.n, fr.cams[0].width) for fr in frames}
    assert len(shapes) >= 6
    return frames, [to_batch_frame(fr) for fr in frames]


def single(fr, bf, sampling=psfs.NEAREST):
    plan = psfs.Plan(fr.cams, fr.grid, sampling=sampling)
    plan.set_backgrounds(bf.means, bf.vars)
    return plan.reconstruct(bf.images)


def test_batch_bitwise_equals_single_frame(mixed):
    frames, bfs = mixed
    b = psfs.Batch(bfs)
    b.run()
    torch.cuda.synchronize()
    for fr, bf in zip(frames, bfs):
        post, occ = single(fr, bf)
        torch.cuda.synchronize()
        assert torch.equal(post, bf.posterior) and torch.equal(occ, bf.occ)


def test_batch_parity_vs_oracle(mixed):
    frames, bfs = mixed
    b = psfs.Batch(bfs)
    b.run()
    torch.cuda.synchronize()
    for fr, bf in sorted(zip(frames, bfs), key=lambda t: t[0].grid.nvox * t[0].n)[:4]:
        maps = [O.slm(i, m, v) for i, m, v in zip(fr.images, fr.mean, fr.var)]
        ref = O.posterior(fr.cams, fr.grid, maps)
        assert_posterior_parity(bf.posterior, ref, combos=lambda v: O.voxel_combos(fr.cams, fr.grid, maps, v),
                                n_enum=50)
        assert_occupancy_parity(bf.occ, ref)


def test_graph_replays_are_identical(mixed):
    frames, bfs = mixed
    b = psfs.Batch(bfs)
    b.run()
    torch.cuda.synchronize()
    first = [(bf.posterior.clone(), bf.occ.clone()) for bf in bfs]
    for _ in range(3):
        for bf in bfs:                       # eager work between replays
            bf.posterior.zero_()
            bf.occ.fill_(7)
        torch.cuda.synchronize()
        b.run()
        torch.cuda.synchronize()
        for (p0, o0), bf in zip(first, bfs):
            assert torch.equal(p0, bf.posterior) and torch.equal(o0, bf.occ)


def test_update_keeps_graph_and_redirects_outputs(mixed):
    frames, bfs = mixed
    b = psfs.Batch(bfs)
    b.run()
    torch.cuda.synchronize()
    ref = [bf.posterior.clone() for bf in bfs]
    # same shapes: swap the inputs of two same-signature-free frames is not
    # allowed, but fresh outputs and a shifted grid origin are
    moved = []
    for fr, bf in zip(frames, bfs):
        moved.append(psfs.BatchFrame(fr.cams, fr.grid, bf.images, bf.means, bf.vars))
    b.update(moved)
    b.run()
    torch.cuda.synchronize()
    for r, m in zip(ref, moved):
        assert torch.equal(r, m.posterior)


def test_update_with_new_shape_is_stale(mixed):
    frames, bfs = mixed
    b = psfs.Batch(bfs[:2])
    fr = frames[0]
    g = S.Grid(fr.grid.nx + 1, fr.grid.ny, fr.grid.nz, fr.grid.origin, fr.grid.voxel)
    bad = [psfs.BatchFrame(fr.cams, g, bfs[0].images, bfs[0].means, bfs[0].vars), bfs[1]]
    with pytest.raises(psfs.PsfsError) as ei:
        b.update(bad)
    assert ei.value.status == -7


def test_autotuner_picks_a_tile_and_keeps_bits(mixed, tmp_path, monkeypatch):
    frames, bfs = mixed
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("PSFS_AUTOTUNE_CACHE", str(cache))
    b = psfs.Batch(bfs[:6])
    b.run()
    torch.cuda.synchronize()
    ref = [bf.posterior.clone() for bf in bfs[:6]]
    best = b.tune(force=True)
    assert 0 <= best < len(psfs.tiles()) and b.tile == best
    assert cache.exists() and "gfx950" in cache.read_text()
    b.run()
    torch.cuda.synchronize()
    for r, bf in zip(ref, bfs[:6]):
        assert torch.equal(r, bf.posterior)
    b2 = psfs.Batch(bfs[:6])
    assert b2.tune() == best                  # served from the cache
    say(f"  tuned tile {best}: {psfs.tiles()[best]}")


def test_bilinear_batch_matches_single_plan(mixed):
    frames, _ = mixed
    bfs = [to_batch_frame(fr) for fr in frames[:5]]
    b = psfs.Batch(bfs, sampling=psfs.BILINEAR)
    b.run()
    torch.cuda.synchronize()
    for fr, bf in zip(frames[:5], bfs):
        post, occ = single(fr, bf, psfs.BILINEAR)
        torch.cuda.synchronize()
        assert torch.equal(post, bf.posterior) and torch.equal(occ, bf.occ)


def test_batch_with_empty_grid_and_no_occupancy_output():
    fr0 = S.config_frame(0, 0)
    bf0 = to_batch_frame(fr0, want_occ=False)
    empty = S.Grid(0, 8, 8, np.zeros(3, np.float32), np.float32(0.1))
    bf1 = psfs.BatchFrame(fr0.cams, empty, bf0.images, bf0.means, bf0.vars)
    b = psfs.Batch([bf1, bf0, bf1])
    b.run()
    torch.cuda.synchronize()
    post, _ = single(fr0, bf0)
    torch.cuda.synchronize()
    assert torch.equal(post, bf0.posterior)


def test_batch_with_the_largest_grid():
    """A 1290^3 frame (just under the 2^31-voxel limit, ~2.1 M bricks) batched
    with two small frames: every frame bit-identical to the frame alone."""
    say("batch: 1290^3 x 4 views with two small frames")
    f, W, H = S.IMAGE_CLASSES[0]
    cams = S.ring_rig(4, f, W, H)
    rng = np.random.default_rng(93)
    frames = [S.render_frame(15, 0, cams, S.cube_grid(1290, 2.0), S.make_body(rng), (15, 0)),
              S.config_frame(3, 0), S.config_frame(3, 1)]
    bfs = [to_batch_frame(fr) for fr in frames]
    b = psfs.Batch(bfs)
    b.run()
    torch.cuda.synchronize()
    for fr, bf in zip(frames, bfs):
        post, occ = single(fr, bf)
        torch.cuda.synchronize()
        assert torch.equal(post, bf.posterior) and torch.equal(occ, bf.occ)


def test_every_tile_keeps_the_bits(mixed):
    """Each tile (one launch per chain step for 256-lane tiles, likelihood
    then fusion launches for the 128-lane one) gives every frame the bits of
    the frame alone."""
    frames, bfs = mixed
    refs = []
    for fr, bf in zip(frames[:7], bfs[:7]):
        post, occ = single(fr, bf)
        refs.append((post, occ))
    torch.cuda.synchronize()
    b = psfs.Batch(bfs[:7])
    for t in range(len(psfs.tiles())):
        say(f"  tile {t}: {psfs.tiles()[t]}")
        b.set_tile(t)
        for bf in bfs[:7]:
            bf.posterior.fill_(-1.0)
            bf.occ.fill_(7)
        b.run()
        torch.cuda.synchronize()
        for (post, occ), bf in zip(refs, bfs[:7]):
            assert torch.equal(post, bf.posterior) and torch.equal(occ, bf.occ)


def test_whole_64_frame_batch_bitwise_equals_single_frames():
    """The whole uneven 64-frame workload (grid edge 64-192, 4-12 views, three
    image sizes) as one batch: every frame bit-identical to the frame
    reconstructed alone."""
    from concurrent.futures import ThreadPoolExecutor
    say("batch: the whole 64-frame uneven workload")
    with ThreadPoolExecutor(8) as ex:
        frames = list(ex.map(lambda f: S.config_frame(3, f), range(64)))
    bfs = [to_batch_frame(fr) for fr in frames]
    b = psfs.Batch(bfs)
    b.run()
    b.run()                                   # the graph replay after the capturing run
    torch.cuda.synchronize()
    for k, (fr, bf) in enumerate(zip(frames, bfs)):
        post, occ = single(fr, bf)
        torch.cuda.synchronize()
        assert torch.equal(post, bf.posterior) and torch.equal(occ, bf.occ), f"frame {k}"
