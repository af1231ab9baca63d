"""psfs_reconstruct_static (no workspace argument, likelihood maps in the
library's static device array) called through the C ABI: its posterior and
occupancy equal psfs_reconstruct's bit for bit on two calls in a row, the
second with a smaller input, and a plan whose maps exceed the array is
refused before anything is enqueued."""
import ctypes as C
import sys

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


def outputs(grid, fill_p=-1.0, fill_o=7):
    shape = (grid.nz, grid.ny, grid.nx)
    return (torch.full(shape, fill_p, dtype=torch.float32, device="cuda"),
            torch.full(shape, fill_o, dtype=torch.uint8, device="cuda"))


def static_call(plan, ims, post, occ):
    arr = L.ptr_array([t.data_ptr() for t in ims])
    return L.lib().psfs_reconstruct_static(plan.handle, arr, post.data_ptr(), occ.data_ptr(),
                                           torch.cuda.current_stream().cuda_stream)


def test_static_scratch_matches_reconstruct_twice():
    for cfg in (1, 0):                                  # 128^3 x 8 views, then the smaller 64^3 x 4
        say(f"static-scratch reconstruction, config {cfg}")
        fr = S.config_frame(cfg, 3)
        ims, mus, vs = upload(fr)
        plan = plan_for(fr, mus, vs)
        assert 0 < plan.workspace_bytes() <= L.STATIC_SCRATCH_BYTES
        p_ref, o_ref = plan.reconstruct(ims)
        p, o = outputs(fr.grid)
        assert static_call(plan, ims, p, o) == 0
        torch.cuda.synchronize()
        assert torch.equal(p, p_ref), f"config {cfg}: posterior differs"
        assert torch.equal(o, o_ref), f"config {cfg}: occupancy differs"


def test_static_scratch_refuses_maps_beyond_its_size():
    say("static-scratch reconstruction, too large")
    fr = S.config_frame(0, 0)
    ims, mus, vs = upload(fr)
    plan = plan_for(fr, mus, vs)
    cams = [S.look_at_camera((4.0, 0.0, 1.5), 3000.0, 4096, 4096)] * 1     # 64 MiB of maps
    plan.set_cameras(cams)
    big = torch.zeros((4096, 4096, 3), dtype=torch.float32, device="cuda")
    plan.set_backgrounds([big], [big])
    img = torch.zeros((4096, 4096, 3), dtype=torch.uint8, device="cuda")
    p, o = outputs(fr.grid)
    assert plan.workspace_bytes() > L.STATIC_SCRATCH_BYTES
    assert static_call(plan, [img], p, o) == -2
    assert "static scratch" in L.lib().psfs_last_error().decode()
    torch.cuda.synchronize()
    assert bool((p == -1.0).all()) and bool((o == 7).all())          # nothing ran
