"""Plan autotuner (psfs_tune): it times the one-frame fusion with every tile,
keeps the fastest and caches the choice; no tile changes a result bit."""
import sys

import pytest
import torch

from synth import scene as S
from tests.gpu_util import plan_for, upload

pytestmark = pytest.mark.gpu


def test_every_tile_gives_the_same_bits_and_the_tuner_caches(tmp_path, monkeypatch):
    import paper_1311_6811_amd as psfs
    print("plan tuner: 128^3 x 8 views", flush=True)
    sys.stdout.flush()
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("PSFS_AUTOTUNE_CACHE", str(cache))
    fr = S.config_frame(1, 2)
    ims, mus, vs = upload(fr)
    plan = plan_for(fr, mus, vs)
    ref_p, ref_o = plan.reconstruct(ims)
    for t in range(len(psfs.tiles())):
        plan.set_tile(t)
        p, o = plan.reconstruct(ims)
        torch.cuda.synchronize()
        assert torch.equal(p, ref_p) and torch.equal(o, ref_o), f"tile {t}"
    best = plan.tune(ims, force=True)
    assert 0 <= best < len(psfs.tiles()) and plan.tile == best
    assert cache.exists() and "/plan/" in cache.read_text()
    p, o = plan.reconstruct(ims)
    torch.cuda.synchronize()
    assert torch.equal(p, ref_p) and torch.equal(o, ref_o)
    other = plan_for(fr, mus, vs)
    other.set_tile(0 if best != 0 else 1)
    assert other.tune(ims) == best and other.tile == best            # served from the cache
