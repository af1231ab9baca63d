"""Helpers of the GPU tests: upload seeded scenes and compare against the
oracle with the tolerances the method's FP32 evaluation allows."""
import numpy as np
import torch

import paper_1311_6811_amd as psfs

POST_TOL = 1e-5          # absolute, on posteriors
OCC_BAND = 1e-4          # occupancy compared where |p_oracle - tau| > this


def upload(frame):
    dev = "cuda"
    ims = [torch.from_numpy(np.ascontiguousarray(i)).to(dev) for i in frame.images]
    mus = [torch.from_numpy(np.ascontiguousarray(m)).to(dev) for m in frame.mean]
    vs = [torch.from_numpy(np.ascontiguousarray(v)).to(dev) for v in frame.var]
    return ims, mus, vs


def plan_for(frame, mus, vs, **kw):
    plan = psfs.Plan(frame.cams, frame.grid, **kw)
    plan.set_backgrounds(mus, vs)
    return plan


def assert_posterior_parity(post_gpu, ref, tol=POST_TOL, combos=None, max_amb_frac=0.1, n_enum=200):
    """ref: oracle.Posterior. Unambiguous voxels within tol of the canonical
    posterior; ambiguous ones within [lo - tol, hi + tol], and a sample of them
    within tol of one admissible pixel-choice combination (combos(voxel))."""
    g = post_gpu.detach().cpu().numpy().astype(np.float64)
    assert g.shape == ref.post.shape
    assert np.all(np.isfinite(g))
    unamb = ref.ncombo == 1
    err = np.abs(g - ref.post)
    worst = float(err[unamb].max()) if unamb.any() else 0.0
    assert worst <= tol, f"max |gpu - oracle| = {worst:.3e} on unambiguous voxels"
    amb = ~unamb
    assert amb.mean() <= max_amb_frac, f"ambiguous fraction {amb.mean():.3f}"
    if amb.any():
        lo_ok = g[amb] >= ref.lo[amb] - tol
        hi_ok = g[amb] <= ref.hi[amb] + tol
        assert lo_ok.all() and hi_ok.all(), "ambiguous voxel outside its admissible range"
        if combos is not None:
            idx = np.flatnonzero(amb.reshape(-1))
            rng = np.random.default_rng(0)
            pick = idx if len(idx) <= n_enum else rng.choice(idx, n_enum, replace=False)
            flat = g.reshape(-1)
            for v in pick:
                vals = combos(int(v))
                assert np.min(np.abs(vals - flat[v])) <= tol, f"voxel {v}: {flat[v]} not in {vals}"
    return worst


def assert_occupancy_parity(occ_gpu, ref, tau=0.5, band=OCC_BAND, min_decided=0.98):
    o = occ_gpu.detach().cpu().numpy()
    assert o.dtype == np.uint8 and set(np.unique(o)) <= {0, 1}
    decided = ((np.minimum(np.minimum(np.abs(ref.lo - tau), np.abs(ref.hi - tau)), np.abs(ref.post - tau)) > band)
               & ((ref.lo > tau) == (ref.hi > tau)))
    want = (ref.post > tau).astype(np.uint8)
    assert decided.mean() >= min_decided
    mism = int((o[decided] != want[decided]).sum())
    assert mism == 0, f"{mism} decided voxels differ"
    return decided.mean()
