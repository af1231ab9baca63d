"""Python binding of the C ABI (argument marshalling only).

Torch provides device memory and the stream: every tensor passed here must be
a contiguous tensor on the current GPU with the documented dtype; all compute
runs in the library's HIP kernels, enqueued on
``torch.cuda.current_stream()``.
"""
from __future__ import annotations

import ctypes as C
import math
from typing import Optional, Sequence, Tuple

import numpy as np
import torch

from . import _lib as L

LOG_U_DEFAULT = -3.0 * math.log(256.0)


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _dev(t: torch.Tensor, dtype: torch.dtype, name: str, shape=None) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t.data_ptr()


def make_camera(width: int, height: int, P) -> L.psfs_camera:
    c = L.psfs_camera()
    c.width, c.height = int(width), int(height)
    flat = np.asarray(P, np.float32).reshape(12)
    for e in range(12):
        c.P[e] = float(flat[e])
    return c


def make_grid(nx, ny, nz, origin, voxel) -> L.psfs_grid:
    g = L.psfs_grid()
    g.nx, g.ny, g.nz = int(nx), int(ny), int(nz)
    o = np.asarray(origin, np.float32).reshape(3)
    for d in range(3):
        g.origin[d] = float(o[d])
    g.voxel = float(np.float32(voxel))
    return g


def threshold(posterior: torch.Tensor, tau: float = 0.5, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    occ = out if out is not None else torch.empty(posterior.shape, dtype=torch.uint8, device=posterior.device)
    L.check(L.lib().psfs_threshold(_dev(posterior, torch.float32, "posterior"), posterior.numel(), float(tau),
                                   _dev(occ, torch.uint8, "occ", posterior.shape), _stream()))
    return occ


class Plan:
    """A reconstruction plan: cameras, grid, parameters and background model.

    ``cams``: objects with ``width``, ``height`` and a 3x4 ``P`` (FP32).
    ``grid``: object with ``nx, ny, nz, origin, voxel``.
    """

    def __init__(self, cams=None, grid=None, prior=0.5, log_u=LOG_U_DEFAULT, threshold=0.5,
                 sampling: int = L.NEAREST):
        h = C.c_void_p()
        L.check(L.lib().psfs_plan_create(C.byref(h)))
        self._h = h
        # held by the object: module globals may be gone when it is collected at exit
        self._destroy = L.lib().psfs_plan_destroy
        self._keep = {}
        self.cams = []
        self.grid = None
        self.set_params(prior, log_u, threshold, sampling)
        if cams is not None:
            self.set_cameras(cams)
        if grid is not None:
            self.set_grid(grid)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    # -------------------------------------------------------------- setup
    def set_cameras(self, cams: Sequence) -> None:
        arr = (L.psfs_camera * max(len(cams), 1))(*[make_camera(c.width, c.height, c.P) for c in cams])
        L.check(L.lib().psfs_set_cameras(self._h, len(cams), arr))
        self.cams = list(cams)
        self._keep = {k: v for k, v in self._keep.items() if not k.startswith("bg")}

    def set_grid(self, grid) -> None:
        g = make_grid(grid.nx, grid.ny, grid.nz, grid.origin, grid.voxel)
        L.check(L.lib().psfs_set_grid(self._h, C.byref(g)))
        self.grid = grid

    def set_params(self, prior=0.5, log_u=LOG_U_DEFAULT, threshold=0.5, sampling: int = L.NEAREST) -> None:
        p = L.psfs_params(float(prior), float(log_u), float(threshold), int(sampling))
        L.check(L.lib().psfs_set_params(self._h, C.byref(p)))
        self.params = p

    def set_tile(self, tile: int) -> None:
        L.check(L.lib().psfs_set_tile(self._h, int(tile)))

    @property
    def tile(self) -> int:
        return L.check(L.lib().psfs_get_tile(self._h))

    def tune(self, images: Sequence[torch.Tensor], force: bool = False) -> int:
        """Times the one-frame fusion with every tile on these images (or
        takes the cached choice) and keeps the fastest; returns its index."""
        ims = self._images(images)
        ws = torch.empty(max(int(L.lib().psfs_tune_workspace_bytes(self._h)), 256), dtype=torch.uint8, device="cuda")
        best = C.c_int32(-1)
        L.check(L.lib().psfs_tune(self._h, ims, ws.data_ptr(), ws.numel(), _stream(), int(bool(force)),
                                  C.byref(best)))
        return int(best.value)

    def set_background(self, view: int, mean: torch.Tensor, var: torch.Tensor) -> None:
        c = self.cams[view]
        shape = (c.height, c.width, 3)
        mp = _dev(mean, torch.float32, "mean", shape)
        vp_ = _dev(var, torch.float32, "var", shape)
        L.check(L.lib().psfs_set_background(self._h, int(view), mp, vp_))
        self._keep[f"bg{view}"] = (mean, var)

    def set_backgrounds(self, means: Sequence[torch.Tensor], vars_: Sequence[torch.Tensor]) -> None:
        for k, (m, v) in enumerate(zip(means, vars_)):
            self.set_background(k, m, v)

    # --------------------------------------------------------- buffers
    def set_input_check(self, flags: Optional[torch.Tensor]) -> None:
        """Device check of the background model (variances positive and
        finite, means finite) in every later likelihood pass of this plan:
        `flags` is a zeroed one-element int32 GPU tensor that receives bit k
        when view k holds an invalid value; None turns the check off."""
        ptr = _dev(flags, torch.int32, "flags", (1,)) if flags is not None else None
        L.check(L.lib().psfs_set_input_check(self._h, ptr))
        self._check_flags = flags                  # keep the word alive while the plan uses it

    def input_status(self) -> None:
        """After synchronising with the checked work: raises PsfsError
        (PSFS_E_INPUT, naming the views) if an invalid value was seen, and
        clears the flags."""
        L.check(L.lib().psfs_input_status(self._h))

    @property
    def n(self) -> int:
        return len(self.cams)

    def lmap_floats(self) -> int:
        return L.check(L.lib().psfs_lmap_floats(self._h))

    def lmap_offset(self, view: int) -> int:
        return L.check(L.lib().psfs_lmap_offset(self._h, int(view)))

    def workspace_bytes(self) -> int:
        return int(L.lib().psfs_workspace_bytes(self._h))

    def new_workspace(self, nbytes: Optional[int] = None) -> torch.Tensor:
        n = self.workspace_bytes() if nbytes is None else nbytes
        return torch.empty(max(n, 16), dtype=torch.uint8, device="cuda")

    def _images(self, images: Sequence[torch.Tensor]):
        if len(images) != self.n:
            raise ValueError(f"expected {self.n} images, got {len(images)}")
        ptrs = [_dev(im, torch.uint8, f"images[{k}]", (c.height, c.width, 3))
                for k, (im, c) in enumerate(zip(images, self.cams))]
        return L.ptr_array(ptrs)

    def _map(self, t: torch.Tensor, frames: int, name: str) -> int:
        """Device pointer of a map buffer that must hold `frames` interleaved
        frames' maps (frames * lmap_floats() FP32 values): the C entry points
        take no length for it, so a short buffer is refused here."""
        need = frames * self.lmap_floats()
        if t is None or t.numel() < need:
            got = None if t is None else t.numel()
            raise ValueError(f"{name}: needs at least {need} float32 elements ({frames} x lmap_floats), got {got}")
        return _dev(t, torch.float32, name)

    def lmap_view(self, lmap: torch.Tensor, view: int) -> torch.Tensor:
        c = self.cams[view]
        off = self.lmap_offset(view)
        return lmap[off:off + c.width * c.height].view(c.height, c.width)

    # --------------------------------------------------------- compute
    def likelihood(self, images: Sequence[torch.Tensor], out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Eq. 1-2: log(2*SLM) maps of all views in one buffer (psfs_lmap_* layout)."""
        lmap = out if out is not None else torch.empty(max(self.lmap_floats(), 4), dtype=torch.float32, device="cuda")
        L.check(L.lib().psfs_likelihood(self._h, self._images(images), self._map(lmap, 1, "lmap"), _stream()))
        return lmap

    def _outputs(self, posterior, occ, want_occ):
        g = self.grid
        shape = (g.nz, g.ny, g.nx)
        post = posterior if posterior is not None else torch.empty(shape, dtype=torch.float32, device="cuda")
        if want_occ and occ is None:
            occ = torch.empty(shape, dtype=torch.uint8, device="cuda")
        pp = _dev(post, torch.float32, "posterior", shape)
        op = _dev(occ, torch.uint8, "occ", shape) if occ is not None else None
        return post, occ, pp, op

    def fuse(self, lmap: torch.Tensor, posterior=None, occ=None, want_occ=True) -> Tuple[torch.Tensor, Optional[torch.Tensor]]:
        """Eq. 3-9 (+ threshold) from likelihood maps."""
        post, occ, pp, op = self._outputs(posterior, occ, want_occ)
        L.check(L.lib().psfs_fuse(self._h, self._map(lmap, 1, "lmap"), pp, op, _stream()))
        return post, occ

    def reconstruct(self, images: Sequence[torch.Tensor], posterior=None, occ=None, workspace=None,
                    want_occ=True) -> Tuple[torch.Tensor, Optional[torch.Tensor]]:
        """Likelihood maps + fusion + threshold for one frame."""
        ims = self._images(images)
        post, occ, pp, op = self._outputs(posterior, occ, want_occ)
        ws = workspace if workspace is not None else self.new_workspace()
        L.check(L.lib().psfs_reconstruct(self._h, ims, pp, op, _dev(ws, torch.uint8, "workspace"),
                                         ws.numel(), _stream()))
        return post, occ

    def reconstruct_static(self, images: Sequence[torch.Tensor], posterior=None, occ=None,
                           want_occ=True) -> Tuple[torch.Tensor, Optional[torch.Tensor]]:
        """reconstruct() with the likelihood maps in the library's static
        device array (psfs_reconstruct_static: for callers that cannot
        allocate; pass preallocated outputs to allocate nothing)."""
        ims = self._images(images)
        post, occ, pp, op = self._outputs(posterior, occ, want_occ)
        L.check(L.lib().psfs_reconstruct_static(self._h, ims, pp, op, _stream()))
        return post, occ

    def new_lmap(self) -> torch.Tensor:
        return torch.empty(max(self.lmap_floats(), 4), dtype=torch.float32, device="cuda")

    def pipeline_step(self, images=None, lmap_next: Optional[torch.Tensor] = None,
                      lmap_cur: Optional[torch.Tensor] = None, posterior=None, occ=None) -> None:
        """One launch: likelihood maps of `images` into `lmap_next` and fusion of
        the maps `lmap_cur` (from an earlier step) into `posterior` / `occ`.
        Either part may be omitted (images=None / posterior=None)."""
        ims = self._images(images) if images is not None else None
        nxt = self._map(lmap_next, 1, "lmap_next") if images is not None else None
        cur = pp = op = None
        if posterior is not None:
            shape = (self.grid.nz, self.grid.ny, self.grid.nx)
            pp = _dev(posterior, torch.float32, "posterior", shape)
            op = _dev(occ, torch.uint8, "occ", shape) if occ is not None else None
            cur = self._map(lmap_cur, 1, "lmap_cur")
        L.check(L.lib().psfs_pipeline_step(self._h, ims, nxt, cur, pp, op, _stream()))

    def new_lmap_pair(self) -> torch.Tensor:
        """Pair-map buffer of two frames (interleaved, see psfs_pipeline_step_pair)."""
        return torch.empty(max(2 * self.lmap_floats(), 4), dtype=torch.float32, device="cuda")

    def pipeline_step_pair(self, images_a=None, images_b=None, lmap2_next: Optional[torch.Tensor] = None,
                           lmap2_cur: Optional[torch.Tensor] = None, post_a=None, occ_a=None, post_b=None,
                           occ_b=None) -> None:
        """One launch for two frames of the sequence: pair maps of (images_a,
        images_b) into lmap2_next and the fusion of the pair maps lmap2_cur into
        (post_a, occ_a) and (post_b, occ_b). Either part may be omitted."""
        ia = self._images(images_a) if images_a is not None else None
        ib = self._images(images_b) if images_b is not None else None
        nxt = self._map(lmap2_next, 2, "lmap2_next") if images_a is not None else None
        shape = (self.grid.nz, self.grid.ny, self.grid.nx)
        pa = _dev(post_a, torch.float32, "post_a", shape) if post_a is not None else None
        pb = _dev(post_b, torch.float32, "post_b", shape) if post_b is not None else None
        oa = _dev(occ_a, torch.uint8, "occ_a", shape) if occ_a is not None else None
        ob = _dev(occ_b, torch.uint8, "occ_b", shape) if occ_b is not None else None
        cur = self._map(lmap2_cur, 2, "lmap2_cur") if (post_a is not None or post_b is not None) else None
        L.check(L.lib().psfs_pipeline_step_pair(self._h, ia, ib, nxt, cur, pa, oa, pb, ob, _stream()))

    def new_lmap_quad(self) -> torch.Tensor:
        """Quad-map buffer of four frames (interleaved, see psfs_pipeline_step_quad)."""
        return torch.empty(max(4 * self.lmap_floats(), 4), dtype=torch.float32, device="cuda")

    def pipeline_step_quad(self, images=None, lmap4_next: Optional[torch.Tensor] = None,
                           lmap4_cur: Optional[torch.Tensor] = None, posts=None, occs=None) -> None:
        """One launch for four frames of the sequence: quad maps of the four
        frames' `images` (a sequence of four per-view image lists) into
        lmap4_next and the fusion of the quad maps lmap4_cur into the four
        posteriors `posts` (and occupancies `occs`, or None). Either part may
        be omitted."""
        ims = None
        nxt = None
        if images is not None:
            if len(images) != 4:
                raise ValueError(f"expected the images of 4 frames, got {len(images)}")
            flat = [p for fr in images for p in self._images(fr)[:self.n]]
            ims = L.ptr_array(flat)
            nxt = self._map(lmap4_next, 4, "lmap4_next")
        pp = op = cur = None
        if posts is not None:
            if len(posts) != 4 or (occs is not None and len(occs) != 4):
                raise ValueError("expected 4 posteriors (and 4 occupancies or None)")
            shape = (self.grid.nz, self.grid.ny, self.grid.nx)
            pp = L.ptr_array([_dev(t, torch.float32, f"posts[{f}]", shape) for f, t in enumerate(posts)])
            if occs is not None:
                op = L.ptr_array([_dev(t, torch.uint8, f"occs[{f}]", shape) if t is not None else None
                                  for f, t in enumerate(occs)])
            cur = self._map(lmap4_cur, 4, "lmap4_cur")
        L.check(L.lib().psfs_pipeline_step_quad(self._h, ims, nxt, cur, pp, op, _stream()))

    # ------------------------------------- smoothing and surface voxels
    def surface_workspace_bytes(self) -> int:
        return int(L.lib().psfs_surface_workspace_bytes(self._h))

    def surface(self, posterior: torch.Tensor, capacity: Optional[int] = None, occ=None, smoothed=None,
                want_smoothed: bool = False, out=None, count=None, workspace=None) -> "Surface":
        """Smoothing (3x3x3 in-grid mean), threshold and surface voxels of a
        posterior grid. Asynchronous: ``Surface.indices()`` synchronises."""
        g = self.grid
        shape = (g.nz, g.ny, g.nx)
        nvox = g.nx * g.ny * g.nz
        cap = nvox if capacity is None else int(capacity)
        occ = occ if occ is not None else torch.empty(shape, dtype=torch.uint8, device="cuda")
        if want_smoothed and smoothed is None:
            smoothed = torch.empty(shape, dtype=torch.float32, device="cuda")
        out = out if out is not None else torch.empty(max(cap, 1), dtype=torch.int32, device="cuda")
        count = count if count is not None else torch.empty((), dtype=torch.int64, device="cuda")
        ws = workspace if workspace is not None else torch.empty(max(self.surface_workspace_bytes(), 4),
                                                                 dtype=torch.uint8, device="cuda")
        if out.numel() < cap:
            raise ValueError("out holds fewer than capacity entries")
        L.check(L.lib().psfs_surface(self._h, _dev(posterior, torch.float32, "posterior", shape),
                                     _dev(smoothed, torch.float32, "smoothed", shape) if smoothed is not None else None,
                                     _dev(occ, torch.uint8, "occ", shape), _dev(out, torch.int32, "out"), cap,
                                     _dev(count, torch.int64, "count"), _dev(ws, torch.uint8, "workspace"),
                                     ws.numel(), _stream()))
        return Surface(occ, smoothed, out, count, cap)

    # ------------------------------------------------ particle weights
    def particle_weights(self, cylinders: torch.Tensor, silhouettes: Sequence[torch.Tensor],
                         edges: Sequence[torch.Tensor], beta: float = 1.0, weights: bool = True,
                         terms: bool = False, out=None):
        """log w of every particle (FP64 [np]) from its body-model cylinders
        (FP32 [np][10][8]: A xyz, B xyz, rA, rB) and each view's silhouette and
        edge maps (FP32 [H][W]); with `weights`, also w^beta normalised over the
        particles; with `terms`, the per-view (Sigma_e, Sigma_r) [np][n][2].
        Returns (log_w, weights or None, terms or None)."""
        nc = L.CYLINDERS
        if cylinders.dim() != 3 or tuple(cylinders.shape[1:]) != (nc, 8):
            raise ValueError(f"cylinders must have shape (np, {nc}, 8), got {tuple(cylinders.shape)}")
        npart = int(cylinders.shape[0])
        if len(silhouettes) != self.n or len(edges) != self.n:
            raise ValueError(f"expected {self.n} silhouette and edge maps")
        sil = L.ptr_array([_dev(m, torch.float32, f"silhouettes[{k}]", (c.height, c.width))
                           for k, (m, c) in enumerate(zip(silhouettes, self.cams))])
        edg = L.ptr_array([_dev(m, torch.float32, f"edges[{k}]", (c.height, c.width))
                           for k, (m, c) in enumerate(zip(edges, self.cams))])
        o = out or {}
        log_w = o.get("log_w")
        log_w = log_w if log_w is not None else torch.empty(npart, dtype=torch.float64, device="cuda")
        w = o.get("weights")
        w = w if w is not None or not weights else torch.empty(npart, dtype=torch.float64, device="cuda")
        t = o.get("terms")
        t = t if t is not None or not terms else torch.empty((npart, self.n, 2), dtype=torch.float64, device="cuda")
        L.check(L.lib().psfs_particle_weights(
            self._h, _dev(cylinders, torch.float32, "cylinders") if npart else None, npart, sil, edg, float(beta),
            _dev(log_w, torch.float64, "log_w", (npart,)) if npart else None,
            _dev(w, torch.float64, "weights", (npart,)) if (w is not None and npart) else None,
            _dev(t, torch.float64, "terms", (npart, self.n, 2)) if (t is not None and npart) else None,
            _stream()))
        return log_w, w, t

    # ------------------------------------- foreground model after frame 1
    def foreground_model(self, images: Sequence[torch.Tensor], masks=None, lmap: Optional[torch.Tensor] = None,
                         out: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Log density per colour bin learned from the foreground pixels of a
        frame: `masks` (u8 [H][W] per view, nonzero = foreground; None entries
        or masks=None use lmap > 0, i.e. SLM > 1/2 in that frame's maps)."""
        ims = self._images(images)
        mp = None
        if masks is not None:
            if len(masks) != self.n:
                raise ValueError(f"expected {self.n} masks, got {len(masks)}")
            mp = L.ptr_array([_dev(m, torch.uint8, f"masks[{k}]", (c.height, c.width)) if m is not None else None
                              for k, (m, c) in enumerate(zip(masks, self.cams))])
        out = out if out is not None else torch.empty(L.FG_BINS, dtype=torch.float32, device="cuda")
        ws = workspace if workspace is not None else torch.empty(4 * L.FG_BINS, dtype=torch.uint8, device="cuda")
        L.check(L.lib().psfs_foreground_model(self._h, ims, mp, self._map(lmap, 1, "lmap") if lmap is not None else None,
                                              _dev(out, torch.float32, "log_density", (L.FG_BINS,)),
                                              _dev(ws, torch.uint8, "workspace"), ws.numel(), _stream()))
        return out

    def set_foreground(self, log_density: Optional[torch.Tensor]) -> None:
        """Use a learned foreground model in the likelihood maps (None: uniform)."""
        ptr = _dev(log_density, torch.float32, "log_density", (L.FG_BINS,)) if log_density is not None else None
        L.check(L.lib().psfs_set_foreground(self._h, ptr))
        self._keep["fg"] = log_density

    # ---------------------------------------------------- voxel colour
    def colour_workspace_bytes(self) -> int:
        return int(L.lib().psfs_colour_workspace_bytes(self._h))

    def colour(self, images: Sequence[torch.Tensor], voxels: torch.Tensor, colour=None, views=None,
               workspace=None) -> Tuple[torch.Tensor, torch.Tensor]:
        """Mean RGB of each listed voxel over the views where it is the nearest
        listed voxel at its pixel, and the number of such views."""
        ims = self._images(images)
        n = int(voxels.numel())
        colour = colour if colour is not None else torch.empty((n, 3), dtype=torch.float32, device="cuda")
        views = views if views is not None else torch.empty(n, dtype=torch.int32, device="cuda")
        ws = workspace if workspace is not None else torch.empty(max(self.colour_workspace_bytes(), 8),
                                                                 dtype=torch.uint8, device="cuda")
        L.check(L.lib().psfs_colour(self._h, ims, _dev(voxels, torch.int32, "voxels") if n else None, n,
                                    _dev(colour, torch.float32, "colour", (n, 3)) if n else None,
                                    _dev(views, torch.int32, "views", (n,)) if n else None,
                                    _dev(ws, torch.uint8, "workspace"), ws.numel(), _stream()))
        return colour, views

    # ------------------------------------------- differentiable variant
    def diff_workspace_bytes(self) -> int:
        return int(L.lib().psfs_diff_workspace_bytes(self._h))

    def new_diff_workspace(self) -> torch.Tensor:
        n = max(self.diff_workspace_bytes(), 256)
        return torch.empty(n, dtype=torch.uint8, device="cuda")

    @staticmethod
    def _sub(sub):
        if sub is None:
            return None
        arr = (C.c_int32 * 6)(*[int(x) for x in sub])
        return arr

    def diff_forward(self, images, labels: torch.Tensor, sub=None, logits=None, loss=None, workspace=None):
        """Bilinear logits [nz][ny][nx] and mean BCE loss over `sub` (default:
        whole grid). Returns (logits, loss, workspace); keep the workspace
        untouched for diff_backward."""
        g = self.grid
        shape = (g.nz, g.ny, g.nx)
        ims = self._images(images)
        lab = _dev(labels, torch.uint8, "labels", shape)
        logits = logits if logits is not None else torch.empty(shape, dtype=torch.float32, device="cuda")
        loss = loss if loss is not None else torch.empty((), dtype=torch.float32, device="cuda")
        ws = workspace if workspace is not None else self.new_diff_workspace()
        L.check(L.lib().psfs_diff_forward(self._h, ims, lab, self._sub(sub), _dev(logits, torch.float32, "logits", shape),
                                          _dev(loss, torch.float32, "loss"), _dev(ws, torch.uint8, "workspace"),
                                          ws.numel(), _stream()))
        return logits, loss, ws

    def diff_backward(self, images, labels, logits, grad_loss: torch.Tensor, workspace, sub=None,
                      gmeans=None, gvars=None, gP=None):
        """Gradients of grad_loss * loss w.r.t. background means, variances
        (lists of [H][W][3]) and camera matrices ([n][3][4])."""
        g = self.grid
        shape = (g.nz, g.ny, g.nx)
        ims = self._images(images)
        gl = grad_loss.detach().to(device="cuda", dtype=torch.float32).contiguous().reshape(())
        gmeans = gmeans if gmeans is not None else [torch.empty((c.height, c.width, 3), dtype=torch.float32, device="cuda") for c in self.cams]
        gvars = gvars if gvars is not None else [torch.empty((c.height, c.width, 3), dtype=torch.float32, device="cuda") for c in self.cams]
        gP = gP if gP is not None else torch.empty((max(self.n, 1), 3, 4), dtype=torch.float32, device="cuda")
        gm_ptr = L.ptr_array([_dev(t, torch.float32, f"gmean[{k}]", (c.height, c.width, 3)) for k, (t, c) in enumerate(zip(gmeans, self.cams))])
        gv_ptr = L.ptr_array([_dev(t, torch.float32, f"gvar[{k}]", (c.height, c.width, 3)) for k, (t, c) in enumerate(zip(gvars, self.cams))])
        L.check(L.lib().psfs_diff_backward(self._h, ims, _dev(labels, torch.uint8, "labels", shape), self._sub(sub),
                                           _dev(logits, torch.float32, "logits", shape), gl.data_ptr(), gm_ptr, gv_ptr,
                                           _dev(gP, torch.float32, "gP"), _dev(workspace, torch.uint8, "workspace"),
                                           workspace.numel(), _stream()))
        self._keep["grad_loss"] = gl
        return gmeans, gvars, gP[: self.n]


class Surface:
    """Result of Plan.surface: occupancy, optional smoothed posterior, and
    the surface-voxel list (capacity-sized buffer + device count)."""

    def __init__(self, occ, smoothed, out, count, capacity):
        self.occ, self.smoothed, self.out, self.count, self.capacity = occ, smoothed, out, count, capacity

    def indices(self) -> torch.Tensor:
        """Ascending int32 linear indices (synchronises on the count)."""
        n = int(self.count.item())
        return self.out[:min(n, self.capacity)]


class Pipeline:
    """Frame sequence from one rig with one launch per frame: push(frame t+1)
    fuses frame t (pushed before) while computing the maps of frame t+1.

        pipe = Pipeline(plan)
        for images in frames:
            out = pipe.push(images)       # outputs of the previous frame, or None
        out = pipe.flush()                # outputs of the last frame
    """

    def __init__(self, plan: Plan, want_occ: bool = True):
        self.plan = plan
        self.want_occ = want_occ
        self._maps = [plan.new_lmap(), plan.new_lmap()]
        self._cur = -1                       # map buffer holding the pending frame

    def _outputs(self):
        g = self.plan.grid
        shape = (g.nz, g.ny, g.nx)
        post = torch.empty(shape, dtype=torch.float32, device="cuda")
        occ = torch.empty(shape, dtype=torch.uint8, device="cuda") if self.want_occ else None
        return post, occ

    def push(self, images, posterior=None, occ=None):
        nxt = 0 if self._cur != 0 else 1
        out = None
        if self._cur >= 0:
            if posterior is None:
                posterior, occ = self._outputs()
            out = (posterior, occ)
            self.plan.pipeline_step(images, self._maps[nxt], self._maps[self._cur], posterior, occ)
        else:
            self.plan.pipeline_step(images, self._maps[nxt])
        self._cur = nxt
        return out

    def flush(self, posterior=None, occ=None):
        if self._cur < 0:
            return None
        if posterior is None:
            posterior, occ = self._outputs()
        self.plan.pipeline_step(None, None, self._maps[self._cur], posterior, occ)
        self._cur = -1
        return posterior, occ


class BatchFrame:
    """One frame of a batch: cameras, grid, device images/background, outputs."""

    def __init__(self, cams, grid, images, means, vars_, posterior=None, occ=None, want_occ=True):
        self.cams, self.grid = list(cams), grid
        self.images, self.means, self.vars = list(images), list(means), list(vars_)
        shape = (grid.nz, grid.ny, grid.nx)
        self.posterior = posterior if posterior is not None else torch.empty(shape, dtype=torch.float32, device="cuda")
        self.occ = occ if occ is not None else (torch.empty(shape, dtype=torch.uint8, device="cuda") if want_occ else None)


class Batch:
    """Many frames of uneven shape in a chain of launches (each frame's
    likelihood beside the previous frame's fusion) replayed from a HIP graph
    (see psfs_batch_* in psfs.h)."""

    def __init__(self, frames: Sequence[BatchFrame], prior=0.5, log_u=LOG_U_DEFAULT, threshold=0.5,
                 sampling: int = L.NEAREST):
        self._params = L.psfs_params(float(prior), float(log_u), float(threshold), int(sampling))
        arr, keep = self._marshal(frames)
        h = C.c_void_p()
        L.check(L.lib().psfs_batch_create(C.byref(h), C.byref(self._params), len(frames), arr))
        self._h, self._keep, self.frames = h, keep, list(frames)
        self._destroy = L.lib().psfs_batch_destroy
        self.workspace = torch.empty(max(int(L.lib().psfs_batch_workspace_bytes(h)), 256), dtype=torch.uint8,
                                     device="cuda")

    @staticmethod
    def _marshal(frames):
        arr = (L.psfs_frame * len(frames))()
        keep = []
        for f, fr in enumerate(frames):
            n = len(fr.cams)
            cams = (L.psfs_camera * n)(*[make_camera(c.width, c.height, c.P) for c in fr.cams])
            ims = L.ptr_array([_dev(im, torch.uint8, f"frame {f} image {k}", (c.height, c.width, 3))
                               for k, (im, c) in enumerate(zip(fr.images, fr.cams))])
            mus = L.ptr_array([_dev(m, torch.float32, f"frame {f} mean {k}", (c.height, c.width, 3))
                               for k, (m, c) in enumerate(zip(fr.means, fr.cams))])
            vs = L.ptr_array([_dev(v, torch.float32, f"frame {f} var {k}", (c.height, c.width, 3))
                              for k, (v, c) in enumerate(zip(fr.vars, fr.cams))])
            g = fr.grid
            shape = (g.nz, g.ny, g.nx)
            arr[f].grid = make_grid(g.nx, g.ny, g.nz, g.origin, g.voxel)
            arr[f].n = n
            arr[f].cams = cams
            arr[f].images_dev = ims
            arr[f].mean_dev = mus
            arr[f].var_dev = vs
            arr[f].posterior_dev = _dev(fr.posterior, torch.float32, f"frame {f} posterior", shape)
            arr[f].occ_dev = _dev(fr.occ, torch.uint8, f"frame {f} occ", shape) if fr.occ is not None else None
            keep.append((cams, ims, mus, vs, fr))
        return arr, keep

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._destroy(h)
            self._h = None

    def run(self) -> None:
        L.check(L.lib().psfs_batch_run(self._h, self.workspace.data_ptr(), self.workspace.numel(), _stream()))

    def update(self, frames: Sequence[BatchFrame]) -> None:
        arr, keep = self._marshal(frames)
        L.check(L.lib().psfs_batch_update(self._h, len(frames), arr))
        self._keep, self.frames = keep, list(frames)

    def set_tile(self, tile: int) -> None:
        L.check(L.lib().psfs_batch_set_tile(self._h, int(tile)))

    @property
    def tile(self) -> int:
        return L.check(L.lib().psfs_batch_get_tile(self._h))

    def tune(self, force: bool = False) -> int:
        best = C.c_int32(-1)
        L.check(L.lib().psfs_batch_tune(self._h, self.workspace.data_ptr(), self.workspace.numel(), _stream(),
                                        int(force), C.byref(best)))
        return best.value


def tiles():
    n = L.lib().psfs_tile_count()
    out = []
    for t in range(n):
        a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
        L.check(L.lib().psfs_tile_describe(t, C.byref(a), C.byref(b), C.byref(c)))
        out.append((a.value, b.value, c.value))
    return out
