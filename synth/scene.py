"""Seeded synthetic multi-view scenes: the inputs of the occupancy pass.

This module only *produces inputs* (cameras, voxel grids, background models,
images, ground-truth occupancy). It holds none of the occupancy method's
arithmetic (no silhouette likelihood, no projection-and-fusion, no posterior),
so the FP64 reference in ``oracle/`` and the HIP path can both consume it
without sharing any of the method.

Scene recipe (stand-in for the paper's multi-camera recordings, Sec. 3.4, whose
grid is at most 150x150x100 samples seen by 8 cameras, Sec. 3.3.3):

* Rig: pinhole cameras on a ring of radius 4 m at height 1.5 m looking at the
  origin with world up +z; optionally 4 more at 3 m height. Intrinsics
  ``K = [[f,0,W/2],[0,f,H/2],[0,0,1]]``, rotation rows (right, down, forward),
  ``P = K [R | -R C]`` (FP32, row-major 3x4, metres -> pixels). Pixel centres
  sit at integer image coordinates.
* Body: a union of 10 ellipsoids, one per body part of the paper's 10-part
  skeleton (Table 1), with seeded jitter of centre, semi-axes and orientation.
* Silhouettes: exact FP64 ray/ellipsoid test through every integer pixel
  centre.
* Background model: per pixel and channel, mean ~ U(0,255), std ~ U(5,15),
  variance = std^2, stored FP32.
* Images (u8 RGB, [H][W][3]): background pixels = clip(round(mean + std*N(0,1)));
  foreground pixels = clip(round(U(0,255) + N(0,10))); 2 % of pixels are
  salt-and-pepper outliers, (0,0,0) or (255,255,255) with equal odds.
* Seeds: ``numpy.random.default_rng([config, frame, stream])`` with one stream
  per purpose (body, background, noise, outliers, foreground, perturbation,
  shape draws).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

STREAM_BODY = 0
STREAM_BG = 1
STREAM_NOISE = 2
STREAM_OUTLIER = 3
STREAM_FG = 4
STREAM_PERTURB = 5
STREAM_SHAPE = 6

# (focal length in px, width, height) of the three image classes.
IMAGE_CLASSES = ((300.0, 320, 240), (600.0, 640, 480), (1000.0, 1280, 720))

# The 10 body parts of the paper's skeleton (Table 1) as ellipsoids:
# name, centre (m), semi-axes (m), before jitter.
BODY_PARTS = (
    ("torso", (0.0, 0.0, 0.25), (0.18, 0.12, 0.30)),
    ("head", (0.0, 0.0, 0.72), (0.10, 0.10, 0.12)),
    ("left_thigh", (0.0, 0.10, -0.27), (0.08, 0.08, 0.22)),
    ("right_thigh", (0.0, -0.10, -0.27), (0.08, 0.08, 0.22)),
    ("left_calf", (0.0, 0.10, -0.65), (0.06, 0.06, 0.20)),
    ("right_calf", (0.0, -0.10, -0.65), (0.06, 0.06, 0.20)),
    ("left_upper_arm", (0.0, 0.25, 0.38), (0.05, 0.05, 0.16)),
    ("right_upper_arm", (0.0, -0.25, 0.38), (0.05, 0.05, 0.16)),
    ("left_lower_arm", (0.0, 0.27, 0.08), (0.05, 0.05, 0.15)),
    ("right_lower_arm", (0.0, -0.27, 0.08), (0.05, 0.05, 0.15)),
)


def rng_for(config: int, frame: int, stream: int, *more: int) -> np.random.Generator:
    return np.random.default_rng([int(config), int(frame), int(stream)] + [int(m) for m in more])


@dataclass
class Camera:
    width: int
    height: int
    P: np.ndarray                      # float32 (3, 4), row-major, metres -> px
    K: Optional[np.ndarray] = None     # float64 (3, 3), rendering only
    R: Optional[np.ndarray] = None     # float64 (3, 3), rows right/down/forward
    C: Optional[np.ndarray] = None     # float64 (3,), camera centre

    def with_P(self, P: np.ndarray) -> "Camera":
        return Camera(self.width, self.height, np.asarray(P, np.float32).reshape(3, 4).copy(),
                      self.K, self.R, self.C)


@dataclass
class Grid:
    nx: int
    ny: int
    nz: int
    origin: np.ndarray                 # float32 (3,): corner of voxel (0,0,0)
    voxel: np.float32                  # edge length (m)

    @property
    def nvox(self) -> int:
        return self.nx * self.ny * self.nz

    def centres64(self, i=None, j=None, k=None):
        """Voxel centres in FP64, widened from the FP32 origin and edge."""
        o = self.origin.astype(np.float64)
        h = float(self.voxel)
        i = np.arange(self.nx) if i is None else np.asarray(i)
        j = np.arange(self.ny) if j is None else np.asarray(j)
        k = np.arange(self.nz) if k is None else np.asarray(k)
        return o[0] + h * (i + 0.5), o[1] + h * (j + 0.5), o[2] + h * (k + 0.5)


@dataclass
class Ellipsoid:
    centre: np.ndarray                 # (3,)
    axes: np.ndarray                   # (3,) semi-axes
    rot: np.ndarray                    # (3, 3), columns = local axes in world


@dataclass
class Frame:
    config: int
    frame: int
    cams: List[Camera]
    grid: Grid
    images: List[np.ndarray]           # u8 [H][W][3] per camera
    mean: List[np.ndarray]             # float32 [H][W][3]
    var: List[np.ndarray]              # float32 [H][W][3]
    masks: List[np.ndarray] = field(default_factory=list)   # bool [H][W]
    body: List[Ellipsoid] = field(default_factory=list)

    @property
    def n(self) -> int:
        return len(self.cams)

    @property
    def npix(self) -> int:
        return sum(c.width * c.height for c in self.cams)


# --------------------------------------------------------------------------- rig

def look_at_camera(C: Sequence[float], f: float, W: int, H: int,
                   target=(0.0, 0.0, 0.0), up=(0.0, 0.0, 1.0)) -> Camera:
    C = np.asarray(C, np.float64)
    fwd = np.asarray(target, np.float64) - C
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.asarray(up, np.float64))
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd])
    K = np.array([[f, 0.0, W / 2.0], [0.0, f, H / 2.0], [0.0, 0.0, 1.0]])
    P = K @ np.concatenate([R, (-R @ C)[:, None]], axis=1)
    return Camera(int(W), int(H), P.astype(np.float32), K, R, C)


def ring_rig(n: int, f: float, W: int, H: int, radius: float = 4.0,
             height: float = 1.5, phase: float = 0.0) -> List[Camera]:
    cams = []
    for k in range(n):
        th = phase + 2.0 * np.pi * k / n
        cams.append(look_at_camera((radius * np.cos(th), radius * np.sin(th), height), f, W, H))
    return cams


def ring_plus_elevated_rig(f: float, W: int, H: int) -> List[Camera]:
    cams = ring_rig(8, f, W, H)
    for k in range(4):
        th = np.pi / 4 + k * np.pi / 2
        cams.append(look_at_camera((4.0 * np.cos(th), 4.0 * np.sin(th), 3.0), f, W, H))
    return cams


def cube_grid(edge: int, side: float) -> Grid:
    h = np.float32(side / edge)
    o = np.full(3, -side / 2.0, np.float32)
    return Grid(int(edge), int(edge), int(edge), o, h)


# -------------------------------------------------------------------------- body

def _axis_angle(axis: np.ndarray, ang: float) -> np.ndarray:
    a = axis / np.linalg.norm(axis)
    Kx = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + np.sin(ang) * Kx + (1 - np.cos(ang)) * (Kx @ Kx)


def make_body(rng: np.random.Generator, shift=(0.0, 0.0, 0.0)) -> List[Ellipsoid]:
    parts = []
    for _, c, ax in BODY_PARTS:
        centre = np.asarray(c) + rng.normal(0.0, 0.02, 3) + np.asarray(shift, np.float64)
        axes = np.clip(np.asarray(ax) * rng.uniform(0.9, 1.1, 3), 0.05, 0.30)
        axis = rng.normal(size=3)
        ang = np.deg2rad(rng.uniform(0.0, 15.0))
        parts.append(Ellipsoid(centre, axes, _axis_angle(axis, ang)))
    return parts


def _ellipsoid_bbox(cam: Camera, e: Ellipsoid):
    """Pixel box containing the ellipsoid's image: the projection of a convex
    set in front of the camera lies in the hull of its bounding cube's
    projected corners. None if the cube is not wholly in front."""
    R = float(np.max(e.axes))
    corners = e.centre + R * np.array([[sx, sy, sz] for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)])
    xc = (corners - cam.C) @ cam.R.T
    if np.any(xc[:, 2] <= 1e-9):
        return None
    u = cam.K[0, 0] * xc[:, 0] / xc[:, 2] + cam.K[0, 2]
    v = cam.K[1, 1] * xc[:, 1] / xc[:, 2] + cam.K[1, 2]
    x0, x1 = int(np.floor(u.min())) - 1, int(np.ceil(u.max())) + 2
    y0, y1 = int(np.floor(v.min())) - 1, int(np.ceil(v.max())) + 2
    return max(x0, 0), min(x1, cam.width), max(y0, 0), min(y1, cam.height)


def render_mask(cam: Camera, body: Sequence[Ellipsoid]) -> np.ndarray:
    """Exact FP64 silhouette: rays through integer pixel centres vs ellipsoids."""
    W, H = cam.width, cam.height
    mask = np.zeros((H, W), bool)
    f, cx, cy = cam.K[0, 0], cam.K[0, 2], cam.K[1, 2]
    for e in body:
        box = _ellipsoid_bbox(cam, e)
        x0, x1, y0, y1 = (0, W, 0, H) if box is None else box
        if x0 >= x1 or y0 >= y1:
            continue
        x, y = np.meshgrid(np.arange(x0, x1, dtype=np.float64), np.arange(y0, y1, dtype=np.float64))
        dc = np.stack([(x - cx) / f, (y - cy) / cam.K[1, 1], np.ones_like(x)], axis=-1)
        d = dc @ cam.R                # world ray directions, R^T applied row-wise
        M = e.rot.T / e.axes[:, None]  # world -> unit-sphere frame (linear part)
        c0 = M @ (cam.C - e.centre)
        dd = d @ M.T
        A = np.einsum("hwk,hwk->hw", dd, dd)
        B = dd @ c0
        Cc = c0 @ c0 - 1.0
        mask[y0:y1, x0:x1] |= (B * B - A * Cc >= 0.0) & (B < 0.0)
    return mask


def gt_occupancy(grid: Grid, body: Sequence[Ellipsoid]) -> np.ndarray:
    """u8 [nz][ny][nx]: 1 where the voxel centre lies inside any ellipsoid."""
    xs, ys, zs = grid.centres64()
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    P = np.stack([X, Y, Z], axis=-1)
    occ = np.zeros(X.shape, bool)
    for e in body:
        M = e.rot.T / e.axes[:, None]
        q = (P - e.centre) @ M.T
        occ |= np.einsum("...k,...k->...", q, q) <= 1.0
    return occ.astype(np.uint8)


# ------------------------------------------------------------- background/images

def make_background(rng: np.random.Generator, H: int, W: int):
    mean = 255.0 * rng.random((H, W, 3), dtype=np.float32)
    std = 5.0 + 10.0 * rng.random((H, W, 3), dtype=np.float32)
    return mean.astype(np.float32), (std * std).astype(np.float32)


def render_image(mask: np.ndarray, mean: np.ndarray, var: np.ndarray,
                 rng_noise: np.random.Generator, rng_fg: np.random.Generator,
                 rng_out: np.random.Generator, outlier_rate: float = 0.02) -> np.ndarray:
    H, W = mask.shape
    std = np.sqrt(var)
    bg = np.clip(np.round(mean + std * rng_noise.standard_normal((H, W, 3), dtype=np.float32)), 0, 255)
    fg = np.clip(np.round(255.0 * rng_fg.random((H, W, 3), dtype=np.float32)
                          + 10.0 * rng_fg.standard_normal((H, W, 3), dtype=np.float32)), 0, 255)
    img = np.where(mask[..., None], fg, bg)
    hit = rng_out.random((H, W), dtype=np.float32) < outlier_rate
    white = rng_out.random((H, W), dtype=np.float32) < 0.5
    img[hit & white] = 255.0
    img[hit & ~white] = 0.0
    return img.astype(np.uint8)


def render_frame(config: int, frame: int, cams: List[Camera], grid: Grid,
                 body: List[Ellipsoid], bg_key: Tuple[int, int], seq: Tuple[int, ...] = ()) -> Frame:
    """Images of `body` seen by `cams` against the background model of
    `bg_key`; image noise is seeded by (config, frame) and, for the later
    frames of a sequence, by `seq` as well."""
    images, means, vars_, masks = [], [], [], []
    rbg = rng_for(bg_key[0], bg_key[1], STREAM_BG)
    rn = rng_for(config, frame, STREAM_NOISE, *seq)
    rf = rng_for(config, frame, STREAM_FG, *seq)
    ro = rng_for(config, frame, STREAM_OUTLIER, *seq)
    for cam in cams:
        m, v = make_background(rbg, cam.height, cam.width)
        mask = render_mask(cam, body)
        images.append(render_image(mask, m, v, rn, rf, ro))
        means.append(m)
        vars_.append(v)
        masks.append(mask)
    return Frame(config, frame, list(cams), grid, images, means, vars_, masks, list(body))


# ------------------------------------------------------------------ the configs

CONFIG_DOC = {
    0: "64^3 grid over 2 m, 4 ring cameras, 320x240, f=300",
    1: "128^3 grid over 2 m, 8 ring cameras, 640x480, f=600",
    2: "256^3 grid over 2.5 m, 8 ring + 4 elevated cameras, 1280x720, f=1000, 16 frames moving +2 cm/frame",
    3: "64 uneven frames: edge in {64,96,128,192}, 4..12 ring cameras, image class in 3 sizes",
    4: "config 1 scene, bilinear sampling, BCE loss vs ellipsoid occupancy, cameras perturbed 1 %",
}


def batch_shape(frame: int):
    """Shape draws of the 64-frame uneven batch: (edge, n_cams, image class)."""
    r = rng_for(3, frame, STREAM_SHAPE)
    edge = int(r.choice([64, 96, 128, 192]))
    n = int(r.integers(4, 13))
    cls = int(r.integers(0, 3))
    return edge, n, cls


def config_frame(config: int, frame: int = 0) -> Frame:
    """One frame of a named workload (see ``CONFIG_DOC``)."""
    if config == 0:
        f, W, H = IMAGE_CLASSES[0]
        cams, grid = ring_rig(4, f, W, H), cube_grid(64, 2.0)
    elif config in (1, 4):
        f, W, H = IMAGE_CLASSES[1]
        cams, grid = ring_rig(8, f, W, H), cube_grid(128, 2.0)
    elif config == 2:
        f, W, H = IMAGE_CLASSES[2]
        cams, grid = ring_plus_elevated_rig(f, W, H), cube_grid(256, 2.5)
    elif config == 3:
        edge, n, cls = batch_shape(frame)
        f, W, H = IMAGE_CLASSES[cls]
        cams, grid = ring_rig(n, f, W, H), cube_grid(edge, 2.0)
    else:
        raise ValueError(f"unknown config {config}")

    if config == 2:
        body = make_body(rng_for(2, 0, STREAM_BODY), shift=(0.02 * frame, 0.0, 0.0))
        bg_key = (2, 0)                 # one background model per rig
    elif config == 4:
        body = make_body(rng_for(1, frame, STREAM_BODY))
        bg_key = (1, frame)
    else:
        body = make_body(rng_for(config, frame, STREAM_BODY))
        bg_key = (config, frame)
    src_cfg = 1 if config == 4 else config
    fr = render_frame(src_cfg, frame, cams, grid, body, bg_key)
    fr.config = config
    return fr


def sequence_frame(config: int, slot: int, t: int) -> Frame:
    """Frame t of the frame sequence that starts with config_frame(config, slot):
    the same rig, grid and background model, the slot's body moved rigidly by
    +2 cm along x per frame, and fresh image noise (t = 0 is that frame).
    The 256^3 workload is already one sequence (config_frame(2, t))."""
    if config == 2:
        return config_frame(2, slot + t)
    if config not in (0, 1):
        raise ValueError(f"no frame sequence for config {config}")
    if t == 0:
        return config_frame(config, slot)
    fr0 = config_frame_rig(config)
    body = make_body(rng_for(config, slot, STREAM_BODY), shift=(0.02 * t, 0.0, 0.0))
    fr = render_frame(config, slot, fr0[0], fr0[1], body, (config, slot), seq=(t,))
    return fr


def config_frame_rig(config: int):
    """(cameras, grid) of a named workload with one rig (configs 0, 1, 2, 4)."""
    if config == 0:
        f, W, H = IMAGE_CLASSES[0]
        return ring_rig(4, f, W, H), cube_grid(64, 2.0)
    if config in (1, 4):
        f, W, H = IMAGE_CLASSES[1]
        return ring_rig(8, f, W, H), cube_grid(128, 2.0)
    if config == 2:
        f, W, H = IMAGE_CLASSES[2]
        return ring_plus_elevated_rig(f, W, H), cube_grid(256, 2.5)
    raise ValueError(f"config {config} has no single rig")


def perturb_cameras(cams: Sequence[Camera], seed=(4, 0), rel: float = 0.01) -> List[Camera]:
    """Multiply every entry of every P by (1 + rel*eps), eps ~ N(0,1), seeded."""
    r = rng_for(seed[0], seed[1], STREAM_PERTURB)
    out = []
    for c in cams:
        eps = r.normal(size=(3, 4))
        out.append(c.with_P(c.P.astype(np.float64) * (1.0 + rel * eps)))
    return out


def fd_subgrid(grid: Grid, body: Sequence[Ellipsoid], size: int = 16):
    """[i0,i1,j0,j1,k0,k1) of the size^3 block centred on the voxel nearest the torso centre."""
    t = body[0].centre
    xs, ys, zs = grid.centres64()
    c = [int(np.argmin(np.abs(a - t[d]))) for d, a in enumerate((xs, ys, zs))]
    dims = (grid.nx, grid.ny, grid.nz)
    lo = [min(max(c[d] - size // 2, 0), max(dims[d] - size, 0)) for d in range(3)]
    hi = [min(lo[d] + size, dims[d]) for d in range(3)]
    return [lo[0], hi[0], lo[1], hi[1], lo[2], hi[2]]


# ------------------------------------------------------ tracking: particles/maps

STREAM_PARTICLE = 7


def body_cylinders(body: Sequence[Ellipsoid]) -> np.ndarray:
    """FP64 [10][8] cylinders (A xyz, B xyz, rA, rB) of a body: each part's axis
    is its ellipsoid's longest semi-axis, its radius the geometric mean of the
    other two; limbs taper to 0.8 of that radius at their far end."""
    out = np.zeros((len(body), 8))
    for i, e in enumerate(body):
        a = int(np.argmax(e.axes))
        d = e.rot[:, a] * e.axes[a]
        others = [e.axes[b] for b in range(3) if b != a]
        r = float(np.sqrt(others[0] * others[1]))
        out[i, 0:3] = e.centre - d
        out[i, 3:6] = e.centre + d
        out[i, 6] = r
        out[i, 7] = r if i < 2 else 0.8 * r
    return out


def make_particles(rng: np.random.Generator, base: np.ndarray, n: int,
                   sd_shift: float = 0.03, sd_end: float = 0.02, rad_jitter: float = 0.1) -> np.ndarray:
    """FP32 [n][10][8]: the base cylinders moved as a whole by N(0, sd_shift) per
    axis, each end point by N(0, sd_end), radii scaled by U(1 -+ rad_jitter)."""
    base = np.asarray(base, np.float64)
    p = np.repeat(base[None], n, axis=0)
    shift = rng.normal(0.0, sd_shift, (n, 1, 3))
    p[..., 0:3] += shift + rng.normal(0.0, sd_end, (n, base.shape[0], 3))
    p[..., 3:6] += shift + rng.normal(0.0, sd_end, (n, base.shape[0], 3))
    p[..., 6:8] *= rng.uniform(1.0 - rad_jitter, 1.0 + rad_jitter, (n, base.shape[0], 2))
    return p.astype(np.float32)


def _dilate(b: np.ndarray) -> np.ndarray:
    """8-neighbour binary dilation with the border treated as 0."""
    pad = np.pad(b, 1)
    H, W = b.shape
    out = np.zeros_like(b)
    for dy in (0, 1, 2):
        for dx in (0, 1, 2):
            out |= pad[dy:dy + H, dx:dx + W]
    return out


def track_maps(mask: np.ndarray):
    """Silhouette and edge maps (FP32 [H][W] in [0,1]) of one view's mask:
    silhouette = the mask; edge = 1 on mask pixels with a 4-neighbour outside
    the mask or the image, 2/3 within one pixel of those (8-neighbourhood), 1/3
    within two, 0 elsewhere."""
    m = np.asarray(mask, bool)
    pad = np.pad(m, 1)
    H, W = m.shape
    inner = pad[0:H, 1:W + 1] & pad[2:H + 2, 1:W + 1] & pad[1:H + 1, 0:W] & pad[1:H + 1, 2:W + 2]
    b0 = m & ~inner
    b1 = _dilate(b0)
    b2 = _dilate(b1)
    edge = np.where(b0, 1.0, np.where(b1, 2.0 / 3.0, np.where(b2, 1.0 / 3.0, 0.0)))
    return m.astype(np.float32), edge.astype(np.float32)


def tracking_inputs(config: int = 1, frame: int = 0, n_particles: int = 200):
    """Cameras, FP32 particle cylinders [n][10][8], silhouette and edge maps of
    a workload's frame: the particles scatter around the cylinders of the
    frame's body, the maps come from its ground-truth masks."""
    fr = config_frame(config, frame)
    base = body_cylinders(fr.body)
    parts = make_particles(rng_for(config, frame, STREAM_PARTICLE), base, n_particles)
    S, E = zip(*(track_maps(m) for m in fr.masks))
    return fr.cams, parts, list(S), list(E)
