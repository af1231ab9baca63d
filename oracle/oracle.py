"""ctypes wrapper of the FP64 C oracle (``psfs_oracle.c``).

TEST INFRASTRUCTURE ONLY: used by ``tests/``, the smoke check and the
benchmark's CPU baseline. The product library never imports this package.

Cameras are any objects with ``width``, ``height`` and a 3x4 ``P``; a grid is
any object with ``nx, ny, nz, origin, voxel``. FP32 inputs are widened exactly
to FP64 here; nothing is rounded on the way in.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "psfs_oracle.c")
LIB = os.path.join(HERE, "libpsfs_oracle.so")

LOG_U_DEFAULT = -3.0 * np.log(256.0)      # uniform density over the 8-bit RGB cube
EPS_PX_DEFAULT = 1e-3                     # rounding-ambiguity band (pixels)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP over voxels)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        dp, ip, u8p, fp = (C.POINTER(C.c_double), C.POINTER(C.c_int32),
                           C.POINTER(C.c_uint8), C.POINTER(C.c_float))
        dpp = C.POINTER(dp)
        L.psfs_oracle_threads.restype = C.c_int
        L.psfs_oracle_set_threads.argtypes = [C.c_int]
        L.psfs_oracle_set_threads.restype = None
        L.psfs_oracle_slm.argtypes = [C.c_int64, u8p, fp, fp, C.c_double, dp]
        L.psfs_oracle_log2slm.argtypes = [C.c_int64, u8p, fp, fp, C.c_double, dp]
        L.psfs_oracle_fuse_views.argtypes = [C.c_int, dp, C.c_double]
        L.psfs_oracle_fuse_views.restype = C.c_double
        geo = [C.c_int, ip, ip, dp, C.c_int, C.c_int, C.c_int, dp, C.c_double, C.c_double]
        L.psfs_oracle_posterior.argtypes = geo + [dpp, C.c_double, dp, dp, dp, ip]
        L.psfs_oracle_voxel_combos.argtypes = geo + [dpp, C.c_double, C.c_int64, dp, C.c_int64]
        L.psfs_oracle_voxel_combos.restype = C.c_int64
        L.psfs_oracle_bilinear_logits.argtypes = geo + [dpp, dp]
        L.psfs_oracle_bce_loss.argtypes = [C.c_int, C.c_int, C.c_int, dp, u8p, ip]
        L.psfs_oracle_bce_loss.restype = C.c_double
        L.psfs_oracle_grad.argtypes = geo + [C.c_double, C.POINTER(u8p), C.POINTER(fp), C.POINTER(fp),
                                             u8p, ip, C.c_double, dpp, dpp, dp]
        _lib = L
    return _lib


def threads() -> int:
    return int(lib().psfs_oracle_threads())


def set_threads(n: int) -> None:
    """OpenMP threads of the later oracle calls (for timing)."""
    lib().psfs_oracle_set_threads(int(n))


# ----------------------------------------------------------------- marshalling

def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _ptr_array(arrs: Sequence[np.ndarray], ct):
    A = C.POINTER(ct) * max(len(arrs), 1)
    return A(*[_ptr(a, ct) for a in arrs])


def _widen_P(P) -> np.ndarray:
    # FP32 matrices (what the library takes) are widened exactly; an FP64
    # matrix is used as given (finite-difference tests perturb it in FP64).
    P = np.asarray(P)
    if P.dtype != np.float64:
        P = P.astype(np.float32).astype(np.float64)
    return P.reshape(12)


def _geom(cams, grid):
    n = len(cams)
    W = np.array([c.width for c in cams] or [0], np.int32)
    H = np.array([c.height for c in cams] or [0], np.int32)
    P = np.concatenate([_widen_P(c.P) for c in cams]) if n else np.zeros(12)
    P = np.ascontiguousarray(P)
    o = np.asarray(grid.origin, np.float32).astype(np.float64)
    keep = (W, H, P, o)
    args = [n, _ptr(W, C.c_int32), _ptr(H, C.c_int32), _ptr(P, C.c_double),
            int(grid.nx), int(grid.ny), int(grid.nz), _ptr(o, C.c_double), float(np.float32(grid.voxel))]
    return args, keep


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


# -------------------------------------------------------------------- the API

def slm(img, mean, var, log_u: float = LOG_U_DEFAULT) -> np.ndarray:
    """Eq. 1-2: SLM per pixel, FP64 [H][W]."""
    img, mean, var = _c(img, np.uint8), _c(mean, np.float32), _c(var, np.float32)
    shape = img.shape[:-1]
    out = np.empty(shape, np.float64)
    rc = lib().psfs_oracle_slm(int(np.prod(shape)), _ptr(img, C.c_uint8), _ptr(mean, C.c_float),
                               _ptr(var, C.c_float), float(log_u), _ptr(out, C.c_double))
    if rc:
        raise ValueError(f"oracle slm rejected its input (rc={rc})")
    return out


def log2slm(img, mean, var, log_u: float = LOG_U_DEFAULT) -> np.ndarray:
    """log(2*SLM) per pixel, FP64 [H][W]."""
    img, mean, var = _c(img, np.uint8), _c(mean, np.float32), _c(var, np.float32)
    shape = img.shape[:-1]
    out = np.empty(shape, np.float64)
    rc = lib().psfs_oracle_log2slm(int(np.prod(shape)), _ptr(img, C.c_uint8), _ptr(mean, C.c_float),
                                   _ptr(var, C.c_float), float(log_u), _ptr(out, C.c_double))
    if rc:
        raise ValueError(f"oracle log2slm rejected its input (rc={rc})")
    return out


def fuse_views(s: Sequence[float], prior: float = 0.5) -> float:
    """Eq. 3-9 for one voxel given its views' SLM values."""
    a = _c(np.asarray(s, np.float64).reshape(-1), np.float64)
    return float(lib().psfs_oracle_fuse_views(len(a), _ptr(a, C.c_double), float(prior)))


class Posterior:
    def __init__(self, post, lo, hi, ncombo):
        self.post, self.lo, self.hi, self.ncombo = post, lo, hi, ncombo

    @property
    def ambiguous(self) -> np.ndarray:
        return self.ncombo != 1


def posterior(cams, grid, slm_maps: Sequence[np.ndarray], prior: float = 0.5,
              eps_px: float = EPS_PX_DEFAULT) -> Posterior:
    """Eq. 3-9 for every voxel (nearest pixel), with the rounding-ambiguity bounds."""
    args, keep = _geom(cams, grid)
    maps = [_c(m, np.float64) for m in slm_maps]
    shape = (grid.nz, grid.ny, grid.nx)
    post, lo, hi = (np.empty(shape, np.float64) for _ in range(3))
    nc = np.empty(shape, np.int32)
    rc = lib().psfs_oracle_posterior(*args, float(prior), _ptr_array(maps, C.c_double), float(eps_px),
                                     _ptr(post, C.c_double), _ptr(lo, C.c_double), _ptr(hi, C.c_double),
                                     _ptr(nc, C.c_int32))
    if rc:
        raise ValueError(f"oracle posterior rejected its input (rc={rc})")
    return Posterior(post, lo, hi, nc)


def voxel_combos(cams, grid, slm_maps, voxel: int, prior: float = 0.5,
                 eps_px: float = EPS_PX_DEFAULT, max_out: int = 4096) -> np.ndarray:
    """All posteriors one voxel can take over its admissible pixel choices."""
    args, keep = _geom(cams, grid)
    maps = [_c(m, np.float64) for m in slm_maps]
    out = np.empty(max_out, np.float64)
    cnt = lib().psfs_oracle_voxel_combos(*args, float(prior), _ptr_array(maps, C.c_double),
                                         float(eps_px), int(voxel), _ptr(out, C.c_double), max_out)
    if cnt < 0:
        raise ValueError("oracle voxel_combos rejected its input")
    return out[:min(cnt, max_out)].copy()


def bilinear_logits(cams, grid, l2s_maps: Sequence[np.ndarray], prior: float = 0.5) -> np.ndarray:
    """Logits with bilinear sampling of log(2*SLM), FP64 [nz][ny][nx]."""
    args, keep = _geom(cams, grid)
    maps = [_c(m, np.float64) for m in l2s_maps]
    L = np.empty((grid.nz, grid.ny, grid.nx), np.float64)
    rc = lib().psfs_oracle_bilinear_logits(*args, float(prior), _ptr_array(maps, C.c_double),
                                           _ptr(L, C.c_double))
    if rc:
        raise ValueError(f"oracle bilinear_logits rejected its input (rc={rc})")
    return L


def _sub(sub):
    return None if sub is None else _c(np.asarray(sub, np.int32).reshape(6), np.int32)


def bce_loss(L: np.ndarray, labels: np.ndarray, sub=None) -> float:
    L, labels = _c(L, np.float64), _c(labels, np.uint8)
    nz, ny, nx = L.shape
    s = _sub(sub)
    return float(lib().psfs_oracle_bce_loss(nx, ny, nz, _ptr(L, C.c_double), _ptr(labels, C.c_uint8),
                                            None if s is None else _ptr(s, C.c_int32)))


def loss(cams, grid, images, means, vars_, labels, sub=None, prior=0.5, log_u=LOG_U_DEFAULT) -> float:
    """Forward of the differentiable variant: BCE of the bilinear logits."""
    l2s = [log2slm(i, m, v, log_u) for i, m, v in zip(images, means, vars_)]
    return bce_loss(bilinear_logits(cams, grid, l2s, prior), labels, sub)


def grad(cams, grid, images, means, vars_, labels, sub=None, prior=0.5, log_u=LOG_U_DEFAULT,
         grad_loss: float = 1.0):
    """Analytic gradient of grad_loss*loss w.r.t. (means, vars, P): FP64."""
    args, keep = _geom(cams, grid)
    imgs = [_c(i, np.uint8) for i in images]
    mus = [_c(m, np.float32) for m in means]
    vs = [_c(v, np.float32) for v in vars_]
    gm = [np.empty(m.shape, np.float64) for m in mus]
    gv = [np.empty(v.shape, np.float64) for v in vs]
    gP = np.empty((max(len(cams), 1), 12), np.float64)
    lab = _c(labels, np.uint8)
    s = _sub(sub)
    rc = lib().psfs_oracle_grad(*args, float(prior), float(log_u), _ptr_array(imgs, C.c_uint8),
                                _ptr_array(mus, C.c_float), _ptr_array(vs, C.c_float),
                                _ptr(lab, C.c_uint8), None if s is None else _ptr(s, C.c_int32),
                                float(grad_loss), _ptr_array(gm, C.c_double), _ptr_array(gv, C.c_double),
                                _ptr(gP, C.c_double))
    if rc:
        raise ValueError(f"oracle grad rejected its input (rc={rc})")
    return gm, gv, gP[:len(cams)].reshape(len(cams), 3, 4)


def reconstruct(cams, grid, images, means, vars_, prior=0.5, log_u=LOG_U_DEFAULT,
                eps_px=EPS_PX_DEFAULT, threshold=0.5):
    """Whole forward pass: SLM maps, posterior with ambiguity bounds, occupancy."""
    maps = [slm(i, m, v, log_u) for i, m, v in zip(images, means, vars_)]
    post = posterior(cams, grid, maps, prior, eps_px)
    occ = (post.post > threshold).astype(np.uint8)
    return maps, post, occ
