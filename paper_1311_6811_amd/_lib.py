"""ctypes loader of libpsfs.so and the C structs of psfs.h.

Loading fails loudly when the library has not been built: there is no
fallback implementation of any step.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libpsfs.so")

MAX_VIEWS = 16
FG_BINS = 4096
STATIC_SCRATCH_BYTES = 48 << 20          # PSFS_STATIC_SCRATCH_BYTES
CYLINDERS = 10
NEAREST, BILINEAR = 0, 1

STATUS = {
    0: "PSFS_OK", -1: "PSFS_E_ARG", -2: "PSFS_E_RANGE", -3: "PSFS_E_NOT_READY",
    -4: "PSFS_E_WORKSPACE", -5: "PSFS_E_HIP", -6: "PSFS_E_DEVICE", -7: "PSFS_E_STALE", -8: "PSFS_E_INPUT",
}


class psfs_camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("P", C.c_float * 12)]


class psfs_grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("origin", C.c_float * 3), ("voxel", C.c_float)]


class psfs_params(C.Structure):
    _fields_ = [("prior", C.c_float), ("log_u", C.c_float), ("threshold", C.c_float),
                ("sampling", C.c_int32)]


class psfs_frame(C.Structure):
    _fields_ = [("grid", psfs_grid), ("n", C.c_int32), ("cams", C.POINTER(psfs_camera)),
                ("images_dev", C.POINTER(C.c_void_p)), ("mean_dev", C.POINTER(C.c_void_p)),
                ("var_dev", C.POINTER(C.c_void_p)), ("posterior_dev", C.c_void_p), ("occ_dev", C.c_void_p)]


class PsfsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None

vp = C.c_void_p
i32p = C.POINTER(C.c_int32)

# name -> (restype, argtypes); mirrors include/psfs.h
SIGNATURES = {
    "psfs_version": (C.c_int, []),
    "psfs_status_str": (C.c_char_p, [C.c_int]),
    "psfs_last_error": (C.c_char_p, []),
    "psfs_default_params": (None, [C.POINTER(psfs_params)]),
    "psfs_plan_create": (C.c_int, [C.POINTER(vp)]),
    "psfs_plan_destroy": (None, [vp]),
    "psfs_set_cameras": (C.c_int, [vp, C.c_int, C.POINTER(psfs_camera)]),
    "psfs_set_grid": (C.c_int, [vp, C.POINTER(psfs_grid)]),
    "psfs_set_params": (C.c_int, [vp, C.POINTER(psfs_params)]),
    "psfs_set_background": (C.c_int, [vp, C.c_int, vp, vp]),
    "psfs_set_input_check": (C.c_int, [vp, vp]),
    "psfs_input_status": (C.c_int, [vp]),
    "psfs_lmap_floats": (C.c_int64, [vp]),
    "psfs_lmap_offset": (C.c_int64, [vp, C.c_int]),
    "psfs_workspace_bytes": (C.c_size_t, [vp]),
    "psfs_likelihood": (C.c_int, [vp, C.POINTER(vp), vp, vp]),
    "psfs_fuse": (C.c_int, [vp, vp, vp, vp, vp]),
    "psfs_reconstruct": (C.c_int, [vp, C.POINTER(vp), vp, vp, vp, C.c_size_t, vp]),
    "psfs_reconstruct_static": (C.c_int, [vp, C.POINTER(vp), vp, vp, vp]),
    "psfs_pipeline_step": (C.c_int, [vp, C.POINTER(vp), vp, vp, vp, vp, vp]),
    "psfs_pipeline_step_pair": (C.c_int, [vp, C.POINTER(vp), C.POINTER(vp), vp, vp, vp, vp, vp, vp, vp]),
    "psfs_pipeline_step_quad": (C.c_int, [vp, C.POINTER(vp), vp, vp, C.POINTER(vp), C.POINTER(vp), vp]),
    "psfs_surface_workspace_bytes": (C.c_size_t, [vp]),
    "psfs_colour_workspace_bytes": (C.c_size_t, [vp]),
    "psfs_foreground_model": (C.c_int, [vp, C.POINTER(vp), C.POINTER(vp), vp, vp, vp, C.c_size_t, vp]),
    "psfs_set_foreground": (C.c_int, [vp, vp]),
    "psfs_colour": (C.c_int, [vp, C.POINTER(vp), vp, C.c_int64, vp, vp, vp, C.c_size_t, vp]),
    "psfs_particle_weights": (C.c_int, [vp, vp, C.c_int64, C.POINTER(vp), C.POINTER(vp), C.c_double, vp, vp, vp, vp]),
    "psfs_surface": (C.c_int, [vp, vp, vp, vp, vp, C.c_int64, vp, vp, C.c_size_t, vp]),
    "psfs_threshold": (C.c_int, [vp, C.c_int64, C.c_float, vp, vp]),
    "psfs_diff_workspace_bytes": (C.c_size_t, [vp]),
    "psfs_diff_forward": (C.c_int, [vp, C.POINTER(vp), vp, i32p, vp, vp, vp, C.c_size_t, vp]),
    "psfs_diff_backward": (C.c_int, [vp, C.POINTER(vp), vp, i32p, vp, vp, C.POINTER(vp), C.POINTER(vp), vp, vp,
                                     C.c_size_t, vp]),
    "psfs_batch_create": (C.c_int, [C.POINTER(vp), C.POINTER(psfs_params), C.c_int, C.POINTER(psfs_frame)]),
    "psfs_batch_workspace_bytes": (C.c_size_t, [vp]),
    "psfs_batch_run": (C.c_int, [vp, vp, C.c_size_t, vp]),
    "psfs_batch_update": (C.c_int, [vp, C.c_int, C.POINTER(psfs_frame)]),
    "psfs_batch_destroy": (None, [vp]),
    "psfs_batch_set_tile": (C.c_int, [vp, C.c_int]),
    "psfs_batch_get_tile": (C.c_int, [vp]),
    "psfs_batch_tune": (C.c_int, [vp, vp, C.c_size_t, vp, C.c_int, i32p]),
    "psfs_tile_count": (C.c_int, []),
    "psfs_tile_describe": (C.c_int, [C.c_int, i32p, i32p, i32p]),
    "psfs_set_tile": (C.c_int, [vp, C.c_int]),
    "psfs_get_tile": (C.c_int, [vp]),
    "psfs_tune_workspace_bytes": (C.c_size_t, [vp]),
    "psfs_tune": (C.c_int, [vp, C.POINTER(vp), vp, C.c_size_t, vp, C.c_int, i32p]),
}


def lib():
    """The loaded library; raises if it was never built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libpsfs.so not built at {LIB_PATH}; run `python -m paper_1311_6811_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(status: int) -> int:
    if status < 0:
        raise PsfsError(status, lib().psfs_last_error().decode())
    return status


def ptr_array(ptrs):
    arr = (vp * max(len(ptrs), 1))()
    for i, p in enumerate(ptrs):
        arr[i] = p
    return arr
