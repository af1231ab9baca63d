"""MI355X (gfx950) probabilistic shape-from-silhouette occupancy library.

The compute lives in ``libpsfs.so`` (HIP kernels behind the C ABI of
``include/psfs.h``); this package is its thin binding. Importing it does not
load the library; the first call does, and raises if it was never built.
"""
from ._lib import BILINEAR, MAX_VIEWS, NEAREST, PsfsError, lib  # noqa: F401
from .api import LOG_U_DEFAULT, Batch, BatchFrame, Pipeline, Plan, Surface, make_camera, make_grid, threshold, tiles  # noqa: F401
from .autograd import DiffPlan, OccupancyLoss, occupancy_loss  # noqa: F401

__all__ = ["Plan", "Pipeline", "Surface", "Batch", "BatchFrame", "threshold", "tiles", "PsfsError", "NEAREST", "BILINEAR", "MAX_VIEWS",
           "LOG_U_DEFAULT", "lib", "make_camera", "make_grid", "DiffPlan", "OccupancyLoss",
           "occupancy_loss"]
