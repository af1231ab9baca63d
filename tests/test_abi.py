"""The C-ABI library loads, exports every symbol psfs.h declares, and rejects
bad arguments before touching any device. No GPU needed (no compute call here
reaches a kernel launch)."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

import paper_1311_6811_amd as psfs
from paper_1311_6811_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "psfs.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(psfs_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    return L.lib()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
    # and the binding declares a signature for each
    assert set(names) <= set(L.SIGNATURES), set(names) - set(L.SIGNATURES)
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (psfs_\w+)", out))
    assert set(names) == exported, (set(names) ^ exported)


def test_header_compiles_as_c_and_validates(tmp_path, lib):
    exe = str(tmp_path / "abi_check")
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                           os.path.join(ROOT, "tests", "abi_check.c"), "-o", exe,
                           L.LIB_PATH, f"-Wl,-rpath,{os.path.dirname(L.LIB_PATH)}"])
    out = subprocess.run([exe], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    sizes = re.search(r"sizes (\d+) (\d+) (\d+)", out.stdout).groups()
    assert tuple(map(int, sizes)) == (C.sizeof(L.psfs_camera), C.sizeof(L.psfs_grid), C.sizeof(L.psfs_params))


def _plan(lib):
    h = C.c_void_p()
    assert lib.psfs_plan_create(C.byref(h)) == 0
    return h


def _cam(W=8, H=6):
    P = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1]], np.float32)
    return psfs.make_camera(W, H, P)


def test_status_strings(lib):
    for s in range(-8, 1):
        assert lib.psfs_status_str(s) and lib.psfs_status_str(s) != b"unknown status"
    assert lib.psfs_version() == 1


def test_default_params(lib):
    p = L.psfs_params()
    lib.psfs_default_params(C.byref(p))
    assert p.prior == 0.5 and p.threshold == 0.5 and p.sampling == 0
    assert p.log_u == pytest.approx(-3 * np.log(256.0), rel=1e-7)


def test_camera_validation(lib):
    h = _plan(lib)
    cams = (L.psfs_camera * 17)(*([_cam()] * 17))
    assert lib.psfs_set_cameras(h, 17, cams) == -2
    assert lib.psfs_set_cameras(h, -1, cams) == -2
    assert lib.psfs_set_cameras(h, 2, None) == -1
    bad = _cam(0, 5)
    assert lib.psfs_set_cameras(h, 1, (L.psfs_camera * 1)(bad)) == -2
    nan = _cam()
    nan.P[3] = float("nan")
    assert lib.psfs_set_cameras(h, 1, (L.psfs_camera * 1)(nan)) == -2
    assert b"not finite" in lib.psfs_last_error()
    huge = _cam(65535, 65535)
    assert lib.psfs_set_cameras(h, 1, (L.psfs_camera * 1)(huge)) == -2
    assert lib.psfs_set_cameras(h, 0, None) == 0          # zero views is valid
    assert lib.psfs_set_cameras(None, 0, None) == -1
    lib.psfs_plan_destroy(h)


def test_grid_and_params_validation(lib):
    h = _plan(lib)
    g = psfs.make_grid(-1, 2, 2, (0, 0, 0), 0.1)
    assert lib.psfs_set_grid(h, C.byref(g)) == -2
    g = psfs.make_grid(2048, 2048, 512, (0, 0, 0), 0.1)       # 2^31 voxels
    assert lib.psfs_set_grid(h, C.byref(g)) == -2
    g = psfs.make_grid(2, 2, 2, (0, 0, 0), 0.0)
    assert lib.psfs_set_grid(h, C.byref(g)) == -2
    g = psfs.make_grid(0, 3, 3, (0, 0, 0), 0.1)                # empty grid is valid
    assert lib.psfs_set_grid(h, C.byref(g)) == 0
    for prior, log_u, tau, samp, want in ((0.0, -1, 0.5, 0, -2), (1.0, -1, 0.5, 0, -2), (0.5, float("inf"), 0.5, 0, -2),
                                          (0.5, -1, 1.5, 0, -2), (0.5, -1, 0.5, 2, -1), (0.3, -1, 0.0, 1, 0)):
        p = L.psfs_params(prior, log_u, tau, samp)
        assert lib.psfs_set_params(h, C.byref(p)) == want
    lib.psfs_plan_destroy(h)


def test_not_ready_and_pointer_checks(lib):
    h = _plan(lib)
    fake = C.c_void_p(0x100000)
    assert lib.psfs_set_background(h, 0, fake, fake) == -3          # cameras not set
    assert lib.psfs_lmap_floats(h) == -3
    assert lib.psfs_workspace_bytes(h) == 0
    cams = (L.psfs_camera * 2)(_cam(8, 6), _cam(5, 3))
    assert lib.psfs_set_cameras(h, 2, cams) == 0
    assert lib.psfs_lmap_floats(h) == 128
    assert lib.psfs_lmap_offset(h, 1) == 64
    assert lib.psfs_lmap_offset(h, 2) == -2
    assert lib.psfs_workspace_bytes(h) == 512
    assert lib.psfs_set_background(h, 2, fake, fake) == -2
    assert lib.psfs_set_background(h, 0, None, fake) == -1
    assert lib.psfs_set_background(h, 0, C.c_void_p(0x100004), fake) == -1   # misaligned
    imgs = L.ptr_array([0x100000, 0x100000])
    assert lib.psfs_likelihood(h, imgs, fake, None) == -3            # backgrounds missing
    assert lib.psfs_set_background(h, 0, fake, fake) == 0
    assert lib.psfs_set_background(h, 1, fake, fake) == 0
    assert lib.psfs_likelihood(h, L.ptr_array([0x100000, 0x100001]), fake, None) == -1  # image misaligned
    assert lib.psfs_likelihood(h, None, fake, None) == -1
    assert lib.psfs_fuse(h, fake, fake, None, None) == -3            # grid missing
    g = psfs.make_grid(4, 4, 4, (0, 0, 0), 0.1)
    assert lib.psfs_set_grid(h, C.byref(g)) == 0
    assert lib.psfs_fuse(h, fake, None, None, None) == -1
    assert lib.psfs_fuse(h, fake, C.c_void_p(0x100008), None, None) == -1
    assert lib.psfs_reconstruct(h, imgs, fake, None, fake, 100, None) == -4   # workspace too small
    assert lib.psfs_reconstruct(h, imgs, fake, None, None, 4096, None) == -4
    # setting cameras again forgets the backgrounds
    assert lib.psfs_set_cameras(h, 2, cams) == 0
    assert lib.psfs_reconstruct(h, imgs, fake, None, fake, 4096, None) == -3
    lib.psfs_plan_destroy(h)


def test_pipeline_step_validation_without_device(lib):
    h = _plan(lib)
    fake, fake2 = C.c_void_p(0x100000), C.c_void_p(0x200000)
    imgs = L.ptr_array([0x100000, 0x100000])
    cams = (L.psfs_camera * 2)(_cam(8, 6), _cam(5, 3))
    assert lib.psfs_set_cameras(h, 2, cams) == 0
    assert lib.psfs_pipeline_step(h, imgs, fake, fake2, fake, None, None) == -3   # grid missing
    g = psfs.make_grid(4, 4, 4, (0, 0, 0), 0.1)
    assert lib.psfs_set_grid(h, C.byref(g)) == 0
    assert lib.psfs_pipeline_step(h, None, None, None, None, None, None) == 0    # nothing to do
    assert lib.psfs_pipeline_step(h, imgs, fake, None, None, None, None) == -3   # backgrounds missing
    assert lib.psfs_set_background(h, 0, fake, fake) == 0
    assert lib.psfs_set_background(h, 1, fake, fake) == 0
    assert lib.psfs_pipeline_step(h, imgs, None, None, None, None, None) == -1   # no lmap_next
    assert lib.psfs_pipeline_step(h, imgs, C.c_void_p(0x100004), None, None, None, None) == -1
    assert lib.psfs_pipeline_step(h, L.ptr_array([0x100000, 0x100002]), fake, None, None, None, None) == -1
    assert lib.psfs_pipeline_step(h, None, None, None, None, fake, None) == -1   # occupancy without posterior
    assert lib.psfs_pipeline_step(h, None, None, None, fake, None, None) == -1   # no lmap_cur
    assert lib.psfs_pipeline_step(h, None, None, fake, C.c_void_p(0x100008), None, None) == -1
    # 128 floats of maps: [0x100000, 0x100200) overlaps a buffer starting 0x100100
    assert lib.psfs_pipeline_step(h, imgs, fake, C.c_void_p(0x100100), fake2, None, None) == -1
    assert "overlap" in lib.psfs_last_error().decode()
    lib.psfs_plan_destroy(h)


def test_pipeline_step_pair_validation_without_device(lib):
    h = _plan(lib)
    fake, fake2, out = C.c_void_p(0x100000), C.c_void_p(0x200000), C.c_void_p(0x300000)
    imgs = L.ptr_array([0x100000, 0x100000])
    cams = (L.psfs_camera * 2)(_cam(8, 6), _cam(5, 3))
    assert lib.psfs_set_cameras(h, 2, cams) == 0
    step = lib.psfs_pipeline_step_pair
    assert step(h, imgs, imgs, fake, fake2, out, None, out, None, None) == -3          # grid missing
    g = psfs.make_grid(4, 4, 4, (0, 0, 0), 0.1)
    assert lib.psfs_set_grid(h, C.byref(g)) == 0
    assert step(h, None, None, None, None, None, None, None, None, None) == 0          # nothing to do
    assert step(h, imgs, imgs, fake, None, None, None, None, None, None) == -3         # backgrounds missing
    assert lib.psfs_set_background(h, 0, fake, fake) == 0
    assert lib.psfs_set_background(h, 1, fake, fake) == 0
    assert step(h, imgs, None, fake, None, None, None, None, None, None) == -1         # frame B's images
    assert step(h, imgs, imgs, None, None, None, None, None, None, None) == -1         # no lmap2_next
    assert step(h, imgs, imgs, C.c_void_p(0x100004), None, None, None, None, None, None) == -1
    assert step(h, None, None, None, fake, out, None, None, None, None) == -1          # frame B's posterior
    assert step(h, None, None, None, None, out, None, out, None, None) == -1           # no lmap2_cur
    assert step(h, None, None, None, fake, C.c_void_p(0x300008), None, out, None, None) == -1
    assert step(h, None, None, None, None, None, out, None, None, None) == -1          # occupancy without posterior
    # 2 x 128 floats of pair maps: [0x100000, 0x100400) overlaps a buffer at 0x100300
    assert step(h, imgs, imgs, fake, C.c_void_p(0x100300), out, None, out, None, None) == -1
    assert "overlap" in lib.psfs_last_error().decode()
    p = L.psfs_params()
    lib.psfs_default_params(C.byref(p))
    p.sampling = psfs.BILINEAR
    assert lib.psfs_set_params(h, C.byref(p)) == 0
    assert step(h, imgs, imgs, fake, None, None, None, None, None, None) == -1         # nearest sampling only
    lib.psfs_plan_destroy(h)


def test_pipeline_step_quad_validation_without_device(lib):
    h = _plan(lib)
    fake, fake2, out = C.c_void_p(0x100000), C.c_void_p(0x200000), C.c_void_p(0x300000)
    imgs = L.ptr_array([0x100000] * 8)                       # 4 frames x 2 views, frame-major
    posts = L.ptr_array([0x300000] * 4)
    cams = (L.psfs_camera * 2)(_cam(8, 6), _cam(5, 3))
    assert lib.psfs_set_cameras(h, 2, cams) == 0
    step = lib.psfs_pipeline_step_quad
    assert step(h, imgs, fake, fake2, posts, None, None) == -3          # grid missing
    g = psfs.make_grid(4, 4, 4, (0, 0, 0), 0.1)
    assert lib.psfs_set_grid(h, C.byref(g)) == 0
    assert step(h, None, None, None, None, None, None) == 0             # nothing to do
    assert step(h, imgs, fake, None, None, None, None) == -3            # backgrounds missing
    assert lib.psfs_set_background(h, 0, fake, fake) == 0
    assert lib.psfs_set_background(h, 1, fake, fake) == 0
    holed = L.ptr_array([0x100000] * 7 + [0])                   # frame 3, view 1 missing
    assert step(h, holed, fake, None, None, None, None) == -1
    assert "view 1" in lib.psfs_last_error().decode()
    odd = L.ptr_array([0x100000] * 5 + [0x100002] + [0x100000] * 2)   # frame 2, view 1 misaligned
    assert step(h, odd, fake, None, None, None, None) == -1
    assert step(h, imgs, None, None, None, None, None) == -1            # no lmap4_next
    assert step(h, imgs, C.c_void_p(0x100004), None, None, None, None) == -1
    assert step(h, None, None, None, L.ptr_array([0x300000] * 3 + [0]), None, None) == -1   # frame 3's posterior
    assert "frame 3" in lib.psfs_last_error().decode()
    assert step(h, None, None, None, L.ptr_array([0x300000, 0x300008, 0x300000, 0x300000]), None, None) == -1
    assert step(h, None, None, None, posts, None, None) == -1           # no lmap4_cur
    assert step(h, None, None, None, None, posts, None) == -1           # occupancy without posteriors
    # 4 x 128 floats of quad maps: [0x100000, 0x100800) overlaps a buffer at 0x100700
    assert step(h, imgs, fake, C.c_void_p(0x100700), posts, None, None) == -1
    assert "overlap" in lib.psfs_last_error().decode()
    p = L.psfs_params()
    lib.psfs_default_params(C.byref(p))
    p.sampling = psfs.BILINEAR
    assert lib.psfs_set_params(h, C.byref(p)) == 0
    assert step(h, imgs, fake, None, None, None, None) == -1            # nearest sampling only
    lib.psfs_default_params(C.byref(p))
    assert lib.psfs_set_params(h, C.byref(p)) == 0
    big = (L.psfs_camera * 2)(_cam(8, 6), _cam(16384, 16384))           # 2^28 pixels
    assert lib.psfs_set_cameras(h, 2, big) == 0
    assert step(h, None, None, None, posts, None, None) == -2           # quad maps need < 2^28 pixels
    assert "2^28" in lib.psfs_last_error().decode()
    lib.psfs_plan_destroy(h)


def test_surface_validation_without_device(lib):
    h = _plan(lib)
    fake = C.c_void_p(0x100000)
    assert lib.psfs_surface_workspace_bytes(h) == 0
    assert lib.psfs_surface(h, fake, None, fake, fake, 10, fake, fake, 4096, None) == -3   # grid missing
    g = psfs.make_grid(40, 30, 20, (0, 0, 0), 0.1)
    assert lib.psfs_set_grid(h, C.byref(g)) == 0
    need = lib.psfs_surface_workspace_bytes(h)
    assert need == 256 + 24064             # 6 int32 block counts (256 B) + one flag byte per voxel, 256-B rounded
    assert lib.psfs_surface(h, fake, None, fake, fake, -1, fake, fake, need, None) == -2
    assert lib.psfs_surface(h, fake, None, fake, fake, 10, None, fake, need, None) == -1
    assert lib.psfs_surface(h, None, None, fake, fake, 10, fake, fake, need, None) == -1
    assert lib.psfs_surface(h, fake, None, None, fake, 10, fake, fake, need, None) == -1
    assert lib.psfs_surface(h, fake, None, fake, None, 10, fake, fake, need, None) == -1
    assert lib.psfs_surface(h, fake, None, fake, fake, 10, C.c_void_p(0x100004), fake, need, None) == -1
    assert lib.psfs_surface(h, fake, None, fake, fake, 10, fake, fake, need - 1, None) == -4
    assert lib.psfs_surface(h, fake, None, fake, fake, 10, fake, None, need, None) == -4
    lib.psfs_plan_destroy(h)


def test_colour_validation_without_device(lib):
    h = _plan(lib)
    fake = C.c_void_p(0x100000)
    imgs = L.ptr_array([0x100000, 0x100000])
    assert lib.psfs_colour_workspace_bytes(h) == 0
    assert lib.psfs_colour(h, imgs, fake, 10, fake, fake, fake, 4096, None) == -3        # cameras missing
    cams = (L.psfs_camera * 2)(_cam(8, 6), _cam(5, 3))
    assert lib.psfs_set_cameras(h, 2, cams) == 0
    assert lib.psfs_colour(h, imgs, fake, 10, fake, fake, fake, 4096, None) == -3        # grid missing
    g = psfs.make_grid(4, 4, 4, (0, 0, 0), 0.1)
    assert lib.psfs_set_grid(h, C.byref(g)) == 0
    need = lib.psfs_colour_workspace_bytes(h)
    assert need == 8 * 128                                   # 8 B per element of the 128-float map layout
    assert lib.psfs_colour(h, imgs, fake, -1, fake, fake, fake, need, None) == -2
    assert lib.psfs_colour(h, None, fake, 10, fake, fake, fake, need, None) == -1
    assert lib.psfs_colour(h, imgs, None, 10, fake, fake, fake, need, None) == -1
    assert lib.psfs_colour(h, imgs, fake, 10, None, fake, fake, need, None) == -1
    assert lib.psfs_colour(h, imgs, fake, 10, fake, None, fake, need, None) == -1
    assert lib.psfs_colour(h, imgs, fake, 10, fake, fake, fake, need - 8, None) == -4
    assert lib.psfs_colour(h, imgs, fake, 0, None, None, fake, need, None) == 0         # empty list: no-op
    lib.psfs_plan_destroy(h)


def test_foreground_validation_without_device(lib):
    h = _plan(lib)
    fake = C.c_void_p(0x100000)
    imgs = L.ptr_array([0x100000, 0x100000])
    assert lib.psfs_foreground_model(h, imgs, None, fake, fake, fake, 16384, None) == -3     # cameras missing
    cams = (L.psfs_camera * 2)(_cam(8, 6), _cam(5, 3))
    assert lib.psfs_set_cameras(h, 2, cams) == 0
    assert lib.psfs_foreground_model(h, None, None, fake, fake, fake, 16384, None) == -1
    assert lib.psfs_foreground_model(h, imgs, None, fake, None, fake, 16384, None) == -1     # no output
    assert lib.psfs_foreground_model(h, imgs, None, None, fake, fake, 16384, None) == -1     # no masks, no maps
    masks = L.ptr_array([0x100000, 0])
    assert lib.psfs_foreground_model(h, imgs, masks, None, fake, fake, 16384, None) == -1    # view 1 needs maps
    assert lib.psfs_foreground_model(h, imgs, None, fake, fake, fake, 16383, None) == -4
    assert lib.psfs_set_foreground(h, C.c_void_p(0x100002)) == -1
    assert lib.psfs_set_foreground(h, fake) == 0
    assert lib.psfs_set_foreground(h, None) == 0
    lib.psfs_plan_destroy(h)


def test_particle_weights_validation_without_device(lib):
    h = _plan(lib)
    fake = C.c_void_p(0x100000)
    maps = L.ptr_array([0x100000, 0x100000])
    out = C.c_void_p(0x200000)
    assert lib.psfs_particle_weights(h, fake, 4, maps, maps, 1.0, out, out, out, None) == -3     # cameras missing
    cams = (L.psfs_camera * 2)(_cam(8, 6), _cam(5, 3))
    assert lib.psfs_set_cameras(h, 2, cams) == 0
    assert lib.psfs_particle_weights(h, fake, -1, maps, maps, 1.0, out, out, out, None) == -2
    assert lib.psfs_particle_weights(h, fake, 1 << 31, maps, maps, 1.0, out, out, out, None) == -2
    assert lib.psfs_particle_weights(h, fake, 4, maps, maps, -0.5, out, out, out, None) == -2    # beta < 0
    assert lib.psfs_particle_weights(h, fake, 4, maps, maps, float("nan"), out, out, out, None) == -2
    assert lib.psfs_particle_weights(h, None, 4, maps, maps, 1.0, out, out, out, None) == -1
    assert lib.psfs_particle_weights(h, C.c_void_p(0x100008), 4, maps, maps, 1.0, out, out, out, None) == -1  # not 16-aligned
    assert lib.psfs_particle_weights(h, fake, 4, maps, maps, 1.0, None, out, out, None) == -1      # log_w required
    assert lib.psfs_particle_weights(h, fake, 4, maps, maps, 1.0, C.c_void_p(0x200004), None, None, None) == -1
    assert lib.psfs_particle_weights(h, fake, 4, None, maps, 1.0, out, None, None, None) == -1
    holes = L.ptr_array([0x100000, 0])
    assert lib.psfs_particle_weights(h, fake, 4, maps, holes, 1.0, out, None, None, None) == -1   # view 1 edge map
    assert lib.psfs_particle_weights(h, fake, 0, None, None, 1.0, None, None, None, None) == 0    # no particles: no-op
    lib.psfs_plan_destroy(h)


def test_empty_work_is_a_no_op_without_device(lib):
    h = _plan(lib)
    assert lib.psfs_set_cameras(h, 0, None) == 0
    g = psfs.make_grid(0, 4, 4, (0, 0, 0), 0.1)
    assert lib.psfs_set_grid(h, C.byref(g)) == 0
    assert lib.psfs_reconstruct(h, None, None, None, None, 0, None) == 0
    assert lib.psfs_threshold(None, 0, 0.5, None, None) == 0
    assert lib.psfs_threshold(None, -1, 0.5, None, None) == -2
    assert lib.psfs_threshold(None, 5, 1.5, None, None) == -2
    lib.psfs_plan_destroy(h)


def test_tiles(lib):
    tiles = psfs.tiles()
    assert len(tiles) >= 4
    for tx, ty, kz in tiles:
        assert tx * ty in (64, 128, 256, 512, 1024) and tx * ty % 64 == 0 and kz >= 1
    assert lib.psfs_tile_describe(len(tiles), None, None, None) == -2
    h = _plan(lib)
    assert lib.psfs_set_tile(h, len(tiles)) == -2
    assert lib.psfs_set_tile(h, -1) == 0
    lib.psfs_plan_destroy(h)


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        L.lib()


def test_diff_validation_without_device(lib):
    h = _plan(lib)
    assert lib.psfs_diff_workspace_bytes(h) == 0
    cams = (L.psfs_camera * 2)(_cam(8, 6), _cam(5, 3))
    assert lib.psfs_set_cameras(h, 2, cams) == 0
    g = psfs.make_grid(40, 8, 9, (0, 0, 0), 0.1)
    assert lib.psfs_set_grid(h, C.byref(g)) == 0
    fake = C.c_void_p(0x100000)
    for k in range(2):
        assert lib.psfs_set_background(h, k, fake, fake) == 0
    need = lib.psfs_diff_workspace_bytes(h)
    # two padded maps (2 x 128 floats), their int64 fixed-point adjoints, one
    # FP64 partial per forward workgroup and 2 x 12 FP32 partials per backward
    # workgroup (both: 16 x 16 voxel columns x 8 slices), each region 256-byte aligned
    nbf = 3 * 1 * 2
    nbb = 3 * 1 * 2
    want = 512 + 1024 + 256 * ((nbf * 8 + 255) // 256) + 256 * ((nbb * 24 * 4 + 255) // 256)
    assert need == want
    imgs = L.ptr_array([0x100000, 0x100000])
    ws = C.c_void_p(0x200000)
    bad = (C.c_int32 * 6)(0, 41, 0, 8, 0, 9)
    assert lib.psfs_diff_forward(h, imgs, fake, bad, fake, fake, ws, need, None) == -2
    bad = (C.c_int32 * 6)(3, 2, 0, 8, 0, 9)
    assert lib.psfs_diff_forward(h, imgs, fake, bad, fake, fake, ws, need, None) == -2
    assert lib.psfs_diff_forward(h, imgs, fake, None, fake, fake, ws, need - 1, None) == -4
    assert lib.psfs_diff_forward(h, imgs, fake, None, fake, fake, C.c_void_p(0x200010), need, None) == -4
    assert lib.psfs_diff_forward(h, imgs, None, None, fake, fake, ws, need, None) == -1
    assert lib.psfs_diff_forward(h, imgs, fake, None, fake, None, ws, need, None) == -1
    assert lib.psfs_diff_backward(h, imgs, fake, None, fake, None, L.ptr_array([0x100000] * 2),
                                  L.ptr_array([0x100000] * 2), fake, ws, need, None) == -1
    assert lib.psfs_diff_backward(h, imgs, fake, None, fake, fake, L.ptr_array([0x100000, 0x100004]),
                                  L.ptr_array([0x100000] * 2), fake, ws, need, None) == -1
    lib.psfs_plan_destroy(h)


def test_batch_validation_without_device(lib):
    params = L.psfs_params()
    lib.psfs_default_params(C.byref(params))
    h = C.c_void_p()
    assert lib.psfs_batch_create(C.byref(h), C.byref(params), 0, None) == -2
    assert lib.psfs_batch_create(C.byref(h), C.byref(params), 1, None) == -1
    cams = (L.psfs_camera * 1)(_cam(8, 6))
    ptrs = L.ptr_array([0x100000])
    fr = (L.psfs_frame * 1)()
    fr[0].grid = psfs.make_grid(4, 4, 4, (0, 0, 0), 0.1)
    fr[0].n = 0
    assert lib.psfs_batch_create(C.byref(h), C.byref(params), 1, fr) == -2       # no views
    fr[0].n = 1
    fr[0].cams, fr[0].images_dev, fr[0].mean_dev, fr[0].var_dev = cams, ptrs, ptrs, ptrs
    fr[0].posterior_dev = None
    assert lib.psfs_batch_create(C.byref(h), C.byref(params), 1, fr) == -1       # posterior NULL
    fr[0].posterior_dev = 0x100000
    fr[0].images_dev = L.ptr_array([0x100002])
    assert lib.psfs_batch_create(C.byref(h), C.byref(params), 1, fr) == -1       # image misaligned
    bad = L.psfs_params(0.5, -1.0, 0.5, 3)
    assert lib.psfs_batch_create(C.byref(h), C.byref(bad), 1, fr) == -1
    assert lib.psfs_batch_workspace_bytes(None) == 0
    assert lib.psfs_batch_set_tile(None, 0) == -1
    assert lib.psfs_batch_run(None, None, 0, None) == -1
    lib.psfs_batch_destroy(None)


def test_short_map_buffers_are_refused_before_any_launch(lib):
    """The map arguments of the C entry points carry no length, so the binding
    checks that a buffer holds k x lmap_floats values (k frames interleaved)
    before it passes the pointer on."""
    import torch
    from synth import scene as S
    cams, grid = S.config_frame_rig(0)
    plan = psfs.Plan(cams, grid)
    nf = plan.lmap_floats()
    assert nf == sum(c.width * c.height for c in cams)        # 64-float aligned views of 320x240
    for frames in (1, 2, 4):
        with pytest.raises(ValueError, match=f"{frames} x lmap_floats"):
            plan._map(torch.empty(frames * nf - 1, dtype=torch.float32), frames, "lmap")
        with pytest.raises(ValueError):
            plan._map(None, frames, "lmap")
    with pytest.raises(TypeError, match="GPU tensor"):              # long enough: the device check follows
        plan._map(torch.empty(4 * nf, dtype=torch.float32), 4, "lmap")


def test_input_check_validation_without_device(lib):
    assert lib.psfs_set_input_check(None, None) == -1
    h = _plan(lib)
    assert lib.psfs_input_status(h) == -3                              # no flags word set
    assert lib.psfs_set_input_check(h, C.c_void_p(0x100002)) == -1     # misaligned
    assert lib.psfs_set_input_check(h, C.c_void_p(0x100004)) == 0
    assert lib.psfs_set_input_check(h, None) == 0                      # off again
    assert lib.psfs_input_status(h) == -3
    assert lib.psfs_input_status(None) == -1
    lib.psfs_plan_destroy(h)


def test_reconstruct_static_validation_without_device(lib):
    h = _plan(lib)
    one = L.ptr_array([0x100000])
    assert lib.psfs_reconstruct_static(None, one, None, None, None) == -1
    assert lib.psfs_reconstruct_static(h, one, C.c_void_p(0x300000), None, None) == -3     # nothing set
    big = (L.psfs_camera * 1)(_cam(8192, 4096))                                            # 128 MiB of maps
    assert lib.psfs_set_cameras(h, 1, big) == 0
    assert lib.psfs_set_background(h, 0, C.c_void_p(0x100000), C.c_void_p(0x100000)) == 0
    g = psfs.make_grid(4, 4, 4, (0, 0, 0), 0.1)
    assert lib.psfs_set_grid(h, C.byref(g)) == 0
    assert lib.psfs_reconstruct_static(h, one, C.c_void_p(0x300004), None, None) == -1     # misaligned posterior
    assert lib.psfs_reconstruct_static(h, one, C.c_void_p(0x300000), None, None) == -2     # beyond the static array
    assert "static scratch" in lib.psfs_last_error().decode()
    lib.psfs_plan_destroy(h)


def test_plan_tuner_validation_without_device(lib):
    h = _plan(lib)
    one = L.ptr_array([0x100000])
    best = C.c_int32(-5)
    assert lib.psfs_tune(None, one, None, 0, None, 0, C.byref(best)) == -1
    assert lib.psfs_tune(h, one, None, 0, None, 0, C.byref(best)) == -3          # nothing set
    assert lib.psfs_tune_workspace_bytes(h) == 0
    cams = (L.psfs_camera * 1)(_cam(8, 6))
    assert lib.psfs_set_cameras(h, 1, cams) == 0
    assert lib.psfs_set_background(h, 0, C.c_void_p(0x100000), C.c_void_p(0x100000)) == 0
    g = psfs.make_grid(4, 5, 6, (0, 0, 0), 0.1)
    assert lib.psfs_set_grid(h, C.byref(g)) == 0
    need = lib.psfs_tune_workspace_bytes(h)
    assert need >= 3 * 256                                          # maps, posterior, occupancy regions
    assert lib.psfs_tune(h, one, C.c_void_p(0x200000), need - 1, None, 0, C.byref(best)) == -4
    assert lib.psfs_tune(h, one, C.c_void_p(0x200080), need, None, 0, C.byref(best)) == -4    # not 256-aligned
    assert best.value == -5
    assert lib.psfs_get_tile(h) >= 0 and lib.psfs_get_tile(None) == -1
    assert lib.psfs_set_tile(h, 3) == 0 and lib.psfs_get_tile(h) == 3
    lib.psfs_plan_destroy(h)
