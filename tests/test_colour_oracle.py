"""Pins of the voxel-colour oracle (depth-buffer visibility, mean colour over
the views that see a voxel) against hand cases, brute-force loops written from
the reading, and counting invariants. No GPU."""
import numpy as np

from oracle import colour as CO
from synth import scene as S


def tiny_grid(nx, ny, nz, origin, h):
    return S.Grid(nx, ny, nz, np.asarray(origin, np.float32), np.float32(h))


def test_hand_case_nearest_voxel_on_a_ray_wins():
    # four voxels on the x axis; camera 0 on the +x axis looks at them end-on
    # (one pixel, the voxel nearest to it wins); camera 1 on the +y axis sees
    # all four side by side.
    grid = tiny_grid(4, 1, 1, (-0.5, -0.0625, -0.0625), 0.125)   # centres x = -0.4375..0.3125, y = z = 0
    cam0 = S.look_at_camera((4.0, 0.0, 0.0), 100.0, 64, 48, up=(0.0, 0.0, 1.0))
    cam1 = S.look_at_camera((0.0, 4.0, 0.0), 100.0, 64, 48, up=(0.0, 0.0, 1.0))
    rng = np.random.default_rng(0)
    im0 = rng.integers(0, 256, (48, 64, 3)).astype(np.uint8)
    im1 = rng.integers(0, 256, (48, 64, 3)).astype(np.uint8)
    idx = np.arange(4)
    col, views, amb = CO.colour([cam0, cam1], grid, [im0, im1], idx)
    assert views.tolist() == [1, 1, 1, 2]                  # only the voxel at x = 0.3125 wins in camera 0
    x1, y1, _, ok1, _, _, _ = CO.project(cam1, CO.voxel_centres(grid, idx))
    x0, y0, _, ok0, _, _, _ = CO.project(cam0, CO.voxel_centres(grid, idx))
    assert ok0.all() and ok1.all() and len(set(zip(x1, y1))) == 4 and len(set(zip(x0, y0))) == 1
    for v in range(3):
        assert np.array_equal(col[v], im1[y1[v], x1[v]].astype(np.float64))
    want = (im0[y0[3], x0[3]].astype(np.float64) + im1[y1[3], x1[3]].astype(np.float64)) / 2
    assert np.array_equal(col[3], want)


def brute_force(cams, grid, images, idx):
    n = len(idx)
    sums = np.zeros((n, 3))
    views = np.zeros(n, dtype=np.int64)
    for cam, img in zip(cams, images):
        P = cam.P.astype(np.float64)
        best = {}
        for q, v in enumerate(idx):
            i, j, k = v % grid.nx, (v // grid.nx) % grid.ny, v // (grid.nx * grid.ny)
            X = np.array([grid.origin[0] + grid.voxel * (i + 0.5), grid.origin[1] + grid.voxel * (j + 0.5),
                          grid.origin[2] + grid.voxel * (k + 0.5), 1.0], np.float64)
            a, b, c = P @ X
            if not c > 0:
                continue
            px, py = int(np.floor(a / c + 0.5)), int(np.floor(b / c + 0.5))
            if not (0 <= px < cam.width and 0 <= py < cam.height):
                continue
            key = (c, q)
            if (px, py) not in best or key < best[(px, py)][0]:
                best[(px, py)] = (key, q)
        for (px, py), (_, q) in best.items():
            sums[q] += img[py, px]
            views[q] += 1
    col = np.where(views[:, None] > 0, sums / np.maximum(views, 1)[:, None], 0.0)
    return col, views


def test_matches_brute_force_on_random_lists():
    rng = np.random.default_rng(11)
    for trial in range(4):
        grid = tiny_grid(12, 10, 9, (-0.6, -0.5, -0.45), 0.1)
        cams = S.ring_rig(3, 60.0, 40, 30, phase=float(rng.uniform(0, 6)))
        images = [rng.integers(0, 256, (c.height, c.width, 3)).astype(np.uint8) for c in cams]
        idx = np.sort(rng.choice(grid.nx * grid.ny * grid.nz, 300, replace=False))
        col, views, _ = CO.colour(cams, grid, images, idx)
        bcol, bviews = brute_force(cams, grid, images, idx)
        assert np.array_equal(views, bviews)
        np.testing.assert_allclose(col, bcol, rtol=0, atol=1e-12)


def test_one_winner_per_pixel():
    rng = np.random.default_rng(2)
    grid = tiny_grid(20, 20, 20, (-1, -1, -1), 0.1)
    cams = S.ring_rig(4, 80.0, 64, 48)
    images = [np.zeros((c.height, c.width, 3), np.uint8) for c in cams]
    idx = np.sort(rng.choice(8000, 2000, replace=False))
    col, views, _ = CO.colour(cams, grid, images, idx)
    X = CO.voxel_centres(grid, idx)
    distinct = 0
    for cam in cams:
        x, y, _, ok, _, _, _ = CO.project(cam, X)
        distinct += len(set(zip(x[ok].tolist(), y[ok].tolist())))
    assert views.sum() == distinct
    assert np.all(col == 0)


def test_voxels_behind_a_camera_inside_the_grid_are_not_seen():
    grid = tiny_grid(10, 10, 10, (-0.5, -0.5, -0.5), 0.1)
    cam = S.look_at_camera((0.01, 0.02, 0.03), 60.0, 80, 60, target=(3.0, 0.3, 0.2))
    rng = np.random.default_rng(4)
    img = rng.integers(0, 256, (60, 80, 3)).astype(np.uint8)
    idx = np.arange(1000)
    col, views, _ = CO.colour([cam], grid, [img], idx)
    X = CO.voxel_centres(grid, idx)
    behind = (X - np.array([0.01, 0.02, 0.03])) @ (np.array([3.0, 0.3, 0.2]) - np.array([0.01, 0.02, 0.03])) < 0
    assert behind.sum() > 300 and views[behind].sum() == 0
    bcol, bviews = brute_force([cam], grid, [img], idx)
    assert np.array_equal(views, bviews) and np.array_equal(col, bcol)
