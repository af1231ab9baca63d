"""Pins of the learned-foreground oracle (colour histogram density used in
place of the uniform density of Eq. 1-2 after the first frame): hand values,
numpy's histogramdd, the uniform special case against the pinned C oracle,
and the normalisation of the density. No GPU."""
import numpy as np

from oracle import foreground as FG
from oracle import oracle as O


def test_bin_index_hand_values():
    cols = np.array([[0, 0, 0], [255, 255, 255], [16, 0, 0], [0, 16, 0], [0, 0, 16], [15, 31, 47]], np.uint8)
    assert FG.bin_index(cols).tolist() == [0, 4095, 256, 16, 1, 18]


def test_histogram_matches_histogramdd():
    rng = np.random.default_rng(3)
    imgs = [rng.integers(0, 256, (30, 40, 3)).astype(np.uint8) for _ in range(3)]
    masks = [rng.random((30, 40)) < 0.3 for _ in range(3)]
    got = FG.histogram(imgs, masks)
    pts = np.concatenate([im[m] for im, m in zip(imgs, masks)]).astype(np.float64)
    edges = [np.arange(0, 257, 16)] * 3
    want, _ = np.histogramdd(pts, bins=edges)
    assert np.array_equal(got, want.reshape(-1).astype(np.int64))
    assert got.sum() == sum(int(m.sum()) for m in masks)


def test_empty_model_is_the_uniform_density_of_the_first_frame():
    logd = FG.log_density(np.zeros(FG.NBINS, np.int64))
    np.testing.assert_allclose(logd, O.LOG_U_DEFAULT, rtol=0, atol=1e-12)
    rng = np.random.default_rng(5)
    img = rng.integers(0, 256, (20, 24, 3)).astype(np.uint8)
    mean = (rng.random((20, 24, 3)) * 255).astype(np.float32)
    var = ((5 + 10 * rng.random((20, 24, 3))) ** 2).astype(np.float32)
    np.testing.assert_allclose(FG.slm(img, mean, var, logd), O.slm(img, mean, var), rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(FG.log2slm(img, mean, var, logd), O.log2slm(img, mean, var), rtol=1e-11, atol=1e-12)


def test_hand_density_and_normalisation():
    counts = np.zeros(FG.NBINS, np.int64)
    counts[0] = 3
    counts[4095] = 1
    logd = FG.log_density(counts)
    assert np.isclose(np.exp(logd[0]), 4.0 / (4100 * 4096), rtol=1e-14)
    assert np.isclose(np.exp(logd[4095]), 2.0 / (4100 * 4096), rtol=1e-14)
    assert np.isclose(np.exp(logd[7]), 1.0 / (4100 * 4096), rtol=1e-14)
    assert np.isclose((np.exp(logd) * 4096).sum(), 1.0, rtol=1e-12)      # a density over the 256^3 cube


def test_more_foreground_evidence_raises_slm():
    rng = np.random.default_rng(8)
    img = rng.integers(0, 256, (10, 10, 3)).astype(np.uint8)
    mean = img.astype(np.float32) + 20.0
    var = np.full((10, 10, 3), 100.0, np.float32)
    c0 = np.zeros(FG.NBINS, np.int64)
    c1 = c0.copy()
    c1[FG.bin_index(img).reshape(-1)] += 50
    s0 = FG.slm(img, mean, var, FG.log_density(c0))
    s1 = FG.slm(img, mean, var, FG.log_density(c1))
    assert np.all(s1 > s0)
    np.testing.assert_allclose(FG.log2slm(img, mean, var, FG.log_density(c1)), np.log(2 * s1), rtol=1e-12)
