"""FP64 oracle of the learned foreground colour model for frames after the
first.

TEST INFRASTRUCTURE ONLY: used by ``tests/``; the product library never
imports this package.

Eq. 1-2 take the foreground likelihood of a pixel colour as uniform, as
nothing is known of the foreground's colours at the first frame (Sec. 2.2.2); the paper implies
but does not describe the model used afterwards. The reading taken here:

* the foreground likelihood is a colour histogram of 16 x 16 x 16 bins over
  the 8-bit RGB cube (bin = (R >> 4) * 256 + (G >> 4) * 16 + (B >> 4)), learned
  from the pixels marked foreground in the previous frame (by default those
  whose SLM exceeds 1/2, i.e. log(2*SLM) > 0), pooled over the views;
* with Laplace smoothing (alpha = 1 per bin) the density of a colour value is
  (count[bin] + alpha) / ((N + 4096 * alpha) * 4096), N = number of training
  pixels, each bin holding 16^3 = 4096 colour values;
* Eq. 1-2 then use this density in place of the uniform u: with equal priors
  SLM = F(I) / (F(I) + N(I | mu, var)).
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

NBINS = 4096
ALPHA = 1.0


def bin_index(img: np.ndarray) -> np.ndarray:
    i = np.asarray(img).astype(np.int64)
    return (i[..., 0] >> 4) * 256 + (i[..., 1] >> 4) * 16 + (i[..., 2] >> 4)


def histogram(images: Sequence[np.ndarray], masks: Sequence[np.ndarray]) -> np.ndarray:
    """int64 counts per bin of the masked pixels of all views."""
    counts = np.zeros(NBINS, dtype=np.int64)
    for img, m in zip(images, masks):
        b = bin_index(img)[np.asarray(m) != 0]
        counts += np.bincount(b, minlength=NBINS)
    return counts


def log_density(counts: np.ndarray, alpha: float = ALPHA) -> np.ndarray:
    """log of the smoothed density of one colour value in each bin (FP64)."""
    c = np.asarray(counts, dtype=np.float64)
    return np.log((c + alpha) / ((c.sum() + NBINS * alpha) * NBINS))


def log_gaussian(img, mean, var) -> np.ndarray:
    """log N(I | mu, diag(var)) per pixel (FP64)."""
    i = np.asarray(img, np.float64)
    m = np.asarray(mean, np.float64)
    v = np.asarray(var, np.float64)
    return -1.5 * np.log(2.0 * np.pi) - 0.5 * np.log(v.prod(axis=-1)) - 0.5 * (((i - m) ** 2) / v).sum(axis=-1)


def slm(img, mean, var, logd: np.ndarray) -> np.ndarray:
    """SLM = F / (F + N) with the learned foreground density F (equal priors)."""
    lf = logd[bin_index(img)]
    ln = log_gaussian(img, mean, var)
    # F/(F+N) = 1/(1 + exp(ln - lf)), evaluated without overflow
    return 0.5 * (1.0 - np.tanh(0.5 * (ln - lf)))


def log2slm(img, mean, var, logd: np.ndarray) -> np.ndarray:
    """log(2*SLM) = log 2 - softplus(log N - log F) (FP64)."""
    d = log_gaussian(img, mean, var) - logd[bin_index(img)]
    return np.log(2.0) - np.logaddexp(0.0, d)
