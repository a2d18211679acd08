"""Presmoothing of the frames and the choice of the image split (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* Presmoothing (Section 1): the method works on f = K_sigma * I, the frames
  convolved with a Gaussian of standard deviation sigma.  Readings: the
  kernel is the Gaussian sampled at integer offsets |k| <= ceil(3 sigma) and
  normalised to sum 1; it is applied along x, then along y; outside the image
  the nearest border pixel is used (clamp to edge); sigma = 0 leaves the frame
  unchanged.
* Split chooser (Section 3.1, figure "ratio"): among the splits Px x Py of a
  W x H image into n = Px Py parts, take the one with the largest
  area / perimeter of a part, with area w h and perimeter 2 (w + h) for a
  part of w = W / Px by h = H / Py pixels (real-valued when the division is
  not exact).  Ties go to the split with more parts across (larger Px).
  The paper's worked example (48 x 48, twelve parts: 1.846, 3, 3.428) pins it.
"""
from __future__ import annotations

import math

import numpy as np


def gaussian_weights(sigma: float) -> np.ndarray:
    """Normalised sampled Gaussian, offsets -R..R with R = ceil(3 sigma)."""
    if sigma == 0.0:
        return np.ones(1)
    R = int(math.ceil(3.0 * sigma))
    k = np.arange(-R, R + 1, dtype=np.float64)
    w = np.exp(-k * k / (2.0 * sigma * sigma))
    return w / w.sum()


def smooth_rows(I: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Convolve every row with w, clamping column indices to the image."""
    H, W = I.shape
    R = (len(w) - 1) // 2
    out = np.zeros_like(I, dtype=np.float64)
    for k in range(-R, R + 1):
        cols = np.clip(np.arange(W) + k, 0, W - 1)
        out += w[k + R] * I[:, cols]
    return out


def presmooth(I: np.ndarray, sigma: float) -> np.ndarray:
    """f = K_sigma * I: rows first, then columns."""
    w = gaussian_weights(sigma)
    if len(w) == 1:
        return np.array(I, dtype=np.float64)
    return smooth_rows(smooth_rows(np.asarray(I, dtype=np.float64), w).T, w).T


def split_ratio(W: int, H: int, px: int, py: int) -> float:
    """area / perimeter of a part of the Px x Py split."""
    w, h = W / px, H / py
    return (w * h) / (2.0 * (w + h))


def choose_split(W: int, H: int, n: int) -> tuple[int, int, float]:
    """The split Px x Py = n with the largest ratio (ties: larger Px)."""
    best = None
    for px in range(1, n + 1):
        if n % px:
            continue
        py = n // px
        if px > W or py > H:
            continue
        r = split_ratio(W, H, px, py)
        if best is None or r > best[2] or (r == best[2] and px > best[0]):
            best = (px, py, r)
    if best is None:
        raise ValueError("no split of the image into that many parts")
    return best
