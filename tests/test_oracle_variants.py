"""Pins of the oracle's presmoothing and split chooser (Sections 1 and 3.1)."""
import math
import os

import numpy as np
import pytest

from oracle import variants


@pytest.mark.parametrize("sigma", [0.5, 1.0, 2.5])
def test_weights_are_a_normalised_symmetric_gaussian(sigma):
    w = variants.gaussian_weights(sigma)
    R = math.ceil(3 * sigma)
    assert len(w) == 2 * R + 1
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.array_equal(w, w[::-1])
    # ratio of neighbouring samples is the Gaussian's: exp(-(2k+1)/(2 sigma^2))
    for k in range(R):
        assert abs(w[R + k + 1] / w[R + k] - math.exp(-(2 * k + 1) / (2 * sigma * sigma))) < 1e-14


def test_sigma_zero_is_the_identity():
    I = np.random.default_rng(0).random((7, 9))
    assert np.array_equal(variants.presmooth(I, 0.0), I)


def test_constant_image_is_unchanged():
    I = np.full((11, 13), 0.37)
    assert np.abs(variants.presmooth(I, 1.7) - 0.37).max() < 1e-15


def test_linear_image_unchanged_away_from_the_border():
    # a symmetric kernel maps a linear function to itself where no clamping occurs
    H, W, sigma = 20, 24, 1.3
    R = math.ceil(3 * sigma)
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    I = 0.2 + 0.03 * x - 0.05 * y
    f = variants.presmooth(I, sigma)
    assert np.abs(f[R:H - R, R:W - R] - I[R:H - R, R:W - R]).max() < 1e-14


def test_separable_pass_equals_direct_2d_convolution():
    # brute force: the 2D kernel w_i w_j applied pixel by pixel with clamping
    rng = np.random.default_rng(3)
    H, W, sigma = 9, 8, 0.9
    I = rng.random((H, W))
    w = variants.gaussian_weights(sigma)
    R = (len(w) - 1) // 2
    ref = np.zeros((H, W))
    for y in range(H):
        for x in range(W):
            s = 0.0
            for dy in range(-R, R + 1):
                for dx in range(-R, R + 1):
                    yy = min(max(y + dy, 0), H - 1)
                    xx = min(max(x + dx, 0), W - 1)
                    s += w[dy + R] * w[dx + R] * I[yy, xx]
            ref[y, x] = s
    assert np.abs(variants.presmooth(I, sigma) - ref).max() < 1e-15


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "split_ratio_48x48.txt")


def load_split_golden():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                px, py, r = line.split()
                rows.append((int(px), int(py), float(r)))
    return rows


def test_split_ratios_of_the_papers_worked_example():
    # every split of the printed figure, to the three decimals printed
    rows = load_split_golden()
    assert len(rows) == 6
    for px, py, r in rows:
        assert math.floor(variants.split_ratio(48, 48, px, py) * 1000) / 1000 == r, (px, py)
    # the chosen split is the one with the largest printed ratio
    best = max(r for _, _, r in rows)
    px, py, r = variants.choose_split(48, 48, 12)
    assert (px, py, best) in [(a, b, c) for a, b, c in rows] and abs(r - 24 / 7) < 1e-15


def test_split_prefers_parts_across_the_longer_side():
    px, py, _ = variants.choose_split(640, 480, 16)
    assert (px, py) == (4, 4)
    px, py, _ = variants.choose_split(1920, 1080, 84)
    assert px > py
