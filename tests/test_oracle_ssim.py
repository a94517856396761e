"""Pins of the SSIM and APE measures of section 5.1 (the paper cites the SSIM
of Wang et al. without restating it): closed forms, symmetry, the window's
definition and a brute-force window."""
import math

import numpy as np
import pytest

from oracle import metrics as Q
import synth

C1 = (0.01 * 255) ** 2
C2 = (0.03 * 255) ** 2


def test_window_is_the_normalised_gaussian():
    w = Q.ssim_window()
    assert w.shape == (11, 11)
    assert math.isclose(w.sum(), 1.0, rel_tol=1e-15)
    g = np.array([math.exp(-(i - 5) ** 2 / (2 * 1.5 ** 2)) for i in range(11)])
    g /= g.sum()
    assert np.allclose(w, np.outer(g, g), rtol=1e-14, atol=0)
    assert w[5, 5] == w.max() and np.allclose(w, w.T)


def test_identical_images_give_one():
    x = synth.ar1_image(40, 50, rho=0.9, seed=1)
    m = Q.ssim_map(x, x)
    assert m.shape == (30, 40)
    assert np.allclose(m, 1.0, rtol=0, atol=1e-14)


def test_constant_images_closed_form():
    for a, b in ((0, 0), (10, 200), (128, 127), (255, 3)):
        x = np.full((16, 16), a, np.uint8)
        y = np.full((16, 16), b, np.uint8)
        want = (2 * a * b + C1) / (a * a + b * b + C1)
        assert np.allclose(Q.ssim_map(x, y), want, rtol=1e-12, atol=0)


def test_symmetric_and_bounded():
    x = synth.ar1_image(32, 32, rho=0.9, seed=2)
    y = synth.ar1_image(32, 32, rho=0.5, seed=3)
    assert np.allclose(Q.ssim_map(x, y), Q.ssim_map(y, x), rtol=1e-14, atol=0)
    m = Q.ssim_map(x, y)
    assert np.all(m <= 1.0) and np.all(m >= -1.0)
    # an image against its negative: the structure term is negative
    assert Q.mean_ssim(x, 255 - x) < 0.5


def test_brute_force_window():
    rng = np.random.default_rng(4)
    x = rng.integers(0, 256, size=(14, 13)).astype(np.uint8)
    y = rng.integers(0, 256, size=(14, 13)).astype(np.uint8)
    w = Q.ssim_window()
    m = Q.ssim_map(x, y)
    for (i, j) in ((0, 0), (3, 2), (2, 1)):
        sx = sy = sxx = syy = sxy = 0.0
        for a in range(11):
            for b in range(11):
                xv, yv, wv = float(x[i + a, j + b]), float(y[i + a, j + b]), float(w[a, b])
                sx += wv * xv
                sy += wv * yv
                sxx += wv * xv * xv
                syy += wv * yv * yv
                sxy += wv * xv * yv
        vx, vy, cxy = sxx - sx * sx, syy - sy * sy, sxy - sx * sy
        want = (2 * sx * sy + C1) * (2 * cxy + C2) / ((sx * sx + sy * sy + C1) * (vx + vy + C2))
        assert math.isclose(m[i, j], want, rel_tol=1e-10)


def test_mean_and_ape():
    x = synth.ar1_image(24, 24, rho=0.9, seed=5)
    y = np.clip(x.astype(np.int16) + 3, 0, 255).astype(np.uint8)
    assert math.isclose(Q.mean_ssim(x, y), float(np.mean(Q.ssim_map(x, y))))
    assert Q.absolute_percentage_error(30.0, 32.0) == pytest.approx(6.25)
    assert Q.absolute_percentage_error(0.9, 0.9) == 0.0
    with pytest.raises(ValueError):
        Q.ssim_map(np.zeros((10, 20)), np.zeros((10, 20)))
