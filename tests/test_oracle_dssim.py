"""Pins of the oracle's Eq. (1) loss: (1 - lambda) L1 + lambda (1 - SSIM)."""
import math

import numpy as np
import pytest
from scipy import ndimage
from scipy.signal import windows


def test_window_is_the_normalised_gaussian(oracle_mod):
    w = oracle_mod.ssim_window()
    ref = windows.gaussian(11, 1.5)
    np.testing.assert_allclose(w, ref / ref.sum(), rtol=1e-14)


def test_ssim_of_an_image_with_itself_is_one(oracle_mod):
    rng = np.random.default_rng(0)
    x = rng.uniform(0, 1, size=(1, 3, 19, 23))
    loss, g, smap = oracle_mod.l1_dssim(x, x, 0.2, with_map=True)
    np.testing.assert_allclose(smap, 1.0, atol=1e-12)
    assert abs(loss) < 1e-12
    np.testing.assert_allclose(g, 0.0, atol=1e-12)


def test_constant_images_closed_form_in_the_interior(oracle_mod):
    a, b = 0.3, 0.7
    x = np.full((1, 1, 30, 30), a)
    y = np.full((1, 1, 30, 30), b)
    _, _, smap = oracle_mod.l1_dssim(x, y, 0.2, with_map=True)
    C1 = 1e-4
    expect = (2 * a * b + C1) / (a * a + b * b + C1)  # variances 0: second factor 1
    np.testing.assert_allclose(smap[0, 0, 5:25, 5:25], expect, rtol=1e-12)


def test_ssim_map_equals_scipy_convolution_route(oracle_mod):
    rng = np.random.default_rng(1)
    x = rng.uniform(0, 1, size=(1, 2, 21, 17))
    y = np.clip(x + rng.normal(0, 0.1, size=x.shape), 0, 1)
    _, _, smap = oracle_mod.l1_dssim(x, y, 0.2, with_map=True)
    g1 = windows.gaussian(11, 1.5)
    w = np.outer(g1, g1) / g1.sum() ** 2
    C1, C2 = 1e-4, 9e-4
    for pl in range(2):
        f = lambda a: ndimage.correlate(a, w, mode="constant", cval=0.0)  # noqa: E731
        xx, yy = x[0, pl], y[0, pl]
        mx, my = f(xx), f(yy)
        sxx, syy, sxy = f(xx * xx) - mx * mx, f(yy * yy) - my * my, f(xx * yy) - mx * my
        S = ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))
        np.testing.assert_allclose(smap[0, pl], S, rtol=1e-11, atol=1e-13)


@pytest.mark.parametrize("lam", [0.2, 1.0])
def test_gradient_matches_central_differences(oracle_mod, lam):
    rng = np.random.default_rng(2)
    x = rng.uniform(0.1, 0.9, size=(2, 3, 13, 15))
    y = rng.uniform(0.1, 0.9, size=x.shape)
    loss, g = oracle_mod.l1_dssim(x, y, lam)
    for _ in range(40):
        idx = tuple(int(rng.integers(s)) for s in x.shape)
        h = 1e-6
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (oracle_mod.l1_dssim(xp, y, lam)[0] - oracle_mod.l1_dssim(xm, y, lam)[0]) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-6 * abs(g[idx]) + 1e-9, (idx, fd, g[idx])


def test_lambda_zero_is_the_l1_term(oracle_mod):
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 1, size=(1, 3, 9, 9))
    y = rng.uniform(0, 1, size=x.shape)
    l0, g0 = oracle_mod.l1_dssim(x, y, 0.0)
    l1, g1 = oracle_mod.l1(x, y)
    assert abs(l0 - l1) < 1e-14
    np.testing.assert_allclose(g0, g1, atol=1e-15)
