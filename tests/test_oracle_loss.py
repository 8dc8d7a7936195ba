"""Pins for the oracle photometric loss (Eq. 6): identities, a closed form for
constant images under zero padding, an independent filter implementation and
finite differences."""
import math

import numpy as np
import pytest
import torch
from scipy import ndimage
from scipy.signal import windows

from oracle import loss as Lm

DT = torch.float64


def test_window_is_normalised_gaussian():
    g = Lm.gaussian_window_1d().numpy()
    ref = windows.gaussian(11, 1.5)
    assert np.allclose(g, ref / ref.sum(), rtol=0, atol=1e-16)


def test_ssim_of_image_with_itself_is_one():
    rng = np.random.default_rng(0)
    x = torch.tensor(rng.uniform(0, 1, (3, 23, 31)))
    assert Lm.ssim(x, x).item() == pytest.approx(1.0, abs=1e-15)
    assert Lm.photometric_loss(x, x).item() == pytest.approx(0.0, abs=1e-15)


def test_ssim_of_constant_images_closed_form():
    """For constant images a, b with zero padding every local statistic is a
    multiple of the in-image window mass m(p) = sx(x) sy(y):
    mu_x = a m, sigma_x^2 = a^2 (m - m^2), sigma_xy = a b (m - m^2)."""
    H, W, a, b = 17, 26, 0.7, 0.3
    g = Lm.gaussian_window_1d().numpy()

    def mass_1d(n):
        out = np.zeros(n)
        for i in range(n):
            for k in range(11):
                j = i + k - 5
                if 0 <= j < n:
                    out[i] += g[k]
        return out

    m = np.outer(mass_1d(H), mass_1d(W))
    C1, C2 = 0.01 ** 2, 0.03 ** 2
    v = m - m * m
    S = ((2 * a * b * m * m + C1) * (2 * a * b * v + C2)) / (((a * a + b * b) * m * m + C1) * ((a * a + b * b) * v + C2))
    x = torch.full((3, H, W), a, dtype=DT)
    y = torch.full((3, H, W), b, dtype=DT)
    got = Lm.ssim_map(x, y).numpy()
    assert np.abs(got - S[None]).max() < 1e-12


def test_ssim_matches_scipy_filtering():
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 1, (3, 19, 24))
    y = np.clip(x + rng.normal(0, 0.1, x.shape), 0, 1)
    g = Lm.gaussian_window_1d().numpy()
    w2 = np.outer(g, g)
    f = lambda z: ndimage.correlate(z, w2, mode="constant", cval=0.0)
    vals = []
    for c in range(3):
        mx, my = f(x[c]), f(y[c])
        sxx = f(x[c] * x[c]) - mx * mx
        syy = f(y[c] * y[c]) - my * my
        sxy = f(x[c] * y[c]) - mx * my
        vals.append(((2 * mx * my + 1e-4) * (2 * sxy + 9e-4)) / ((mx * mx + my * my + 1e-4) * (sxx + syy + 9e-4)))
    ref = float(np.mean(vals))
    assert Lm.ssim(torch.tensor(x), torch.tensor(y)).item() == pytest.approx(ref, abs=1e-14)
    l1 = np.abs(x - y).mean()
    assert Lm.photometric_loss(x, y).item() == pytest.approx(0.8 * l1 + 0.2 * (1 - ref), abs=1e-14)


def test_l1_derivative_at_zero_is_zero():
    x = torch.tensor(np.full((3, 12, 12), 0.5))
    y = x.clone()
    y[0, 3, 3] = 0.9
    _, g = Lm.photometric_loss_and_grad(x, y, lam=0.0)
    g = g.numpy()
    assert g[0, 3, 3] == pytest.approx(-1.0 / x.numel())
    assert np.all(g.reshape(-1)[np.arange(g.size) != 3 * 12 + 3] == 0.0)


def test_loss_gradient_matches_central_differences():
    rng = np.random.default_rng(6)
    x = rng.uniform(0.1, 0.9, (3, 15, 17))
    y = rng.uniform(0.1, 0.9, (3, 15, 17))
    _, g = Lm.photometric_loss_and_grad(x, y)
    g = g.numpy()
    h = 1e-6
    for _ in range(40):
        c, i, j = rng.integers(3), rng.integers(15), rng.integers(17)
        if abs(x[c, i, j] - y[c, i, j]) < 1e-4:
            continue
        xp, xm = x.copy(), x.copy()
        xp[c, i, j] += h; xm[c, i, j] -= h
        fd = (Lm.photometric_loss(xp, y).item() - Lm.photometric_loss(xm, y).item()) / (2 * h)
        assert fd == pytest.approx(g[c, i, j], rel=1e-6, abs=1e-12)
