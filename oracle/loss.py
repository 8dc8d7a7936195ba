"""Oracle photometric loss (FP64, torch on the CPU). Test infrastructure only.

Eq. 6: L = (1 - lambda) L1 + lambda (1 - SSIM) with lambda = 0.2, SSIM as in
Wang et al. 2004. The paper fixes lambda and cites SSIM; the remaining
details are readings:

* L1 = mean |C - C_hat| over the 3 H W values (derivative of |x| at 0 taken as 0);
* SSIM per channel with an 11 x 11 Gaussian window (sigma 1.5, normalised to
  sum 1), constants C1 = 0.01^2, C2 = 0.03^2 (dynamic range 1), "same" size
  filtering with zero padding, averaged over the 3 H W map values;
* no clamping of the rendered image before the loss.
"""
from __future__ import annotations

import math

import torch
import torch.nn.functional as F

DT = torch.float64
LAMBDA_DSSIM = 0.2
SSIM_C1 = 0.01 ** 2
SSIM_C2 = 0.03 ** 2
WINDOW = 11
SIGMA = 1.5


def gaussian_window_1d(size: int = WINDOW, sigma: float = SIGMA) -> torch.Tensor:
    k = torch.arange(size, dtype=DT) - (size // 2)
    g = torch.exp(-(k * k) / (2.0 * sigma * sigma))
    return g / g.sum()


def _filter(x: torch.Tensor) -> torch.Tensor:
    """Zero-padded 'same' 2D filtering of each channel of (3, H, W) with the
    11 x 11 window outer(g, g)."""
    g = gaussian_window_1d()
    w2 = torch.outer(g, g)
    ch = x.shape[0]
    weight = w2.expand(ch, 1, WINDOW, WINDOW).contiguous()
    return F.conv2d(x[None], weight, padding=WINDOW // 2, groups=ch)[0]


def ssim_map(x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    mu_x = _filter(x)
    mu_y = _filter(y)
    sxx = _filter(x * x) - mu_x * mu_x
    syy = _filter(y * y) - mu_y * mu_y
    sxy = _filter(x * y) - mu_x * mu_y
    num = (2.0 * mu_x * mu_y + SSIM_C1) * (2.0 * sxy + SSIM_C2)
    den = (mu_x * mu_x + mu_y * mu_y + SSIM_C1) * (sxx + syy + SSIM_C2)
    return num / den


def ssim(x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    return ssim_map(x, y).mean()


def l1(x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    return (x - y).abs().mean()


def photometric_loss(x, y, lam: float = LAMBDA_DSSIM) -> torch.Tensor:
    """Eq. 6 on planar images (3, H, W)."""
    x = torch.as_tensor(x, dtype=DT) if not isinstance(x, torch.Tensor) else x.to(DT)
    y = torch.as_tensor(y, dtype=DT) if not isinstance(y, torch.Tensor) else y.to(DT)
    return (1.0 - lam) * l1(x, y) + lam * (1.0 - ssim(x, y))


def photometric_loss_and_grad(x, y, lam: float = LAMBDA_DSSIM):
    """Loss value and dL/dx (same shape as x), float64."""
    xt = torch.tensor(x, dtype=DT, requires_grad=True) if not isinstance(x, torch.Tensor) \
        else x.detach().to(DT).clone().requires_grad_(True)
    L = photometric_loss(xt, y, lam)
    L.backward()
    return float(L.detach()), xt.grad.detach()
