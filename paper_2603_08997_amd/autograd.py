"""torch.autograd wrappers over the C ABI: the render of a batch of views
(projection, binning and compositing, paper Sec. 3, Eqs. 1-5) and the
photometric loss (Eq. 6).

Argument marshalling only: every step runs in the library's kernels. The
render backward either keeps the forward workspace alive until the backward
(``recompute=False``) or frees it after the forward and runs the forward
again inside the backward (``recompute=True``), trading one forward for the
workspace memory (records, pair lists and per-pixel state) between the two
passes.
"""
from __future__ import annotations

import torch

from . import skipgs as sk


def _forward(planes, n, sh_degree, cams, rp, capacity):
    """Forward into a fresh workspace (one host synchronisation); on an
    overflow the pair capacity grows to the reported need and the forward runs
    again (twice at most: the tile-list need is exact once the super-tile pairs
    fit)."""
    px = sum(c.width * c.height for c in cams)
    rgb = torch.empty(3 * px, dtype=torch.float32, device=planes.device)
    for _ in range(3):
        ws = sk.alloc_bytes(sk.forward_workspace_size(rp, n, cams, capacity))
        sk.clear_status(ws)
        sk.render_forward(planes, n, sh_degree, cams, rp, ws, capacity, rgb)
        flags, _, pairs = sk.read_status(ws)
        if not flags & sk.STATUS_PAIR_OVERFLOW:
            return rgb, ws, capacity
        capacity = int(pairs * 1.05) + 4096
        del ws
    raise RuntimeError("pair capacity still exceeded after resizing")


class RenderFn(torch.autograd.Function):
    """planes [F][stride] -> planar image [3][sum of H*W over the views]."""

    @staticmethod
    def forward(ctx, planes, n, sh_degree, cams, rp, capacity, recompute):
        rgb, ws, capacity = _forward(planes, n, sh_degree, cams, rp, capacity)
        ctx.save_for_backward(planes)
        ctx.meta = (n, sh_degree, cams, rp, capacity)
        ctx.ws = None if recompute else ws
        return rgb

    @staticmethod
    def backward(ctx, g_rgb):
        (planes,) = ctx.saved_tensors
        n, sh_degree, cams, rp, capacity = ctx.meta
        ws = ctx.ws
        if ws is None:
            _, ws, capacity = _forward(planes, n, sh_degree, cams, rp, capacity)
        grads = torch.zeros_like(planes)
        sk.render_backward(planes, n, sh_degree, cams, rp, ws, capacity, g_rgb.contiguous(),
                           None, grads)
        ctx.ws = None
        return grads, None, None, None, None, None, None


def render(planes: torch.Tensor, n: int, sh_degree: int, cams, rp: sk.RasterParams | None = None,
           capacity: int | None = None, recompute: bool = True) -> torch.Tensor:
    """Differentiable render of ``cams`` (one launch for all views).
    ``capacity``: (tile, Gaussian) pairs to reserve; by default 16 per
    Gaussian and view, grown once if the forward reports more."""
    rp = rp or sk.RasterParams()
    capacity = capacity or max(4096, 16 * n * len(cams))
    return RenderFn.apply(planes, n, sh_degree, list(cams), rp, int(capacity), bool(recompute))


class LossFn(torch.autograd.Function):
    """Eq. 6 on one planar image [3][H][W]: 0.8 L1 + 0.2 (1 - SSIM)."""

    @staticmethod
    def forward(ctx, rgb, target, width, height, lam):
        lws = sk.alloc_bytes(sk.loss_workspace_size(width, height))
        out = torch.empty(1, dtype=torch.float32, device=rgb.device)
        sk.photometric_loss(rgb, target, width, height, lam, lws, out)
        ctx.save_for_backward(rgb, target)
        ctx.meta = (width, height, lam, lws)
        return out[0]

    @staticmethod
    def backward(ctx, g):
        rgb, target = ctx.saved_tensors
        width, height, lam, lws = ctx.meta
        dl = torch.empty_like(rgb)
        sk.photometric_loss_backward(rgb, target, width, height, lam, lws, None, dl)
        if not (g.numel() == 1 and float(g) == 1.0):
            dl = dl * g
        return dl, None, None, None, None


def photometric_loss(rgb: torch.Tensor, target: torch.Tensor, width: int, height: int,
                     lam: float = 0.2) -> torch.Tensor:
    return LossFn.apply(rgb.contiguous(), target.contiguous(), int(width), int(height),
                        float(lam))
