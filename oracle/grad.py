"""Oracle gradients (FP64 autograd on the CPU). Test infrastructure only.

The gradient the training step needs is the exact derivative of the forward
(render, Eqs. 1-5; loss, Eq. 6) with respect to the raw parameters: means,
log-scales, the unnormalised quaternion, the opacity logit and the SH
coefficients. Every discrete decision of the forward (culling, tile overlap,
skip rules, termination, clamps) is held fixed, which is what autograd does
with the masks computed under ``no_grad``. No gradient flows through the
depth order, the radius or the tile rectangle.
"""
from __future__ import annotations

import numpy as np
import torch

from . import render as R
from . import loss as Lm

DT = torch.float64


def _leaf(x):
    return torch.tensor(np.asarray(x, dtype=np.float64), dtype=DT, requires_grad=True)


def render_vjp(scene_arrays: dict, sh_degree: int, cam, rp: R.RasterParams, dl_drgb,
               px=None, py=None):
    """Forward one view and pull back the cotangent ``dl_drgb`` ((3, n_px)
    matching the requested pixels). Returns (forward dict, grads dict)."""
    leaves = {k: _leaf(scene_arrays[k]) for k in
              ("means", "log_scales", "quats", "opacity_logits", "sh")}
    out = R.render(leaves["means"], leaves["log_scales"], leaves["quats"],
                   leaves["opacity_logits"], leaves["sh"], sh_degree, cam, rp, px=px, py=py)
    ct = torch.as_tensor(np.asarray(dl_drgb, dtype=np.float64), dtype=DT).reshape(out["rgb"].shape)
    s = (out["rgb"] * ct).sum()
    if s.requires_grad:
        s.backward()
    grads = {k: (v.grad.numpy().copy() if v.grad is not None else np.zeros(v.shape))
             for k, v in leaves.items()}
    return out, grads


def loss_and_grads(scene_arrays: dict, sh_degree: int, cam, rp: R.RasterParams, target):
    """Full image forward, Eq. 6 loss against ``target`` (3, H, W), and its
    gradient w.r.t. every raw parameter group and w.r.t. the image."""
    leaves = {k: _leaf(scene_arrays[k]) for k in
              ("means", "log_scales", "quats", "opacity_logits", "sh")}
    out = R.render(leaves["means"], leaves["log_scales"], leaves["quats"],
                   leaves["opacity_logits"], leaves["sh"], sh_degree, cam, rp)
    img = out["rgb"].reshape(3, cam.height, cam.width)
    img.retain_grad()
    L = Lm.photometric_loss(img, torch.as_tensor(np.asarray(target, dtype=np.float64)))
    L.backward()
    grads = {k: (v.grad.numpy().copy() if v.grad is not None else np.zeros(v.shape))
             for k, v in leaves.items()}
    return float(L.detach()), img.detach().numpy(), img.grad.numpy().copy(), grads, out


def scene_dict(scene) -> dict:
    return dict(means=scene.means, log_scales=scene.log_scales, quats=scene.quats,
                opacity_logits=scene.opacity_logits, sh=scene.sh)
