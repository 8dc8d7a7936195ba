"""Which pixels the FP64 oracle itself calls decision-sensitive.

The forward takes discrete decisions per (pixel, Gaussian): skip below
alpha_min, stop before the transmittance falls below t_min, and the clamp at
alpha_max (which only changes the gradient). FP32 and FP64 arithmetic can
take a different decision only where the oracle's own result moves when the
threshold moves by a small relative amount. This module finds those pixels
with the oracle alone (nothing here looks at the GPU's answer):

* ``colour``: pixels whose colour moves by more than half the forward
  tolerance when alpha_min or t_min moves by +-rel;
* ``last``: pixels whose last blended Gaussian or blended count changes when
  alpha_min or t_min moves by +-rel;

(The alpha_max clamp only changes which gradient terms vanish; a flip needs
a raw alpha within a few FP32 ulps of alpha_max, about one (pixel, Gaussian)
pair in a million, and its effect stays within the gradient tolerance.)

Parity tests compare the GPU with the oracle on every other pixel and allow
no mismatch there.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from oracle import render as R


def decision_sensitive(composite, rp: R.RasterParams, rel: float, fwd_tol: float, base=None):
    """composite(rp) -> oracle composite dict for the pixels under test.
    Returns (base output, dict of boolean masks colour / last)."""
    with torch.no_grad():
        out = composite(rp) if base is None else base
        rgb = out["rgb"].detach().numpy()
        last = out["last"].numpy()
        nb = out["n_blended"].numpy()
        scale = max(float(np.abs(rgb).max()), 1e-30)
        colour = np.zeros(len(last), bool)
        dlast = np.zeros(len(last), bool)
        for f in (1.0 - rel, 1.0 + rel):
            variants = [dataclasses.replace(rp, t_min=rp.t_min * f)]
            if rp.alpha_min > 0:
                variants.append(dataclasses.replace(rp, alpha_min=rp.alpha_min * f))
            for v in variants:
                o = composite(v)
                colour |= np.abs(o["rgb"].detach().numpy() - rgb).max(0) > 0.5 * fwd_tol * scale
                dlast |= (o["last"].numpy() != last) | (o["n_blended"].numpy() != nb)
    return out, {"colour": colour, "last": dlast}
