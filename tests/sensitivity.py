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
* ``box_edge_sensitive``: pixels on the edge of the overlap box of a Gaussian
  that reaches alpha_min there, where FP32 may place the edge one pixel over;
* ``order_sensitive``: pixels where two consecutively blended Gaussians are
  tied in FP32 depth and their order matters to the colour;

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


def box_edge_sensitive(pr, xs, ys):
    """Pixels on the edge of the overlap box of a Gaussian that reaches
    alpha_min there, by the oracle's projection alone: the box half-widths are
    ceilings, which FP32 may round to the other integer when their argument
    lies within its FP32 error bound of one, and the centre carries the FP32
    rounding of the projection (a few ulps of |u|). The bound of each argument
    is taken from the arithmetic that forms it: the larger eigenvalue
    mid + sqrt(mid^2 - det) loses up to sqrt(eps) relative accuracy when the
    covariance is nearly isotropic (the difference under the root cancels),
    and sqrt(2 tau Sigma) is as uncertain as tau = ln(o / alpha_min) is
    relative to itself."""
    rp = R.RasterParams().as_f32()
    eps = 2.0 ** -24
    u, v = pr["uv"][:, 0].numpy(), pr["uv"][:, 1].numpy()
    a, b, c = (pr["conic"][:, k].numpy() for k in range(3))
    o = pr["opacity"].numpy()
    ext = np.asarray(pr["extent"]).reshape(-1, 2).astype(np.float64)
    cov = pr["cov2d"].numpy()
    mid = 0.5 * (cov[:, 0] + cov[:, 2])
    det = cov[:, 0] * cov[:, 2] - cov[:, 1] ** 2
    root = np.sqrt(np.maximum(mid * mid - det, 0.0))
    lam = mid + root
    dlam = 16 * eps * mid + np.minimum(16 * eps * mid * mid / np.maximum(root, 1e-300),
                                       mid * np.sqrt(32 * eps))
    x0 = 3.0 * np.sqrt(lam)
    args = [(x0, 1.5 * dlam / np.sqrt(np.maximum(lam, 1e-300)) + 8 * eps * x0)]
    tau = np.log(np.maximum(o, 1e-300) / rp.alpha_min)
    t = np.maximum(tau, 0.0)
    dtau = 8 * eps * (1.0 + np.abs(np.log(np.maximum(o, 1e-300))) + abs(np.log(rp.alpha_min)))
    for s2 in (cov[:, 0], cov[:, 2]):
        x = np.sqrt(2.0 * t * s2)
        args.append((x, x * (16 * eps + dtau / (2.0 * np.maximum(t, 1e-300)))))
    # an argument x within its bound of the integer n may give the half-width
    # n or n + 1 in FP32: pixels at |d| in (n, n + 1] on its axes may flip
    # (the radius bounds both axes, the others one each)
    band = np.full((len(u), 2), -1.0)   # per axis: n of an unsure argument, -1: none
    for k, (x, dx) in enumerate(args):
        n = np.round(x)
        uns = np.abs(x - n) <= 2.0 * dx + 1e-12
        for ax in ((0, 1) if k == 0 else (k - 1,)):
            band[:, ax] = np.where(uns, n, band[:, ax])
    out = np.zeros(len(xs), bool)
    for k, (x, y) in enumerate(zip(xs + 0.5, ys + 0.5)):
        dx, dy = np.abs(x - u), np.abs(y - v)
        near = (dx <= ext[:, 0] + 1.0) & (dy <= ext[:, 1] + 1.0)
        if not near.any():
            continue
        i = np.nonzero(near)[0]
        tol_x = 4e-7 * (np.abs(u[i]) + 16.0) + 1e-5
        tol_y = 4e-7 * (np.abs(v[i]) + 16.0) + 1e-5
        on_edge = ((np.abs(dx[i] - ext[i, 0]) <= tol_x) & (dy[i] <= ext[i, 1] + tol_y)) | \
                  ((np.abs(dy[i] - ext[i, 1]) <= tol_y) & (dx[i] <= ext[i, 0] + tol_x))
        nx, ny = band[i, 0], band[i, 1]
        ring = ((nx >= 0) & (dx[i] > nx - tol_x) & (dx[i] <= nx + 1 + tol_x)) | \
               ((ny >= 0) & (dy[i] > ny - tol_y) & (dy[i] <= ny + 1 + tol_y))
        ddx, ddy = x - u[i], y - v[i]
        power = -0.5 * (a[i] * ddx * ddx + c[i] * ddy * ddy) - b[i] * ddx * ddy
        # the box decides only where the Gaussian reaches alpha_min (nearer
        # the threshold the oracle's threshold test already flags the pixel)
        reach = o[i] * np.exp(np.minimum(power, 0.0)) >= (1.0 - 1e-4) * rp.alpha_min
        out[k] = bool(((on_edge | ring) & reach).any())
    return out


def order_sensitive(pr, xs, ys, scale, fwd_tol, order_ulps=8):
    """Pixels at which two consecutively blended Gaussians have depths closer
    than order_ulps units in the last place of FP32 and swapping them would
    move the colour by more than half the tolerance: the GPU's FP32 depth may
    order such a pair the other way round than the oracle's FP64 depth."""
    rp = R.RasterParams().as_f32()
    u, v = pr["uv"][:, 0].numpy(), pr["uv"][:, 1].numpy()
    a, b, c = (pr["conic"][:, k].numpy() for k in range(3))
    o = pr["opacity"].numpy()
    col = pr["rgb"].numpy()
    d = pr["depth"].numpy()
    ext = np.asarray(pr["extent"]).reshape(-1, 2)
    out = np.zeros(len(xs), bool)
    # candidates per 16x16 pixel block first, then per pixel
    blocks = {}
    for k, (x, y) in enumerate(zip(xs, ys)):
        blocks.setdefault((x // 16, y // 16), []).append(k)
    for (bx, by), ks in blocks.items():
        x0, y0 = bx * 16 + 0.5, by * 16 + 0.5
        cand = np.nonzero((u + ext[:, 0] >= x0) & (u - ext[:, 0] <= x0 + 15) &
                          (v + ext[:, 1] >= y0) & (v - ext[:, 1] <= y0 + 15))[0]
        for k in ks:
            out[k] = _order_sensitive_pixel(xs[k] + 0.5, ys[k] + 0.5, cand, u, v, a, b, c, o,
                                            col, d, ext, rp, scale, fwd_tol, order_ulps)
    return out


def _order_sensitive_pixel(x, y, cand, u, v, a, b, c, o, col, d, ext, rp, scale, fwd_tol,
                           order_ulps):
    dx, dy = x - u[cand], y - v[cand]
    m = (np.abs(dx) <= ext[cand, 0]) & (np.abs(dy) <= ext[cand, 1])
    i, dx, dy = cand[m], dx[m], dy[m]
    p = -0.5 * (a[i] * dx ** 2 + c[i] * dy ** 2) - b[i] * dx * dy
    al = np.minimum(o[i] * np.exp(p), rp.alpha_max)
    keep = (p <= 0) & (al >= rp.alpha_min)
    i, al = i[keep], al[keep]
    order = np.lexsort((i, d[i].astype(np.float32)))
    i, al = i[order], al[order]
    t_after = np.cumprod(1.0 - al)
    bl = t_after >= rp.t_min
    i, al = i[bl], al[bl]
    if len(i) < 2:
        return False
    T = np.concatenate([[1.0], np.cumprod(1.0 - al)[:-1]])
    dd = d[i]
    gap = np.diff(dd)
    tol = order_ulps * np.spacing(dd[1:].astype(np.float32)).astype(np.float64)
    effect = al[:-1] * al[1:] * T[:-1] * np.abs(col[i[:-1]] - col[i[1:]]).max(1)
    return bool(((gap <= tol) & (effect > 0.5 * fwd_tol * scale)).any())


def oracle_view_masks(sc, cam, orp: R.RasterParams, rel: float, fwd_tol: float):
    """Oracle image ((3, H W) float64) of one view of scene ``sc`` and its
    masks of decision-sensitive pixels over the whole view: colour (may
    differ beyond half the forward tolerance) and last (the set of blended
    Gaussians may differ), from the threshold, depth-tie and box-edge tests."""
    with torch.no_grad():
        pr = R.project(*(torch.as_tensor(np.asarray(a, np.float64)) for a in
                         (sc.means, sc.log_scales, sc.quats, sc.opacity_logits, sc.sh)),
                       sc.sh_degree, cam, orp)

        def comp(rp_):
            return R.composite(pr["uv"], pr["conic"], pr["opacity"], pr["rgb"], pr["depth"],
                               pr["extent"], pr["ids"], cam.width, cam.height, rp_)

        out, sens = decision_sensitive(comp, orp, rel, fwd_tol)
    px, py = R.pixel_grid(cam.width, cam.height)
    xs, ys = px.numpy(), py.numpy()
    ref = out["rgb"].numpy()
    scale = max(float(np.abs(ref).max()), 1e-30)
    extra = order_sensitive(pr, xs, ys, scale, fwd_tol) | box_edge_sensitive(pr, xs, ys)
    return ref, sens["colour"] | extra, sens["last"] | extra
