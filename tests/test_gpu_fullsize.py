"""Parity at full size: the single-view configurations (1M Gaussians at
1245x825, 3M at 1600x1060, the dense 6M cluster at 1600x1060) and the batched
launch (2M Gaussians, eight views of four resolutions in one launch), run
through the C ABI with 16x16 tiles as the benchmark runs them.

The oracle cannot composite millions of pixels, so the checks use outputs it
can compute one by one:
* forward: sampled pixels (random, plus tile-border pixels): the last blended
  Gaussian must agree exactly, and colour and final transmittance to the
  forward tolerance, on every pixel the oracle does not itself call
  decision-sensitive. The oracle's own sensitivity tests: the skip or
  termination threshold moved by a small relative amount changes the pixel;
  two Gaussians the pixel blends lie within a few FP32 ulps in depth; or the
  pixel sits on the edge of an overlap box of a Gaussian that reaches
  alpha_min there (the box half-widths are ceilings, and u, v carry FP32
  rounding);
* backward: a cotangent that is nonzero only in a 32x32 pixel window (less
  its decision-sensitive pixels). Only the Gaussians reaching the window get
  a nonzero gradient, so the oracle's gradient of that window equals the full
  gradient; every parameter group of all N Gaussians is compared (norm and
  maximum), zeros included.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

from oracle import grad as G
from oracle import render as R
from paper_2603_08997_amd import scenes as S

from .gpu_util import (last_blended, tile_lists, region, rel_max_err, rel_norm_err,
                       require_gpu, say, sg, to_dev)
from .sensitivity import decision_sensitive

pytestmark = pytest.mark.gpu

FWD_TOL = 1e-5
GRAD_TOL = 1e-3
DECISION_REL = 3e-5
ORDER_ULPS = 8
WIN = 32


def _config(name):
    if name == "n1M_1245x825":
        return S.mixture_scene(S.SEED_SCENE, 1_000_000, 3), \
            S.hemisphere_cameras(S.SEED_CAMERAS, 150, 1245, 825)[:1]
    if name == "n3M_1600x1060":
        return S.mixture_scene(S.SEED_SCENE, 3_000_000, 3), \
            S.hemisphere_cameras(S.SEED_CAMERAS, 200, 1600, 1060)[:1]
    if name == "dense6M_1600x1060":
        return S.dense_cluster_scene(S.SEED_SCENE, 6_000_000, 3), \
            S.hemisphere_cameras(S.SEED_CAMERAS, 1, 1600, 1060)
    if name == "n2M_batched8":
        return S.mixture_scene(S.SEED_SCENE, 2_000_000, 3), S.batched_cameras()
    raise KeyError(name)


CONFIGS = ["n1M_1245x825", "n3M_1600x1060", "dense6M_1600x1060", "n2M_batched8"]


class FullRender:
    """Forward of one configuration with a pair capacity sized by probe
    launches (a forward reports the capacity it needed: first the super-tile
    pairs, then, with those stored, the tile-list entries)."""

    def __init__(self, name):
        m = sg()
        self.m = m
        self.scene, self.cams = _config(name)
        self.n = self.scene.n
        self.rp = m.RasterParams()
        self.planes = to_dev(self.scene.to_planes())
        self.px = sum(c.width * c.height for c in self.cams)
        self.rgb = torch.zeros(3 * self.px, dtype=torch.float32, device="cuda")
        cap = 1 << 16
        for _ in range(3):
            ws = m.alloc_bytes(m.forward_workspace_size(self.rp, self.n, self.cams, cap)).zero_()
            m.render_forward(self.planes, self.n, 3, self.cams, self.rp, ws, cap, self.rgb)
            flags, _, pairs = m.read_status(ws)
            del ws
            if not flags & m.STATUS_PAIR_OVERFLOW:
                break
            cap = int(pairs * 1.02) + 4096
        self.cap = cap
        self.ws = m.alloc_bytes(m.forward_workspace_size(self.rp, self.n, self.cams, self.cap))
        self.ws.zero_()
        self.L = m.get_workspace_layout(self.rp, self.n, self.cams, self.cap)
        m.render_forward(self.planes, self.n, 3, self.cams, self.rp, self.ws, self.cap, self.rgb)
        flags, self.visible, self.pairs = m.read_status(self.ws)
        assert flags == 0, flags
        cnt = m.read_counters(self.ws)
        self.blended = cnt["blended"]
        torch.cuda.synchronize()
        self.rgb_np = self.rgb.cpu().numpy()
        self.tf = region(self.ws, self.L.t_final, self.L.total_pixels, np.float32)
        self.nl = region(self.ws, self.L.n_last, self.L.total_pixels, np.uint32)
        self.lists = tile_lists(self.ws, self.L)
        # per entry: projected centre and overlap box (0 where not visible)
        rec = region(self.ws, self.L.records, 12 * self.L.entries, np.float32).reshape(-1, 12)
        vis = region(self.ws, self.L.tiles, self.L.entries, np.uint32) != 0
        self.uv = rec[:, 0:2].copy()
        self.ext = np.where(vis[:, None], rec[:, 6:8], 0.0).astype(np.int64)
        del rec
        say(f"  n={self.n} views={len(self.cams)} visible={self.visible} pairs={self.pairs} "
            f"blended/px={self.blended / self.px:.1f}")

    def view_offsets(self, v):
        px_off = sum(c.width * c.height for c in self.cams[:v])
        tile_off = sum(((c.width + 15) // 16) * ((c.height + 15) // 16) for c in self.cams[:v])
        return px_off, tile_off

    def gpu_pixels(self, v, xs, ys):
        """Colour (3, k), final transmittance and last blended Gaussian index
        (-1: none) of pixels (xs, ys) of view v."""
        cam = self.cams[v]
        px_off, tile_off = self.view_offsets(v)
        pix = ys * cam.width + xs
        plane = cam.width * cam.height
        base = 3 * px_off
        rgb = np.stack([self.rgb_np[base + c * plane + pix] for c in range(3)])
        nl = self.nl[px_off + pix].astype(np.int64)
        tiles = tile_off + (ys // 16) * ((cam.width + 15) // 16) + xs // 16
        g = last_blended(self.lists, nl, tiles)
        last = np.where(g >= 0, g - v * self.n, -1)
        return rgb, self.tf[px_off + pix], last


_proj = {}


@pytest.fixture(scope="module", params=CONFIGS)
def fr(request):
    """One configuration at a time (pytest groups the tests by it)."""
    require_gpu()
    _proj.clear()
    torch.cuda.empty_cache()
    say(f"full-size {request.param}")
    r = FullRender(request.param)
    yield r
    _proj.clear()
    del r
    torch.cuda.empty_cache()


def _box_edge_sensitive(pr, xs, ys):
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


def _order_sensitive(pr, xs, ys, scale):
    """Pixels at which two consecutively blended Gaussians have depths closer
    than ORDER_ULPS units in the last place of FP32 and swapping them would
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
                                            col, d, ext, rp, scale)
    return out


def _order_sensitive_pixel(x, y, cand, u, v, a, b, c, o, col, d, ext, rp, scale):
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
    tol = ORDER_ULPS * np.spacing(dd[1:].astype(np.float32)).astype(np.float64)
    effect = al[:-1] * al[1:] * T[:-1] * np.abs(col[i[:-1]] - col[i[1:]]).max(1)
    return bool(((gap <= tol) & (effect > 0.5 * FWD_TOL * scale)).any())


def _oracle_pixels(scene, cam, xs, ys):
    """Oracle colour, final transmittance and last blended Gaussian of the
    given pixels (the projection of the view is computed once and kept), and
    the oracle's own masks of decision-sensitive pixels (colour: the colour
    may differ beyond half the tolerance; last: the last blended Gaussian may
    differ)."""
    key = (id(scene), id(cam))
    if key not in _proj:
        if len(_proj) > 1:
            _proj.clear()
        say(f"  oracle projection of {scene.n} Gaussians, {cam.width}x{cam.height}")
        arrs = [torch.as_tensor(np.asarray(a, np.float64)) for a in
                (scene.means, scene.log_scales, scene.quats, scene.opacity_logits, scene.sh)]
        with torch.no_grad():
            _proj[key] = R.project(*arrs, scene.sh_degree, cam, R.RasterParams())
    pr = _proj[key]

    def comp(rp):
        with torch.no_grad():
            return R.composite(pr["uv"], pr["conic"], pr["opacity"], pr["rgb"], pr["depth"],
                               pr["extent"], pr["ids"], cam.width, cam.height, rp,
                               px=xs, py=ys)

    out, sens = decision_sensitive(comp, R.RasterParams(), DECISION_REL, FWD_TOL)
    rgb = out["rgb"].numpy()
    scale = max(np.abs(rgb).max(), 1e-30)
    osens = _order_sensitive(pr, xs, ys, scale)
    bsens = _box_edge_sensitive(pr, xs, ys)
    say(f"  oracle-sensitive pixels: thresholds {int(sens['last'].sum())}, depth ties "
        f"{int(osens.sum())}, box edges {int(bsens.sum())} of {len(xs)}")
    colour = sens["colour"] | osens | bsens
    last = sens["last"] | osens | bsens
    return rgb, out["T_final"].numpy(), out["last"].numpy(), colour, last


def _samples(cam, k, seed):
    rng = np.random.default_rng(seed)
    xs = rng.integers(0, cam.width, k)
    ys = rng.integers(0, cam.height, k)
    # pixels on both sides of tile borders and at the image edges
    bx = np.array([15, 16, 31, 32, cam.width - 1, 0, (cam.width // 16) * 16 - 1])
    by = np.array([16, 15, 32, 31, cam.height - 1, 0, (cam.height // 16) * 16 - 1])
    bx = np.clip(bx, 0, cam.width - 1)
    by = np.clip(by, 0, cam.height - 1)
    return np.concatenate([xs, bx]), np.concatenate([ys, by])


def test_fullsize_forward_sampled_pixels(fr):
    k = 256 if len(fr.cams) == 1 else 64
    excl = total = 0
    for v, cam in enumerate(fr.cams):
        xs, ys = _samples(cam, k, 100 + v)
        g_rgb, g_t, g_last = fr.gpu_pixels(v, xs, ys)
        o_rgb, o_t, o_last, s_col, s_last = _oracle_pixels(fr.scene, cam, xs, ys)
        # no unexplained mismatch: every pixel the oracle does not call
        # sensitive has the same last blended Gaussian
        bad = (g_last != o_last) & ~s_last
        assert not bad.any(), (v, np.nonzero(bad)[0][:5], g_last[bad][:5], o_last[bad][:5])
        ok = ~s_col
        excl += int(s_col.sum())
        total += len(xs)
        assert rel_max_err(g_rgb[:, ok], o_rgb[:, ok]) <= FWD_TOL
        # T_final lies in [0, 1]; on pixels the Gaussians saturate it is
        # ~1e-4 and its relative error grows with the number of blended
        # factors, so the tolerance is taken against the range of the tensor
        err_t = np.abs(g_t[ok] - o_t[ok]).max()
        assert err_t <= FWD_TOL * max(1.0, np.abs(o_t).max()), (v, err_t)
    say(f"  {total} sampled pixels, {excl} decision-sensitive by the oracle")
    assert excl <= max(3, total // 20)


def _window_pixels(fr, v):
    """The pixels of a WIN x WIN window at the centre of view v, without the
    pixels the oracle calls decision-sensitive: the cotangent is zero there,
    so a decision that flips between FP32 and FP64 contributes nothing on
    either side. Elsewhere the last blended Gaussian must agree."""
    cam = fr.cams[v]
    x0, y0 = cam.width // 2 - WIN // 2, cam.height // 2 - WIN // 2
    ys, xs = np.meshgrid(np.arange(y0, y0 + WIN), np.arange(x0, x0 + WIN), indexing="ij")
    xs, ys = xs.reshape(-1), ys.reshape(-1)
    _, _, g_last = fr.gpu_pixels(v, xs, ys)
    _, _, o_last, _, s_last = _oracle_pixels(fr.scene, cam, xs, ys)
    assert not ((g_last != o_last) & ~s_last).any()
    keep = ~s_last
    say(f"  window of view {v}: {int((~keep).sum())} of {len(xs)} pixels sensitive")
    # (at the centre of the dense cluster hundreds of Gaussians overlap each
    # pixel, and about one pixel in ten lies on a box edge that FP32 may move)
    assert keep.mean() >= 0.8
    return xs[keep], ys[keep]


def test_fullsize_backward_window(fr):
    views = [0] if len(fr.cams) == 1 else [1, 5]
    dl = np.zeros(3 * fr.px, np.float32)
    ref = None
    for v in views:
        cam = fr.cams[v]
        xs, ys = _window_pixels(fr, v)
        ct = np.random.default_rng(300 + v).normal(0.0, 1.0, (3, len(xs))).astype(np.float32)
        px_off, _ = fr.view_offsets(v)
        plane = cam.width * cam.height
        for c in range(3):
            dl[3 * px_off + c * plane + ys * cam.width + xs] = ct[c]
        say(f"  oracle gradient of a {WIN}x{WIN} window of view {v}")
        _, g = G.render_vjp(G.scene_dict(fr.scene), 3, cam, R.RasterParams(),
                            ct.astype(np.float64), px=xs, py=ys)
        ref = g if ref is None else {k: ref[k] + g[k] for k in g}
    grads = torch.zeros_like(fr.planes)
    fr.m.render_backward(fr.planes, fr.n, 3, fr.cams, fr.rp, fr.ws, fr.cap, to_dev(dl), None,
                         grads)
    torch.cuda.synchronize()
    got = S.Scene.from_planes(grads.cpu().numpy(), fr.n, 3)
    touched = int((np.abs(ref["means"]).sum(1) > 0).sum())
    say(f"  window gradient reaches {touched} Gaussians")
    assert touched > 0
    pairs = [("means", got.means, ref["means"]), ("log_scales", got.log_scales, ref["log_scales"]),
             ("quats", got.quats, ref["quats"]),
             ("opacity", got.opacity_logits, ref["opacity_logits"]), ("sh", got.sh, ref["sh"])]
    for k, a, b in pairs:
        assert rel_norm_err(a, b) <= GRAD_TOL, (k, rel_norm_err(a, b))
        assert rel_max_err(a, b) <= GRAD_TOL, (k, rel_max_err(a, b))
