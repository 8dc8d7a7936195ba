"""Oracle renderer (FP64, torch on the CPU). Test infrastructure only.

Follows Sec. 3 of the paper: Gaussian density (Eq. 1), covariance
factorisation Sigma = R S S^T R^T (Eq. 2), EWA projection
Sigma2D = J W Sigma W^T J^T (Eq. 3), and front-to-back compositing
C(p) = sum_i c_i alpha'_i T_i with T_i = prod_{j<i} (1 - alpha'_j) (Eq. 4), i
running in depth order over the Gaussians that cover p, with the effective
opacity alpha'_i = alpha_i exp(-1/2 dp^T (Sigma2D)^-1 dp) (Eq. 5); c_i is the
spherical-harmonic expansion of Gaussian i evaluated at the viewing direction
(Sec. 3).

The paper leaves the camera model, culling, the screen-space low-pass, the
cut-off radius, the SH basis, the overlap rule and the opacity/transmittance
thresholds unstated; the readings used here (fixed in ``RasterParams``) are:

* pinhole camera, OpenCV axes; pixel (x, y) has centre (x + 0.5, y + 0.5);
* near-plane cull at camera depth <= near;
* quaternion (w, x, y, z) normalised before use; scale = exp(log-scale);
  opacity = sigmoid(logit);
* W of Eq. 3 is the world-to-camera rotation; J is the Jacobian of the
  perspective map at the Gaussian centre, with tx/tz and ty/tz clamped to
  +-jac_clamp * (image half-extent) / focal (0 disables the clamp);
* Sigma2D gets a low-pass dilation h * I; det <= 0 culls;
* radius r = ceil(3 sqrt(lambda_max(Sigma2D))) pixels;
* a Gaussian overlaps pixel p iff |p_x - u| <= r_x and |p_y - v| <= r_y with
  r_x = min(r, ceil(sqrt(2 ln(o/alpha_min) Sigma2D_xx))), r_y likewise with
  Sigma2D_yy: outside that box (p - mu)^T Sigma2D^-1 (p - mu) > 2 ln(o/alpha_min),
  so o exp(P) < alpha_min and the pixel would skip the Gaussian anyway. With
  alpha_min = 0 the box is the square r_x = r_y = r; a Gaussian with
  o < alpha_min overlaps nothing;
* Gaussians whose centre or radius exceeds 2^24 pixels are degenerate and culled;
* alpha' = min(alpha_max, o exp(P)), P = -1/2 dp^T conic dp; P > 0 or
  alpha' < alpha_min skips the Gaussian for that pixel; compositing stops
  before a Gaussian that would take the transmittance below t_min;
* background colour bg is added with weight T_final;
* the depth order is that of the float32 camera depth; ties (equal float32
  depths) are broken by ascending Gaussian index.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

DT = torch.float64


def f32(x: float) -> float:
    """The float32 value of a constant, as the FP32 kernels see it."""
    return float(np.float32(x))


@dataclass
class RasterParams:
    tile_w: int = 16
    tile_h: int = 16
    bg: tuple = (0.0, 0.0, 0.0)
    near: float = 0.2
    dilation: float = 0.3
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    t_min: float = 1e-4
    jac_clamp: float = 1.3

    def as_f32(self) -> "RasterParams":
        """Thresholds rounded to float32, the values the FP32 kernels compare against."""
        return RasterParams(self.tile_w, self.tile_h, tuple(f32(b) for b in self.bg),
                            f32(self.near), f32(self.dilation), f32(self.alpha_min),
                            f32(self.alpha_max), f32(self.t_min), f32(self.jac_clamp))


def smooth_params(**kw) -> RasterParams:
    """Thresholds disabled (alpha_min = 0, t_min = 0, alpha_max = 1): the forward
    is then smooth in every parameter apart from overlap, which finite
    differences can check."""
    base = dict(alpha_min=0.0, t_min=0.0, alpha_max=1.0)
    base.update(kw)
    return RasterParams(**base)


# ---------------------------------------------------------------------------
# Spherical harmonics (colour as a function of view direction, Sec. 3)
# ---------------------------------------------------------------------------
# Real SH with the Condon-Shortley phase, index k = l^2 + l + m, direction
# d = (x, y, z): the normalisation constants of Y_l^m for l <= 3.
SH_C0 = 0.28209479177387814
SH_C1 = 0.4886025119029199
SH_C2 = (1.0925484305920792, -1.0925484305920792, 0.31539156525252005,
         -1.0925484305920792, 0.5462742152960396)
SH_C3 = (-0.5900435899266435, 2.890611442640554, -0.4570457994644658,
         0.3731763325901154, -0.4570457994644658, 1.445305721320277,
         -0.5900435899266435)
SH_OFFSET = 0.5


def sh_basis(d: torch.Tensor, degree: int) -> torch.Tensor:
    """Y_k(d) for k < (degree+1)^2; d is (N, 3) unit vectors. Returns (N, K)."""
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    out = [torch.full_like(x, SH_C0)]
    if degree >= 1:
        out += [-SH_C1 * y, SH_C1 * z, -SH_C1 * x]
    if degree >= 2:
        xx, yy, zz = x * x, y * y, z * z
        out += [SH_C2[0] * x * y,
                SH_C2[1] * y * z,
                SH_C2[2] * (2.0 * zz - xx - yy),
                SH_C2[3] * x * z,
                SH_C2[4] * (xx - yy)]
    if degree >= 3:
        out += [SH_C3[0] * y * (3.0 * xx - yy),
                SH_C3[1] * x * y * z,
                SH_C3[2] * y * (4.0 * zz - xx - yy),
                SH_C3[3] * z * (2.0 * zz - 3.0 * xx - 3.0 * yy),
                SH_C3[4] * x * (4.0 * zz - xx - yy),
                SH_C3[5] * z * (xx - yy),
                SH_C3[6] * x * (xx - 3.0 * yy)]
    return torch.stack(out, dim=1)


# ---------------------------------------------------------------------------
# Covariance (Eq. 2) and projection (Eq. 3)
# ---------------------------------------------------------------------------
def quat_to_rotation(q: torch.Tensor) -> torch.Tensor:
    """Rotation matrix of the unit quaternion q / |q|, q = (w, x, y, z). (N, 3, 3)."""
    qn = q / torch.linalg.norm(q, dim=1, keepdim=True)
    w, x, y, z = qn.unbind(1)
    rows = [
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], 1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], 1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], 1),
    ]
    return torch.stack(rows, dim=1)


def covariance_3d(log_scales: torch.Tensor, quats: torch.Tensor) -> torch.Tensor:
    """Sigma = R S S^T R^T with S = diag(exp(log_scale)) (Eq. 2). (N, 3, 3)."""
    R = quat_to_rotation(quats)
    M = R * torch.exp(log_scales)[:, None, :]      # R S
    return M @ M.transpose(1, 2)


def camera_tensors(cam):
    R = torch.as_tensor(np.asarray(cam.R, dtype=np.float64), dtype=DT)
    t = torch.as_tensor(np.asarray(cam.t, dtype=np.float64), dtype=DT)
    return R, t


def camera_centre(cam) -> torch.Tensor:
    R, t = camera_tensors(cam)
    return -(R.T @ t)


def _t(x):
    if isinstance(x, torch.Tensor):
        return x.to(DT)
    return torch.as_tensor(np.asarray(x, dtype=np.float64), dtype=DT)


def project(means, log_scales, quats, opacity_logits, sh, sh_degree: int, cam,
            rp: RasterParams) -> dict:
    """Project every Gaussian into camera ``cam``.

    Returns a dict over the *visible* Gaussians (ascending index ``ids``):
    ``uv`` (n,2), ``depth`` (n,), ``cov2d`` (n,3) = (xx, xy, yy) incl. dilation,
    ``conic`` (n,3) = (a, b, c) of the inverse, ``radius`` (n,) int64,
    ``extent`` (n,2) int64 = (r_x, r_y) of the overlap box,
    ``opacity`` (n,), ``rgb`` (n,3), ``rgb_raw`` (n,3) before the clamp at 0.
    Tensors keep autograd history to the inputs.
    """
    means, log_scales, quats = _t(means), _t(log_scales), _t(quats)
    opacity_logits, sh = _t(opacity_logits), _t(sh)
    rp = rp.as_f32()
    n = means.shape[0]
    Rc, tc = camera_tensors(cam)
    fx, fy, cx, cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    W_img, H_img = int(cam.width), int(cam.height)

    with torch.no_grad():
        tz_all = means @ Rc[2] + tc[2]
        qnorm = torch.linalg.norm(quats, dim=1)
        finite = (torch.isfinite(means).all(1) & torch.isfinite(log_scales).all(1)
                  & torch.isfinite(quats).all(1) & torch.isfinite(opacity_logits)
                  & torch.isfinite(sh.reshape(n, -1)).all(1))
        keep = (tz_all > rp.near) & finite & (qnorm > 0)
    idx = torch.nonzero(keep).flatten()

    mu = means[idx]
    tcam = mu @ Rc.T + tc
    tx, ty, tz = tcam[:, 0], tcam[:, 1], tcam[:, 2]

    # EWA Jacobian (Eq. 3) with the clamp on tx/tz, ty/tz.
    xr, yr = tx / tz, ty / tz
    if rp.jac_clamp > 0:
        lim_x = rp.jac_clamp * (W_img / 2.0) / fx
        lim_y = rp.jac_clamp * (H_img / 2.0) / fy
        xr = torch.clamp(xr, -lim_x, lim_x)
        yr = torch.clamp(yr, -lim_y, lim_y)
    zero = torch.zeros_like(tz)
    J = torch.stack([
        torch.stack([fx / tz, zero, -fx * xr / tz], 1),
        torch.stack([zero, fy / tz, -fy * yr / tz], 1)], dim=1)       # (n, 2, 3)
    Sigma = covariance_3d(log_scales[idx], quats[idx])
    T = J @ Rc                                                         # J W
    S2 = T @ Sigma @ T.transpose(1, 2)
    sxx = S2[:, 0, 0] + rp.dilation
    sxy = S2[:, 0, 1]
    syy = S2[:, 1, 1] + rp.dilation
    det = sxx * syy - sxy * sxy

    u = fx * tx / tz + cx
    v = fy * ty / tz + cy

    with torch.no_grad():
        mid = 0.5 * (sxx + syy)
        lam = mid + torch.sqrt(torch.clamp(mid * mid - det, min=0.0))
        rf = torch.ceil(3.0 * torch.sqrt(torch.clamp(lam, min=0.0)))
        ok = (det > 0) & torch.isfinite(u) & torch.isfinite(v) & torch.isfinite(rf)
        ok &= (u.abs() < MAX_EXTENT) & (v.abs() < MAX_EXTENT) & (rf < MAX_EXTENT)
        radius = torch.where(ok, rf, torch.zeros_like(rf)).to(torch.int64)
        o_all = torch.sigmoid(opacity_logits[idx])
        ext = overlap_extent(radius, o_all, sxx, syy, rp.alpha_min)
        ok &= ext[:, 0] >= 0
        tiles_x = (W_img + rp.tile_w - 1) // rp.tile_w
        tiles_y = (H_img + rp.tile_h - 1) // rp.tile_h
        x0, x1, y0, y1 = tile_rect(u, v, ext, rp.tile_w, rp.tile_h, tiles_x, tiles_y)
        ok &= (x1 > x0) & (y1 > y0)
    sel = torch.nonzero(ok).flatten()

    det_s = det[sel]
    conic = torch.stack([syy[sel] / det_s, -sxy[sel] / det_s, sxx[sel] / det_s], 1)

    # SH colour for the direction from the camera centre to the Gaussian.
    mu_s = mu[sel]
    dirs = mu_s - camera_centre(cam)
    d = dirs / torch.linalg.norm(dirs, dim=1, keepdim=True)
    Y = sh_basis(d, sh_degree)                                          # (n, K)
    coeffs = sh[idx][sel]                                               # (n, K, 3)
    rgb_raw = (Y[:, :, None] * coeffs).sum(1) + SH_OFFSET
    rgb = torch.clamp(rgb_raw, min=0.0)

    opacity = torch.sigmoid(opacity_logits[idx][sel])
    return dict(ids=idx[sel], uv=torch.stack([u[sel], v[sel]], 1), depth=tz[sel],
                cov2d=torch.stack([sxx[sel], sxy[sel], syy[sel]], 1), conic=conic,
                radius=radius[sel], extent=ext[sel], opacity=opacity, rgb=rgb, rgb_raw=rgb_raw,
                tiles_x=tiles_x, tiles_y=tiles_y)


# ---------------------------------------------------------------------------
# Tile binning: the order-defining step of the tile-based rasteriser
# ---------------------------------------------------------------------------
MAX_EXTENT = float(2 ** 24)


def overlap_extent(radius, opacity, sxx, syy, alpha_min):
    """(r_x, r_y) of the overlap box: min(r, ceil(sqrt(2 ln(o/alpha_min) Sigma_xx)))
    and likewise in y; r_x = r_y = r when alpha_min = 0; (-1, -1) when
    o < alpha_min (the Gaussian reaches alpha_min nowhere)."""
    r = torch.as_tensor(radius).to(DT)
    if alpha_min <= 0:
        return torch.stack([r, r], 1).to(torch.int64)
    o = torch.as_tensor(opacity, dtype=DT).detach()
    tau = torch.log(o / alpha_min)
    t = torch.clamp(tau, min=0.0)
    ex = torch.ceil(torch.sqrt(2.0 * t * torch.as_tensor(sxx, dtype=DT).detach()))
    ey = torch.ceil(torch.sqrt(2.0 * t * torch.as_tensor(syy, dtype=DT).detach()))
    ext = torch.stack([torch.minimum(r, ex), torch.minimum(r, ey)], 1)
    ext = torch.where((tau >= 0)[:, None], ext, torch.full_like(ext, -1.0))
    return ext.to(torch.int64)


def tile_rect(u, v, extent, tile_w, tile_h, tiles_x, tiles_y):
    """Tiles [x0, x1) x [y0, y1) covered by the box |x-u| <= r_x, |y-v| <= r_y
    (extent (n,2) = (r_x, r_y)): x0 = clamp(floor((u - r_x)/tile_w), 0, tiles_x),
    x1 = clamp(floor((u + r_x)/tile_w) + 1, 0, tiles_x), likewise in y. Computed
    in float64 on the given u, v (exact for float32 inputs)."""
    u = torch.as_tensor(u, dtype=DT)
    v = torch.as_tensor(v, dtype=DT)
    e = torch.as_tensor(extent).to(DT).reshape(-1, 2)
    rx, ry = e[:, 0], e[:, 1]
    x0 = torch.clamp(torch.floor((u - rx) / tile_w), 0, tiles_x).to(torch.int64)
    x1 = torch.clamp(torch.floor((u + rx) / tile_w) + 1, 0, tiles_x).to(torch.int64)
    y0 = torch.clamp(torch.floor((v - ry) / tile_h), 0, tiles_y).to(torch.int64)
    y1 = torch.clamp(torch.floor((v + ry) / tile_h) + 1, 0, tiles_y).to(torch.int64)
    empty = (rx < 0) | (ry < 0)
    x1 = torch.where(empty, x0, x1)
    return x0, x1, y0, y1


def rect_contributes(u, v, a, b, c, o, rx, ry, x0, x1, y0, y1, rp: "RasterParams") -> bool:
    """Whether a Gaussian can take part in the compositing of any pixel of
    the pixel rectangle [x0, x1) x [y0, y1): some pixel centre p lies in its
    overlap box and has P <= 0 and alpha' = min(alpha_max, o exp(P)) >=
    alpha_min (Eq. 5 with the skip rule), by brute force over the pixels in
    FP64. A list may drop exactly the entries for which this is false without
    changing any of those pixels."""
    rp = rp.as_f32()
    xs = np.arange(x0, x1) + 0.5
    ys = np.arange(y0, y1) + 0.5
    px, py = np.meshgrid(xs, ys)
    dx, dy = px - float(u), py - float(v)
    inbox = (np.abs(dx) <= rx) & (np.abs(dy) <= ry)
    power = -0.5 * (a * dx * dx + c * dy * dy) - b * dx * dy
    alpha = np.minimum(o * np.exp(np.minimum(power, 0.0)), rp.alpha_max)
    return bool((inbox & (power <= 0) & (alpha >= rp.alpha_min)).any())


def tile_contributes(u, v, a, b, c, o, rx, ry, tx, ty, tile_w, tile_h, width, height,
                     rp: "RasterParams") -> bool:
    """rect_contributes on the pixels of tile (tx, ty) inside the image."""
    return rect_contributes(u, v, a, b, c, o, rx, ry, tx * tile_w, min((tx + 1) * tile_w, width),
                            ty * tile_h, min((ty + 1) * tile_h, height), rp)


def float32_bits(x) -> np.ndarray:
    return np.asarray(x, dtype=np.float32).view(np.uint32)


def bin_and_sort(u32, v32, depth32, extent, ids, width, height, tile_w, tile_h,
                 tile_offset: int = 0):
    """The per-tile depth-ordered lists.

    For every visible Gaussian (given in ascending ``ids`` order) and every tile
    of its rect (row-major), emit key = (global_tile << 32) | bits(depth_f32)
    with value = Gaussian index; sort the keys stably. Equal keys keep emission
    order, so ties in depth are broken by ascending Gaussian index.
    Returns (keys uint64, values int64, ranges (tiles, 2) int64 [start, end)).
    """
    u32 = np.asarray(u32, dtype=np.float32)
    v32 = np.asarray(v32, dtype=np.float32)
    dbits = float32_bits(depth32).astype(np.uint64)
    extent = np.asarray(extent, dtype=np.int64).reshape(-1, 2)
    ids = np.asarray(ids, dtype=np.int64)
    tx_n = (width + tile_w - 1) // tile_w
    ty_n = (height + tile_h - 1) // tile_h
    x0, x1, y0, y1 = (a.numpy() for a in tile_rect(u32.astype(np.float64), v32.astype(np.float64),
                                                     extent, tile_w, tile_h, tx_n, ty_n))
    keys, vals = [], []
    for k in range(len(ids)):
        for ty in range(y0[k], y1[k]):
            for tx in range(x0[k], x1[k]):
                tile = tile_offset + ty * tx_n + tx
                keys.append((np.uint64(tile) << np.uint64(32)) | dbits[k])
                vals.append(ids[k])
    keys = np.asarray(keys, dtype=np.uint64)
    vals = np.asarray(vals, dtype=np.int64)
    order = np.argsort(keys, kind="stable")
    keys, vals = keys[order], vals[order]
    n_tiles = tx_n * ty_n
    ranges = np.zeros((n_tiles, 2), dtype=np.int64)
    tiles = (keys >> np.uint64(32)).astype(np.int64) - tile_offset
    for i, t in enumerate(tiles):
        if i == 0 or tiles[i - 1] != t:
            ranges[t, 0] = i
        ranges[t, 1] = i + 1
    return keys, vals, ranges


def super_tile_lists(u32, v32, depth32, extent, ids, width, height, tile_w, tile_h, super_tile,
                     super_offset: int = 0):
    """Depth-ordered lists at the granularity of super-tiles (squares of
    ``super_tile`` x ``super_tile`` tiles): the list of super-tile s holds
    every visible Gaussian whose tile rectangle meets s, in (float32 depth,
    index) order. A tile's own list is the ordered subsequence of its
    super-tile's list whose rectangles contain the tile.
    Returns (super index int64 per list entry, values int64, ranges
    (supers, 2) int64 [start, end)), the entries sorted by super-tile."""
    u32 = np.asarray(u32, dtype=np.float32)
    v32 = np.asarray(v32, dtype=np.float32)
    dbits = float32_bits(depth32).astype(np.uint64)
    extent = np.asarray(extent, dtype=np.int64).reshape(-1, 2)
    ids = np.asarray(ids, dtype=np.int64)
    tx_n = (width + tile_w - 1) // tile_w
    ty_n = (height + tile_h - 1) // tile_h
    sx_n = (tx_n + super_tile - 1) // super_tile
    sy_n = (ty_n + super_tile - 1) // super_tile
    x0, x1, y0, y1 = (a.numpy() for a in tile_rect(u32.astype(np.float64), v32.astype(np.float64),
                                                     extent, tile_w, tile_h, tx_n, ty_n))
    keys, vals = [], []
    for k in range(len(ids)):
        if x1[k] <= x0[k] or y1[k] <= y0[k]:
            continue
        for sy in range(y0[k] // super_tile, (y1[k] - 1) // super_tile + 1):
            for sx in range(x0[k] // super_tile, (x1[k] - 1) // super_tile + 1):
                sup = super_offset + sy * sx_n + sx
                keys.append((np.uint64(sup) << np.uint64(32)) | dbits[k])
                vals.append(ids[k])
    keys = np.asarray(keys, dtype=np.uint64)
    vals = np.asarray(vals, dtype=np.int64)
    order = np.argsort(keys, kind="stable")
    keys, vals = keys[order], vals[order]
    sups = (keys >> np.uint64(32)).astype(np.int64)
    ranges = np.zeros((sx_n * sy_n, 2), dtype=np.int64)
    for i, t in enumerate(sups - super_offset):
        if i == 0 or sups[i - 1] - super_offset != t:
            ranges[t, 0] = i
        ranges[t, 1] = i + 1
    return sups, vals, ranges


# ---------------------------------------------------------------------------
# Compositing (Eqs. 4-5)
# ---------------------------------------------------------------------------
def depth_order(depth: torch.Tensor, ids: torch.Tensor) -> torch.Tensor:
    """Permutation sorting by (depth rounded to float32, Gaussian index)
    ascending: the renderer's depth key is the float32 camera depth, so two
    Gaussians whose depths round to the same float32 value count as tied and
    keep ascending index order."""
    d = np.asarray(depth.detach().numpy(), dtype=np.float32)
    i = ids.numpy() if isinstance(ids, torch.Tensor) else np.asarray(ids)
    return torch.as_tensor(np.lexsort((i, d)), dtype=torch.int64)


def pixel_grid(width: int, height: int):
    ys, xs = torch.meshgrid(torch.arange(height, dtype=torch.int64),
                            torch.arange(width, dtype=torch.int64), indexing="ij")
    return xs.flatten(), ys.flatten()


def composite(uv, conic, opacity, rgb, depth, extent, ids, width, height,
              rp: RasterParams, px=None, py=None, max_elems: int = 4_000_000) -> dict:
    """Front-to-back compositing of Eq. 4 with alpha' from Eq. 5.

    For every requested pixel p (default: the whole image; ``px``, ``py`` are
    integer pixel indices), the Gaussians overlapping p are taken in
    (depth, index) order; the pixel colour is sum_i c_i alpha'_i T_i plus
    bg * T_final. Returns ``rgb`` (3, n_px), ``T_final`` (n_px,),
    ``n_blended`` (n_px,) and ``last`` (n_px,): the Gaussian index of the last
    blended Gaussian (-1 if none). Tensors keep autograd history.

    Work is split over pixel chunks; each chunk only looks at the Gaussians
    whose square reaches the chunk's pixel-centre bounding box, which drops
    only Gaussians that overlap none of its pixels.
    """
    rp = rp.as_f32()
    if px is None:
        px, py = pixel_grid(width, height)
    px = torch.as_tensor(px, dtype=torch.int64)
    py = torch.as_tensor(py, dtype=torch.int64)
    ids = torch.as_tensor(ids, dtype=torch.int64)
    order = depth_order(depth, ids)
    u = uv[order, 0]
    v = uv[order, 1]
    a, b, c = conic[order, 0], conic[order, 1], conic[order, 2]
    o = opacity[order]
    col = rgb[order]
    ext = torch.as_tensor(extent).reshape(-1, 2)[order].to(DT)
    rx, ry = ext[:, 0], ext[:, 1]
    gid = ids[order]
    bg = torch.tensor(rp.bg, dtype=DT)

    n_px = px.shape[0]
    out_rgb, out_T, out_n, out_last = [], [], [], []
    ng = max(1, u.shape[0])
    chunk = max(1, min(n_px, max_elems // ng))
    # Sort pixels spatially so chunks are compact.
    start = 0
    while start < n_px:
        sl = slice(start, min(n_px, start + chunk))
        pcx = px[sl].to(DT) + 0.5
        pcy = py[sl].to(DT) + 0.5
        with torch.no_grad():
            cand = ((u + rx >= pcx.min()) & (u - rx <= pcx.max()) &
                    (v + ry >= pcy.min()) & (v - ry <= pcy.max()))
            ci = torch.nonzero(cand).flatten()
        res = _composite_block(pcx, pcy, u[ci], v[ci], a[ci], b[ci], c[ci], o[ci],
                               col[ci], rx[ci], ry[ci], gid[ci], bg, rp)
        out_rgb.append(res[0]); out_T.append(res[1]); out_n.append(res[2]); out_last.append(res[3])
        start += chunk
    return dict(rgb=torch.cat(out_rgb, 1), T_final=torch.cat(out_T), n_blended=torch.cat(out_n),
                last=torch.cat(out_last))


def _composite_block(pcx, pcy, u, v, a, b, c, o, col, rx, ry, gid, bg, rp):
    npx = pcx.shape[0]
    if u.shape[0] == 0:
        T = torch.ones(npx, dtype=DT)
        return ((bg[:, None] * T[None, :]).clone(), T,
                torch.zeros(npx, dtype=torch.int64), torch.full((npx,), -1, dtype=torch.int64))
    dx = pcx[:, None] - u[None, :]
    dy = pcy[:, None] - v[None, :]
    power = -0.5 * (a[None, :] * dx * dx + c[None, :] * dy * dy) - b[None, :] * dx * dy
    alpha = torch.clamp(o[None, :] * torch.exp(power), max=rp.alpha_max)
    with torch.no_grad():
        member = (dx.abs() <= rx[None, :]) & (dy.abs() <= ry[None, :])
        active = member & (power <= 0) & (alpha >= rp.alpha_min)
        a_act = torch.where(active, alpha, torch.zeros_like(alpha))
        # Transmittance after each Gaussian (front to back) counting every
        # active one; blending stops before the first Gaussian that would
        # take it below t_min, and nothing after that blends.
        t_after = torch.cumprod(1.0 - a_act, dim=1)
        blended = active & (t_after >= rp.t_min)
    a_bl = torch.where(blended, alpha, torch.zeros_like(alpha))
    one_minus = 1.0 - a_bl
    T_incl = torch.cumprod(one_minus, dim=1)
    T_excl = torch.cat([torch.ones(npx, 1, dtype=DT), T_incl[:, :-1]], dim=1)
    w = a_bl * T_excl                                                   # alpha'_i T_i
    T_final = T_incl[:, -1]
    out = (w @ col).T + bg[:, None] * T_final[None, :]                  # (3, npx)
    with torch.no_grad():
        n_bl = blended.sum(1)
        pos = torch.arange(u.shape[0]).expand_as(blended)
        lastpos = torch.where(blended, pos, torch.full_like(pos, -1)).max(1).values
        last = torch.where(lastpos >= 0, gid[lastpos.clamp(min=0)], torch.full_like(lastpos, -1))
    return out, T_final, n_bl, last


def render(means, log_scales, quats, opacity_logits, sh, sh_degree, cam, rp: RasterParams,
           px=None, py=None) -> dict:
    """Project and composite: the forward image of one view (3, H*W) plus
    per-pixel T_final, blended count and last blended Gaussian."""
    pr = project(means, log_scales, quats, opacity_logits, sh, sh_degree, cam, rp)
    out = composite(pr["uv"], pr["conic"], pr["opacity"], pr["rgb"], pr["depth"], pr["extent"],
                    pr["ids"], cam.width, cam.height, rp, px=px, py=py)
    out["proj"] = pr
    return out
