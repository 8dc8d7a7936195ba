"""Seeded synthetic inputs: Gaussian scenes, pinhole cameras, view sequences.

This module draws inputs only. It holds none of the renderer's, loss's, gate's or
optimizer's arithmetic, so both the HIP path and the FP64 oracle can be fed from
it without sharing any of the method. Every array is drawn in float64 with
``numpy.random.default_rng(seed)`` and cast to float32; the float32 values are
what both sides consume.

Scene shapes follow the paper's post-densification regime (Sec. 3: a fixed set
of 1M-5M Gaussians after densification; Sec. 5.1: 30k iterations with
densification until 15k) with synthetic stand-ins for the Mip-NeRF 360 / Deep
Blending / Tanks and Temples photographs, which are not used.

Parameter layout ("planes"): one float32 array ``[F][stride]`` with planes
  0..2   mean x, y, z (world)
  3..5   log-scale x, y, z   (per-axis standard deviation = exp(log-scale), Eq. 2)
  6..9   quaternion w, x, y, z (unnormalised; the renderer normalises)
  10     opacity logit       (opacity = sigmoid(logit))
  11..   SH coefficients, coefficient-major, RGB-minor: plane 11 + 3*k + ch
with F = 11 + 3*(D+1)^2 for SH degree D.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Seeds of the synthetic workloads.
SEED_TINY_RENDER = 0
SEED_TINY_TARGET = 1
SEED_SCENE = 2
SEED_CAMERAS = 3
SEED_VIEW_SEQUENCE = 4
SEED_INIT_PERTURB = 5
SEED_BATCH_CAMERAS = 6

# Resolutions of the batched multi-view launch: two views of each.
BATCH_RESOLUTIONS = ((640, 480), (1245, 825), (1600, 1060), (980, 545))

# Range of the degree-0 SH coefficient that spans colours [0, 1] once the
# renderer adds its +0.5 offset: the DC basis constant is 1/(2*sqrt(pi)).
SH_DC_HALF_RANGE = math.sqrt(math.pi)

PLANE_MEAN = 0
PLANE_LOG_SCALE = 3
PLANE_QUAT = 6
PLANE_OPACITY = 10
PLANE_SH = 11


def n_sh_coeffs(sh_degree: int) -> int:
    return (sh_degree + 1) ** 2


def n_planes(sh_degree: int) -> int:
    return PLANE_SH + 3 * n_sh_coeffs(sh_degree)


def padded_stride(n: int, align: int = 64) -> int:
    return max(align, ((n + align - 1) // align) * align)


@dataclass
class Scene:
    means: np.ndarray          # (N, 3) float32
    log_scales: np.ndarray     # (N, 3) float32
    quats: np.ndarray          # (N, 4) float32, w x y z
    opacity_logits: np.ndarray # (N,)   float32
    sh: np.ndarray             # (N, K, 3) float32, K = (D+1)^2
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def to_planes(self, stride: int | None = None) -> np.ndarray:
        """Pack into the ``[F][stride]`` float32 plane layout (zero padded)."""
        n = self.n
        stride = padded_stride(n) if stride is None else stride
        if stride < n:
            raise ValueError("stride < n")
        f = n_planes(self.sh_degree)
        out = np.zeros((f, stride), dtype=np.float32)
        out[PLANE_MEAN:PLANE_MEAN + 3, :n] = self.means.T
        out[PLANE_LOG_SCALE:PLANE_LOG_SCALE + 3, :n] = self.log_scales.T
        out[PLANE_QUAT:PLANE_QUAT + 4, :n] = self.quats.T
        out[PLANE_OPACITY, :n] = self.opacity_logits
        k = n_sh_coeffs(self.sh_degree)
        out[PLANE_SH:PLANE_SH + 3 * k, :n] = self.sh.reshape(n, 3 * k).T
        return out

    @staticmethod
    def from_planes(planes: np.ndarray, n: int, sh_degree: int) -> "Scene":
        k = n_sh_coeffs(sh_degree)
        p = np.asarray(planes, dtype=np.float32)
        return Scene(
            means=np.ascontiguousarray(p[PLANE_MEAN:PLANE_MEAN + 3, :n].T),
            log_scales=np.ascontiguousarray(p[PLANE_LOG_SCALE:PLANE_LOG_SCALE + 3, :n].T),
            quats=np.ascontiguousarray(p[PLANE_QUAT:PLANE_QUAT + 4, :n].T),
            opacity_logits=np.ascontiguousarray(p[PLANE_OPACITY, :n]),
            sh=np.ascontiguousarray(p[PLANE_SH:PLANE_SH + 3 * k, :n].T.reshape(n, k, 3)),
            sh_degree=sh_degree,
        )

    def subset(self, idx) -> "Scene":
        return Scene(self.means[idx], self.log_scales[idx], self.quats[idx],
                     self.opacity_logits[idx], self.sh[idx], self.sh_degree)


@dataclass
class Camera:
    """Pinhole camera, world->camera rotation R and translation t, OpenCV axes
    (x right, y down, z forward). All values float32."""
    R: np.ndarray   # (3, 3)
    t: np.ndarray   # (3,)
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int

    def shifted(self, cx: float, cy: float, width: int, height: int) -> "Camera":
        return Camera(self.R.copy(), self.t.copy(), self.fx, self.fy,
                      float(np.float32(cx)), float(np.float32(cy)), width, height)


def _f32(x) -> float:
    return float(np.float32(x))


def look_at_camera(center, width: int, height: int, fov_x_deg: float = 60.0,
                   target=(0.0, 0.0, 0.0), up=(0.0, 0.0, 1.0)) -> Camera:
    """Camera at ``center`` looking at ``target`` with world up ``up``.

    Rows of R are the camera axes in world coordinates: z_c towards the
    target, x_c = z_c x up, y_c = z_c x x_c; t = -R C. Focal length from the
    horizontal field of view, principal point at the image centre."""
    c = np.asarray(center, dtype=np.float64)
    z = np.asarray(target, dtype=np.float64) - c
    z /= np.linalg.norm(z)
    x = np.cross(z, np.asarray(up, dtype=np.float64))
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    R = np.stack([x, y, z])
    t = -R @ c
    f = (width / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)
    return Camera(R.astype(np.float32), t.astype(np.float32), _f32(f), _f32(f),
                  _f32(width / 2.0), _f32(height / 2.0), int(width), int(height))


def tetra_cameras(radius: float = 4.0, width: int = 64, height: int = 64,
                  fov_x_deg: float = 60.0) -> list[Camera]:
    """Four cameras at the regular-tetrahedron directions, looking at the origin."""
    dirs = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=np.float64)
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    return [look_at_camera(radius * d, width, height, fov_x_deg) for d in dirs]


def hemisphere_cameras(seed: int, count: int, width: int, height: int,
                       r_lo: float = 4.0, r_hi: float = 5.0,
                       elev_lo_deg: float = 10.0, elev_hi_deg: float = 80.0,
                       fov_x_deg: float = 60.0) -> list[Camera]:
    """Cameras on the upper hemisphere: azimuth U[0, 2pi), elevation
    U[elev_lo, elev_hi], radius U[r_lo, r_hi], all looking at the origin."""
    rng = np.random.default_rng(seed)
    az = rng.uniform(0.0, 2.0 * math.pi, count)
    el = np.radians(rng.uniform(elev_lo_deg, elev_hi_deg, count))
    rad = rng.uniform(r_lo, r_hi, count)
    cams = []
    for a, e, r in zip(az, el, rad):
        c = r * np.array([math.cos(e) * math.cos(a), math.cos(e) * math.sin(a), math.sin(e)])
        cams.append(look_at_camera(c, width, height, fov_x_deg))
    return cams


def batched_cameras(seed: int = SEED_BATCH_CAMERAS) -> list[Camera]:
    """Eight hemisphere views of mixed resolution for one batched launch:
    two of each size in BATCH_RESOLUTIONS, poses drawn as in
    hemisphere_cameras."""
    cams = []
    for k, (w, h) in enumerate(BATCH_RESOLUTIONS):
        cams += hemisphere_cameras(seed * 100 + k, 2, w, h)
    return cams


def _random_quats(rng, n):
    q = rng.normal(0.0, 1.0, (n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def tiny_scene(seed: int, n: int = 1000, log_scale_mean: float = -3.0,
               log_scale_std: float = 0.3) -> Scene:
    """N Gaussians, means U[-1,1]^3, log-scales N(mean, std), normalised
    N(0,1)^4 quaternions, opacity logits N(0,1), SH degree 0 with colours U[0,1]."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(-1.0, 1.0, (n, 3))
    log_scales = rng.normal(log_scale_mean, log_scale_std, (n, 3))
    quats = _random_quats(rng, n)
    logits = rng.normal(0.0, 1.0, n)
    dc = rng.uniform(-SH_DC_HALF_RANGE, SH_DC_HALF_RANGE, (n, 1, 3))
    return Scene(means.astype(np.float32), log_scales.astype(np.float32),
                 quats.astype(np.float32), logits.astype(np.float32),
                 dc.astype(np.float32), 0)


def _mixture_means(rng, n, disk_radius=6.0, plane_sigma=0.05,
                   centres=((1.0, 1.0, 0.5), (-1.0, -1.0, 0.5)), cluster_sigma=0.5,
                   max_norm=6.0, weights=(1 / 3, 1 / 3, 1 / 3)):
    out = np.empty((0, 3))
    while out.shape[0] < n:
        m = 2 * (n - out.shape[0]) + 1024
        comp = rng.choice(3, size=m, p=np.asarray(weights) / np.sum(weights))
        pts = np.empty((m, 3))
        k0 = comp == 0
        r = disk_radius * np.sqrt(rng.uniform(0.0, 1.0, k0.sum()))
        th = rng.uniform(0.0, 2.0 * math.pi, k0.sum())
        pts[k0, 0] = r * np.cos(th)
        pts[k0, 1] = r * np.sin(th)
        pts[k0, 2] = rng.normal(0.0, plane_sigma, k0.sum())
        for ci, c in enumerate(centres, start=1):
            kc = comp == ci
            pts[kc] = rng.normal(0.0, cluster_sigma, (kc.sum(), 3)) + np.asarray(c)
        pts = pts[np.linalg.norm(pts, axis=1) <= max_norm]
        out = np.concatenate([out, pts])
    return out[:n]


def mixture_scene(seed: int, n: int, sh_degree: int = 3, log_scale_mean: float = -4.0,
                  log_scale_std: float = 0.5, logit_std: float = 1.5,
                  sh_rest_std: float = 0.05) -> Scene:
    """Ground-plane disk (radius 6, z ~ N(0, 0.05)) plus two N(., 0.5^2 I)
    clusters at (1,1,0.5) and (-1,-1,0.5), equal weights, means within
    radius 6; log-scales N(-4, 0.5); opacity logits N(0, 1.5); SH DC spanning
    colours [0,1], higher orders N(0, 0.05)."""
    rng = np.random.default_rng(seed)
    means = _mixture_means(rng, n)
    log_scales = rng.normal(log_scale_mean, log_scale_std, (n, 3))
    quats = _random_quats(rng, n)
    logits = rng.normal(0.0, logit_std, n)
    k = n_sh_coeffs(sh_degree)
    sh = rng.normal(0.0, sh_rest_std, (n, k, 3))
    sh[:, 0, :] = rng.uniform(-SH_DC_HALF_RANGE, SH_DC_HALF_RANGE, (n, 3))
    return Scene(means.astype(np.float32), log_scales.astype(np.float32),
                 quats.astype(np.float32), logits.astype(np.float32),
                 sh.astype(np.float32), sh_degree)


def dense_cluster_scene(seed: int, n: int, sh_degree: int = 3, cluster_sigma: float = 0.35,
                        log_scale_mean: float = -3.6, logit_mean: float = -0.45,
                        logit_std: float = 1.0) -> Scene:
    """All Gaussians in the two clusters of the mixture scene (no ground
    plane): a dense scene with high depth complexity. The opacity-logit mean
    is set so that 6M Gaussians seen from the hemisphere cameras at 1600x1060
    blend about 60 Gaussians per pixel on average."""
    rng = np.random.default_rng(seed)
    means = _mixture_means(rng, n, cluster_sigma=cluster_sigma, weights=(0.0, 0.5, 0.5))
    log_scales = rng.normal(log_scale_mean, 0.5, (n, 3))
    quats = _random_quats(rng, n)
    logits = rng.normal(logit_mean, logit_std, n)
    k = n_sh_coeffs(sh_degree)
    sh = rng.normal(0.0, 0.05, (n, k, 3))
    sh[:, 0, :] = rng.uniform(-SH_DC_HALF_RANGE, SH_DC_HALF_RANGE, (n, 3))
    return Scene(means.astype(np.float32), log_scales.astype(np.float32),
                 quats.astype(np.float32), logits.astype(np.float32),
                 sh.astype(np.float32), sh_degree)


def perturb(scene: Scene, seed: int, mean_sigma: float = 0.02, log_scale_sigma: float = 0.1,
            logit_sigma: float = 0.5, dc_sigma: float = 0.1) -> Scene:
    """Trainable initialisation = ground truth plus seeded noise, so that a
    fixed-N refinement has something to fit."""
    rng = np.random.default_rng(seed)
    n = scene.n
    sh = scene.sh.astype(np.float64).copy()
    sh[:, 0, :] += rng.normal(0.0, dc_sigma, (n, 3))
    return Scene(
        (scene.means + rng.normal(0.0, mean_sigma, (n, 3))).astype(np.float32),
        (scene.log_scales + rng.normal(0.0, log_scale_sigma, (n, 3))).astype(np.float32),
        scene.quats.copy(),
        (scene.opacity_logits + rng.normal(0.0, logit_sigma, n)).astype(np.float32),
        sh.astype(np.float32), scene.sh_degree)


def view_sequence(seed: int, n_views: int, length: int) -> np.ndarray:
    """I.i.d. uniform view indices (the 'sample view' step of the training loop)."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, n_views, size=length, dtype=np.int64).astype(np.int32)


def random_records(seed: int, n: int, width: int, height: int, max_radius: int = 24,
                   depth_lo: float = 0.5, depth_hi: float = 8.0, margin: float = 12.0,
                   tie_fraction: float = 0.0, sh_free: bool = True) -> dict:
    """Projected-Gaussian records drawn directly (no projection involved), for
    exercising binning, sorting and compositing on identical float32 inputs.

    Fields: u, v (pixel coords), depth, extent (n, 2) int32 half-sizes of the
    overlap box (each between r/2 and r for a drawn radius r), conic (a, b, c)
    with a, c > 0 and b^2 < a c, opacity in (0, 1), rgb in [0, 1]. A fraction
    of depths can be forced to repeat to exercise the tie-break."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(-margin, width + margin, n)
    v = rng.uniform(-margin, height + margin, n)
    depth = rng.uniform(depth_lo, depth_hi, n)
    if tie_fraction > 0 and n > 1:
        k = int(tie_fraction * n)
        src = rng.integers(0, n, k)
        dst = rng.integers(0, n, k)
        depth[dst] = depth[src]
    radius = rng.integers(1, max_radius + 1, n)
    sig = rng.uniform(0.3, 1.0, (n, 2)) * radius[:, None] / 3.0
    a = 1.0 / sig[:, 0] ** 2
    c = 1.0 / sig[:, 1] ** 2
    b = rng.uniform(-0.9, 0.9, n) * np.sqrt(a * c)
    opacity = rng.uniform(0.05, 0.999, n)
    rgb = rng.uniform(0.0, 1.0, (n, 3))
    ext = np.stack([rng.integers((radius + 1) // 2, radius + 1),
                    rng.integers((radius + 1) // 2, radius + 1)], axis=1)
    f32 = lambda x: np.asarray(x, dtype=np.float32)
    return dict(u=f32(u), v=f32(v), depth=f32(depth), extent=ext.astype(np.int32),
                conic=f32(np.stack([a, b, c], axis=1)), opacity=f32(opacity), rgb=f32(rgb))
