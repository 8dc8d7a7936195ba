"""Pins for the oracle's covariance (Eq. 2), EWA projection (Eq. 3), SH colour
and culling, checked against closed forms, library routines and invariants."""
import math

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation
from scipy import special

from oracle import render as R
from paper_2603_08997_amd import scenes as S

DT = torch.float64


def test_identity_quaternion_gives_diagonal_covariance():
    ls = torch.tensor([[-1.0, -2.0, 0.5]], dtype=DT)
    q = torch.tensor([[1.0, 0.0, 0.0, 0.0]], dtype=DT)
    sig = R.covariance_3d(ls, q)[0]
    expect = torch.diag(torch.exp(2 * ls[0]))
    assert torch.allclose(sig, expect, rtol=0, atol=1e-15)


def test_rotation_about_z_closed_form():
    th = 0.7
    s = np.array([0.3, 0.1, 0.2])
    q = torch.tensor([[math.cos(th / 2), 0.0, 0.0, math.sin(th / 2)]], dtype=DT)
    sig = R.covariance_3d(torch.tensor(np.log(s))[None], q)[0].numpy()
    c, sn = math.cos(th), math.sin(th)
    assert sig[0, 0] == pytest.approx(s[0] ** 2 * c * c + s[1] ** 2 * sn * sn, abs=1e-15)
    assert sig[1, 1] == pytest.approx(s[0] ** 2 * sn * sn + s[1] ** 2 * c * c, abs=1e-15)
    assert sig[0, 1] == pytest.approx((s[0] ** 2 - s[1] ** 2) * sn * c, abs=1e-15)
    assert sig[2, 2] == pytest.approx(s[2] ** 2, abs=1e-15)
    assert abs(sig[0, 2]) < 1e-16 and abs(sig[1, 2]) < 1e-16


def test_rotation_matches_scipy_and_is_normalised():
    rng = np.random.default_rng(11)
    q = rng.normal(size=(64, 4)) * rng.uniform(0.1, 5.0, (64, 1))   # unnormalised on purpose
    Rm = R.quat_to_rotation(torch.tensor(q)).numpy()
    ref = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()      # scipy: (x, y, z, w)
    assert np.abs(Rm - ref).max() < 1e-13


def test_covariance_is_symmetric_psd_with_scale_eigenvalues():
    rng = np.random.default_rng(12)
    ls = rng.normal(-2, 0.7, (50, 3))
    q = rng.normal(size=(50, 4))
    sig = R.covariance_3d(torch.tensor(ls), torch.tensor(q)).numpy()
    assert np.abs(sig - sig.transpose(0, 2, 1)).max() < 1e-15
    ev = np.linalg.eigvalsh(sig)
    assert np.allclose(np.sort(ev, 1), np.sort(np.exp(2 * ls), 1), rtol=1e-10, atol=0)


def _one_gaussian(mean, log_scale, quat=(1, 0, 0, 0), logit=0.0, dc=0.0):
    return dict(means=np.array([mean], np.float64), log_scales=np.array([log_scale], np.float64),
                quats=np.array([quat], np.float64), opacity_logits=np.array([logit], np.float64),
                sh=np.full((1, 1, 3), dc, np.float64))


def test_on_axis_projection_closed_form():
    cam = S.look_at_camera((0.0, -4.0, 1.0), 96, 64)
    Rc = cam.R.astype(np.float64)
    C = -Rc.T @ cam.t.astype(np.float64)
    d = 3.0
    mean = C + d * Rc[2]                      # on the optical axis at depth d
    ls = np.log([0.05, 0.12, 0.2])
    quat = np.array([0.9, 0.1, -0.3, 0.2])
    g = _one_gaussian(mean, ls, quat)
    rp = R.RasterParams(dilation=0.3, jac_clamp=0.0)
    pr = R.project(g["means"], g["log_scales"], g["quats"], g["opacity_logits"], g["sh"], 0, cam, rp)
    sig = R.covariance_3d(torch.tensor(ls)[None], torch.tensor(quat)[None])[0].numpy()
    # float32 rotation rows are orthonormal only to ~1e-8: use the actual depth
    d_act = (Rc @ mean + cam.t.astype(np.float64))[2]
    cam_sig = (Rc @ sig @ Rc.T)[:2, :2] * (float(cam.fx) / d_act) ** 2
    h = R.f32(0.3)
    expect = np.array([cam_sig[0, 0] + h, cam_sig[0, 1], cam_sig[1, 1] + h])
    assert np.allclose(pr["cov2d"][0].detach().numpy(), expect, rtol=1e-6)
    assert pr["uv"][0, 0].item() == pytest.approx(cam.cx, abs=1e-5)
    assert pr["uv"][0, 1].item() == pytest.approx(cam.cy, abs=1e-5)


def test_projection_jacobian_matches_finite_differences_of_pinhole_map():
    """Without dilation and clamp, Sigma2D = A Sigma A^T with A = d(u, v)/d(mean),
    the Jacobian of the pinhole map, which central differences give directly."""
    cam = S.look_at_camera((3.0, -2.0, 2.0), 80, 60)
    rng = np.random.default_rng(5)
    rp = R.RasterParams(dilation=0.0, jac_clamp=0.0)
    for _ in range(10):
        mean = rng.uniform(-0.5, 0.5, 3)
        ls = rng.normal(-2.5, 0.3, 3)
        quat = rng.normal(size=4)
        g = _one_gaussian(mean, ls, quat)
        pr = R.project(g["means"], g["log_scales"], g["quats"], g["opacity_logits"], g["sh"], 0, cam, rp)
        Rc, t = cam.R.astype(np.float64), cam.t.astype(np.float64)

        def pin(m):
            x = Rc @ m + t
            return np.array([cam.fx * x[0] / x[2] + cam.cx, cam.fy * x[1] / x[2] + cam.cy])

        A = np.zeros((2, 3))
        for k in range(3):
            e = np.zeros(3); e[k] = 1e-6
            A[:, k] = (pin(mean + e) - pin(mean - e)) / 2e-6
        sig = R.covariance_3d(torch.tensor(ls)[None], torch.tensor(quat)[None])[0].numpy()
        s2 = A @ sig @ A.T
        got = pr["cov2d"][0].detach().numpy()
        assert np.allclose(got, [s2[0, 0], s2[0, 1], s2[1, 1]], rtol=1e-7)


def test_conic_is_inverse_and_radius_is_three_sigma_of_major_axis():
    sc = S.tiny_scene(3, 200, log_scale_mean=-2.0)
    cam = S.tetra_cameras()[1]
    pr = R.project(sc.means, sc.log_scales, sc.quats, sc.opacity_logits, sc.sh, 0, cam, R.RasterParams())
    cov = pr["cov2d"].detach().numpy()
    con = pr["conic"].detach().numpy()
    M = np.stack([np.stack([cov[:, 0], cov[:, 1]], 1), np.stack([cov[:, 1], cov[:, 2]], 1)], 1)
    Q = np.stack([np.stack([con[:, 0], con[:, 1]], 1), np.stack([con[:, 1], con[:, 2]], 1)], 1)
    assert np.abs(M @ Q - np.eye(2)).max() < 1e-10
    lam = np.linalg.eigvalsh(M)[:, 1]
    assert np.array_equal(pr["radius"].numpy(), np.ceil(3 * np.sqrt(lam)).astype(np.int64))


def _real_sh_scipy(l, m, d):
    """Real SH from scipy's complex Y_l^m (Condon-Shortley phase included):
    sqrt(2) Re Y_l^m for m > 0, sqrt(2) Im Y_l^|m| for m < 0, Y_l^0 for m = 0."""
    theta = np.arccos(np.clip(d[:, 2], -1, 1))
    phi = np.arctan2(d[:, 1], d[:, 0])
    y = special.sph_harm_y(l, abs(m), theta, phi)
    if m > 0:
        return math.sqrt(2) * y.real
    if m < 0:
        return math.sqrt(2) * y.imag
    return y.real


def test_sh_basis_matches_scipy_spherical_harmonics():
    rng = np.random.default_rng(8)
    d = rng.normal(size=(200, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    Y = R.sh_basis(torch.tensor(d), 3).numpy()
    for l in range(4):
        for m in range(-l, l + 1):
            k = l * l + l + m
            assert np.abs(Y[:, k] - _real_sh_scipy(l, m, d)).max() < 1e-12, (l, m)


def test_sh_basis_orthonormal_by_quadrature():
    xg, wg = np.polynomial.legendre.leggauss(12)          # in cos(theta)
    nphi = 24
    phi = (np.arange(nphi) + 0.5) * 2 * np.pi / nphi
    ct, ph = np.meshgrid(xg, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    d = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    w = (wg[:, None] * np.full(nphi, 2 * np.pi / nphi)[None]).reshape(-1)
    Y = R.sh_basis(torch.tensor(d), 3).numpy()
    G = (Y * w[:, None]).T @ Y
    assert np.abs(G - np.eye(16)).max() < 1e-12


def test_colour_is_dc_plus_offset_clamped_at_zero():
    cam = S.tetra_cameras()[0]
    Rc = cam.R.astype(np.float64); C = -Rc.T @ cam.t.astype(np.float64)
    mean = C + 4.0 * Rc[2]
    for dc, expect in [(0.0, 0.5), (1.0, 0.5 + 1 / (2 * math.sqrt(math.pi))), (-5.0, 0.0)]:
        g = _one_gaussian(mean, np.log([0.05] * 3), dc=dc)
        pr = R.project(g["means"], g["log_scales"], g["quats"], g["opacity_logits"], g["sh"], 0,
                       cam, R.RasterParams())
        assert np.allclose(pr["rgb"].detach().numpy(), expect, atol=1e-15)


def test_culling_near_plane_and_off_screen():
    cam = S.tetra_cameras()[0]
    Rc = cam.R.astype(np.float64); C = -Rc.T @ cam.t.astype(np.float64)
    pts = np.stack([C + 0.1 * Rc[2],                       # in front but nearer than 0.2
                    C - 1.0 * Rc[2],                       # behind
                    C + 3.0 * Rc[2] + 50.0 * Rc[0],        # far off-screen to the right
                    C + 3.0 * Rc[2]])                      # visible
    n = len(pts)
    pr = R.project(pts, np.full((n, 3), np.log(0.01)), np.tile([1.0, 0, 0, 0], (n, 1)),
                   np.zeros(n), np.zeros((n, 1, 3)), 0, cam, R.RasterParams())
    assert pr["ids"].tolist() == [3]


def test_opacity_is_sigmoid_of_logit():
    cam = S.tetra_cameras()[0]
    Rc = cam.R.astype(np.float64); C = -Rc.T @ cam.t.astype(np.float64)
    g = _one_gaussian(C + 4.0 * Rc[2], np.log([0.05] * 3), logit=0.7)
    pr = R.project(g["means"], g["log_scales"], g["quats"], g["opacity_logits"], g["sh"], 0, cam,
                   R.RasterParams())
    assert pr["opacity"].item() == pytest.approx(1 / (1 + math.exp(-0.7)), abs=1e-15)


def _sigma2d_by_hand(cam, mean, ls, quat, lim_x, lim_y, h):
    """Sigma2D of the EWA step written out independently of the oracle: the
    covariance from scipy's rotation, the camera-space point, the Jacobian of
    the pinhole map with tx/tz and ty/tz clamped to +-lim, then J W Sigma W^T
    J^T + h I (W the world-to-camera rotation)."""
    Rc, t = cam.R.astype(np.float64), cam.t.astype(np.float64)
    rot = Rotation.from_quat(np.asarray(quat, np.float64)[[1, 2, 3, 0]]).as_matrix()
    sig = rot @ np.diag(np.exp(2 * np.asarray(ls, np.float64))) @ rot.T
    tx, ty, tz = Rc @ mean + t
    xr = min(max(tx / tz, -lim_x), lim_x)
    yr = min(max(ty / tz, -lim_y), lim_y)
    J = np.array([[cam.fx / tz, 0.0, -cam.fx * xr / tz],
                  [0.0, cam.fy / tz, -cam.fy * yr / tz]])
    s2 = J @ Rc @ sig @ Rc.T @ J.T
    uv = (cam.fx * tx / tz + cam.cx, cam.fy * ty / tz + cam.cy)
    return np.array([s2[0, 0] + h, s2[0, 1], s2[1, 1] + h]), uv, (tx / tz, ty / tz)


def _beyond_clamp_gaussians(cam, frac_x, frac_y, depth=3.0):
    """Large Gaussians whose centres sit at tx/tz = frac_x * half-width / fx
    (and likewise in y): beyond the Jacobian clamp for |frac| > 1.3 while
    their 3-sigma boxes still reach into the image."""
    Rc, t = cam.R.astype(np.float64), cam.t.astype(np.float64)
    C = -Rc.T @ t
    out = []
    for fx_, fy_ in zip(frac_x, frac_y):
        xr = fx_ * (cam.width / 2.0) / cam.fx
        yr = fy_ * (cam.height / 2.0) / cam.fy
        out.append(C + depth * (Rc[2] + xr * Rc[0] + yr * Rc[1]))
    return np.array(out)


def test_jacobian_clamp_beyond_the_limit_matches_hand_built_jacobian():
    """Gaussians outside +-1.3 half-extents: Sigma2D equals J W Sigma W^T J^T
    + h I with J evaluated at the clamped tx/tz, ty/tz (the centre u, v stays
    the unclamped pinhole projection); with the clamp off the same Gaussians
    give the unclamped Jacobian, and the two differ."""
    cam = S.look_at_camera((0.5, -4.0, 1.5), 96, 64)
    fracs_x = [1.6, -2.0, 1.8, 0.2, -1.45]
    fracs_y = [0.1, 1.9, -1.7, -2.2, 1.5]
    means = _beyond_clamp_gaussians(cam, fracs_x, fracs_y)
    rng = np.random.default_rng(21)
    n = len(means)
    ls = rng.normal(np.log(0.55), 0.1, (n, 3))
    quat = rng.normal(size=(n, 4))
    lim_x = R.f32(1.3) * (cam.width / 2.0) / float(cam.fx)
    lim_y = R.f32(1.3) * (cam.height / 2.0) / float(cam.fy)
    h = R.f32(0.3)
    for clamp, lims in ((1.3, (lim_x, lim_y)), (0.0, (np.inf, np.inf))):
        pr = R.project(means, ls, quat, np.zeros(n), np.zeros((n, 1, 3)), 0, cam,
                       R.RasterParams(jac_clamp=clamp))
        assert pr["ids"].tolist() == list(range(n)), "every test Gaussian must be visible"
        for k in range(n):
            exp_cov, exp_uv, ratios = _sigma2d_by_hand(cam, means[k], ls[k], quat[k], *lims, h)
            got = pr["cov2d"][k].detach().numpy()
            assert np.allclose(got, exp_cov, rtol=1e-9, atol=0), (clamp, k, got, exp_cov)
            assert np.allclose(pr["uv"][k].detach().numpy(), exp_uv, rtol=1e-12)
            if clamp > 0:
                beyond = abs(ratios[0]) > lim_x or abs(ratios[1]) > lim_y
                assert beyond or abs(fracs_x[k]) <= 1.3
    # the clamp changes the covariance of every Gaussian beyond it
    c_on = R.project(means, ls, quat, np.zeros(n), np.zeros((n, 1, 3)), 0, cam,
                     R.RasterParams())["cov2d"].detach().numpy()
    c_off = R.project(means, ls, quat, np.zeros(n), np.zeros((n, 1, 3)), 0, cam,
                      R.RasterParams(jac_clamp=0.0))["cov2d"].detach().numpy()
    differs = np.abs(c_on - c_off).max(1) > 1e-6 * np.abs(c_off).max(1)
    assert differs.tolist() == [True] * n


def test_sh_degree_one_colour_follows_the_view_direction():
    """Degree-1 closed form: with only the three l = 1 coefficients set, the
    colour is 0.5 + f_1 Y_1(d) + f_2 Y_2(d) + f_3 Y_3(d), d the unit vector
    from the camera centre to the Gaussian, Y_1 = -c y, Y_2 = c z, Y_3 = -c x,
    c = sqrt(3 / (4 pi)). A Gaussian straight to the camera's right and one
    straight ahead, and off-axis ones in general directions."""
    cam = S.look_at_camera((2.0, -3.0, 1.0), 96, 64)
    Rc, t = cam.R.astype(np.float64), cam.t.astype(np.float64)
    C = -Rc.T @ t
    c1 = math.sqrt(3.0 / (4.0 * math.pi))
    rng = np.random.default_rng(31)
    offs = [(0.0, 0.0), (0.25, 0.0), (-0.2, 0.15), (0.1, -0.2), (0.3, 0.2)]
    means = np.array([C + 3.0 * (Rc[2] + a * Rc[0] + b * Rc[1]) for a, b in offs])
    n = len(means)
    sh = np.zeros((n, 4, 3))
    sh[:, 1:4, :] = rng.normal(0.0, 0.3, (n, 3, 3))
    pr = R.project(means, np.full((n, 3), np.log(0.05)), np.tile([1.0, 0, 0, 0], (n, 1)),
                   np.zeros(n), sh, 1, cam, R.RasterParams())
    assert pr["ids"].tolist() == list(range(n))
    got = pr["rgb_raw"].detach().numpy()
    for k in range(n):
        d = means[k] - C
        d /= np.linalg.norm(d)
        expect = 0.5 + sh[k, 1] * (-c1 * d[1]) + sh[k, 2] * (c1 * d[2]) + sh[k, 3] * (-c1 * d[0])
        assert np.allclose(got[k], expect, rtol=0, atol=1e-14), (k, got[k], expect)
    # one coefficient on the x-type basis function, for the Gaussian whose
    # direction has the largest world-x component: the colour moves from 0.5
    # against the sign of that component (a reversed direction would move it
    # the other way)
    dirs = means - C
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    k = int(np.argmax(np.abs(dirs[:, 0])))
    assert abs(dirs[k, 0]) > 0.3
    sh1 = np.zeros((1, 4, 3))
    sh1[0, 3, :] = 1.0
    pr1 = R.project(means[k:k + 1], np.full((1, 3), np.log(0.05)), np.array([[1.0, 0, 0, 0]]),
                    np.zeros(1), sh1, 1, cam, R.RasterParams())
    col = pr1["rgb_raw"][0].detach().numpy()
    assert np.allclose(col, 0.5 - c1 * dirs[k, 0], atol=1e-14)
    assert (np.sign(col - 0.5) == -np.sign(dirs[k, 0])).all()
