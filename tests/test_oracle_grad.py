"""Pins for the oracle gradients: central finite differences of the oracle's
own forward, for every parameter group, in smooth mode (thresholds off) and
with thresholds on at points whose discrete decisions stay fixed."""
import numpy as np
import pytest
import torch

from oracle import render as R
from oracle import grad as G
from oracle import loss as Lm
from paper_2603_08997_amd import scenes as S

GROUPS = ("means", "log_scales", "quats", "opacity_logits", "sh")


def _scene(seed, n, deg, ls=-1.6):
    sc = S.tiny_scene(seed, n, log_scale_mean=ls, log_scale_std=0.3)
    if deg > 0:
        rng = np.random.default_rng(seed + 100)
        k = (deg + 1) ** 2
        sh = np.zeros((n, k, 3), np.float32)
        sh[:, 0] = sc.sh[:, 0]
        sh[:, 1:] = rng.normal(0, 0.3, (n, k - 1, 3))
        sc = S.Scene(sc.means * 0.6, sc.log_scales, sc.quats, sc.opacity_logits, sh, deg)
    return {k: np.asarray(v, np.float64) for k, v in G.scene_dict(sc).items()}


def _forward_value(arrs, deg, cam, rp, ct):
    with torch.no_grad():
        out = R.render(arrs["means"], arrs["log_scales"], arrs["quats"], arrs["opacity_logits"],
                       arrs["sh"], deg, cam, rp)
    return float((out["rgb"] * torch.tensor(ct)).sum()), out


def _decisions(out):
    return (out["proj"]["ids"].numpy().tobytes(), out["n_blended"].numpy().tobytes(),
            out["last"].numpy().tobytes(), out["proj"]["radius"].numpy().tobytes())


@pytest.mark.parametrize("deg", [0, 3])
@pytest.mark.parametrize("mode", ["smooth", "thresholds"])
def test_gradient_matches_central_differences(deg, mode):
    arrs = _scene(7 + deg, 24, deg)
    cam = S.tetra_cameras(radius=3.0, width=28, height=22)[1]
    rp = R.smooth_params() if mode == "smooth" else R.RasterParams()
    rng = np.random.default_rng(1)
    ct = rng.normal(0, 1, (3, cam.width * cam.height))
    _, grads = G.render_vjp(arrs, deg, cam, rp, ct)
    base_val, base_out = _forward_value(arrs, deg, cam, rp, ct)
    base_dec = _decisions(base_out)
    checked = 0
    for grp in GROUPS:
        a = arrs[grp]
        flat_idx = rng.choice(a.size, size=min(a.size, 14), replace=False)
        for fi in flat_idx:
            idx = np.unravel_index(fi, a.shape)
            h = 1e-6 * max(1.0, abs(a[idx]))
            vals = []
            ok = True
            for sgn in (1, -1):
                b = {k: v.copy() for k, v in arrs.items()}
                b[grp][idx] += sgn * h
                val, out = _forward_value(b, deg, cam, rp, ct)
                if _decisions(out) != base_dec:
                    ok = False
                vals.append(val)
            if not ok:
                continue
            fd = (vals[0] - vals[1]) / (2 * h)
            an = grads[grp][idx]
            scale = max(1e-6, np.abs(grads[grp]).max())
            assert abs(fd - an) <= 2e-6 * scale + 1e-6 * abs(an), (grp, idx, fd, an)
            checked += 1
    assert checked >= 40


def test_loss_gradient_end_to_end_matches_central_differences():
    arrs = _scene(3, 20, 0)
    cam = S.tetra_cameras(radius=3.0, width=24, height=24)[0]
    rp = R.RasterParams()
    tgt_sc = _scene(4, 20, 0)
    with torch.no_grad():
        tgt = R.render(tgt_sc["means"], tgt_sc["log_scales"], tgt_sc["quats"], tgt_sc["opacity_logits"],
                       tgt_sc["sh"], 0, cam, rp)["rgb"].reshape(3, 24, 24)
    L, img, dimg, grads, out = G.loss_and_grads(arrs, 0, cam, rp, tgt)
    dec = _decisions(out)
    rng = np.random.default_rng(2)
    checked = 0
    for grp in GROUPS:
        a = arrs[grp]
        for fi in rng.choice(a.size, size=min(a.size, 8), replace=False):
            idx = np.unravel_index(fi, a.shape)
            h = 1e-6 * max(1.0, abs(a[idx]))
            vals, same = [], True
            for sgn in (1, -1):
                b = {k: v.copy() for k, v in arrs.items()}
                b[grp][idx] += sgn * h
                with torch.no_grad():
                    o = R.render(b["means"], b["log_scales"], b["quats"], b["opacity_logits"], b["sh"], 0, cam, rp)
                same &= _decisions(o) == dec
                vals.append(Lm.photometric_loss(o["rgb"].reshape(3, 24, 24), tgt).item())
            if not same:
                continue
            fd = (vals[0] - vals[1]) / (2 * h)
            an = grads[grp][idx]
            assert abs(fd - an) <= 1e-6 * max(np.abs(grads[grp]).max(), 1e-8) + 1e-9, (grp, idx, fd, an)
            checked += 1
    assert checked >= 25


def test_dense_crop_gradient_matches_central_differences():
    """The crop of the dense configuration (200 Gaussians, 64x64 window) with
    the default thresholds: the analytic loss gradient against central
    differences at points whose discrete decisions stay fixed."""
    from .crops import dense_crop
    crop, cam = dense_crop()
    arrs = {k: np.asarray(v, np.float64) for k, v in G.scene_dict(crop).items()}
    rp = R.RasterParams()
    rng = np.random.default_rng(12)
    ct = rng.normal(0, 1, (3, cam.width * cam.height))
    _, grads = G.render_vjp(arrs, 3, cam, rp, ct)
    base_val, base_out = _forward_value(arrs, 3, cam, rp, ct)
    base_dec = _decisions(base_out)
    assert base_out["n_blended"].numpy().mean() > 5
    checked = 0
    for grp in GROUPS:
        a = arrs[grp]
        for fi in rng.choice(a.size, size=min(a.size, 12), replace=False):
            idx = np.unravel_index(fi, a.shape)
            h = 1e-6 * max(1.0, abs(a[idx]))
            vals, ok = [], True
            for sgn in (1, -1):
                b = {k: v.copy() for k, v in arrs.items()}
                b[grp][idx] += sgn * h
                val, out = _forward_value(b, 3, cam, rp, ct)
                ok = ok and _decisions(out) == base_dec
                vals.append(val)
            if not ok:
                continue
            fd = (vals[0] - vals[1]) / (2 * h)
            an = grads[grp][idx]
            scale = max(1e-6, np.abs(grads[grp]).max())
            assert abs(fd - an) <= 2e-6 * scale + 1e-6 * abs(an), (grp, idx, fd, an)
            checked += 1
    assert checked >= 40


def test_gradient_beyond_the_jacobian_clamp_matches_central_differences():
    """Large Gaussians whose centres lie beyond the Jacobian clamp (tx/tz or
    ty/tz past +-1.3 half-extents over the focal length) with thresholds on:
    the analytic gradient (zero through the clamped coordinates) against
    central differences of the forward, at decision-stable points, for every
    parameter group."""
    cam = S.look_at_camera((0.5, -4.0, 1.5), 40, 30)
    Rc, t = cam.R.astype(np.float64), cam.t.astype(np.float64)
    C = -Rc.T @ t
    fr = [(1.613, 0.217), (-1.907, -0.389), (0.291, 1.823), (-0.517, -2.093), (1.541, 1.487),
          (0.109, 0.123)]
    means = np.array([C + (2.6 + 0.13 * k) * (Rc[2] + a * (cam.width / 2.0) / cam.fx * Rc[0]
                                              + b * (cam.height / 2.0) / cam.fy * Rc[1])
                      for k, (a, b) in enumerate(fr)])
    n = len(means)
    rng = np.random.default_rng(41)
    arrs = dict(means=means, log_scales=rng.normal(np.log(0.5), 0.1, (n, 3)),
                quats=rng.normal(size=(n, 4)), opacity_logits=rng.normal(0.5, 0.3, n),
                sh=np.concatenate([rng.uniform(-1.0, 1.0, (n, 1, 3)),
                                   rng.normal(0, 0.3, (n, 3, 3))], 1))
    rp = R.RasterParams()
    # the clamp is active for all but the last Gaussian
    tc = means @ Rc.T + t
    lim_x = 1.3 * (cam.width / 2.0) / cam.fx
    lim_y = 1.3 * (cam.height / 2.0) / cam.fy
    beyond = (np.abs(tc[:, 0] / tc[:, 2]) > lim_x) | (np.abs(tc[:, 1] / tc[:, 2]) > lim_y)
    assert beyond.tolist() == [True] * (n - 1) + [False]
    ct = rng.normal(0, 1, (3, cam.width * cam.height))
    _, grads = G.render_vjp(arrs, 1, cam, rp, ct)
    _, base_out = _forward_value(arrs, 1, cam, rp, ct)
    assert base_out["proj"]["ids"].tolist() == list(range(n))
    base_dec = _decisions(base_out)
    checked = clamped_means = 0
    for grp in GROUPS:
        a = arrs[grp]
        for fi in range(a.size):
            idx = np.unravel_index(fi, a.shape)
            h = 1e-6 * max(1.0, abs(a[idx]))
            vals, ok = [], True
            for sgn in (1, -1):
                b = {k: v.copy() for k, v in arrs.items()}
                b[grp][idx] += sgn * h
                val, out = _forward_value(b, 1, cam, rp, ct)
                ok = ok and _decisions(out) == base_dec
                vals.append(val)
            if not ok:
                continue
            fd = (vals[0] - vals[1]) / (2 * h)
            an = grads[grp][idx]
            scale = max(1e-6, np.abs(grads[grp]).max())
            assert abs(fd - an) <= 2e-6 * scale + 1e-6 * abs(an), (grp, idx, fd, an)
            checked += 1
            clamped_means += int(grp == "means" and beyond[idx[0]])
    assert checked >= 60 and clamped_means >= 10, (checked, clamped_means)
