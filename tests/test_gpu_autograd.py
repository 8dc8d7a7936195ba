"""The torch.autograd wrappers over the C ABI: render + photometric loss
through autograd against the oracle's loss gradient (the tiny configuration
and the crop of the dense configuration), the recomputing backward against
the one that keeps the forward workspace, and the dense 6M view's peak device
memory with both."""
from __future__ import annotations

import numpy as np
import pytest
import torch

from oracle import grad as G
from oracle import render as R
from paper_2603_08997_amd import scenes as S

from .crops import dense_crop
from .gpu_util import rel_max_err, rel_norm_err, require_gpu, say, to_dev

pytestmark = pytest.mark.gpu

GROUPS = ("means", "log_scales", "quats", "opacity_logits", "sh")


def _grad_groups(planes_grad, n, deg):
    sc = S.Scene.from_planes(planes_grad, n, deg)
    return dict(means=sc.means, log_scales=sc.log_scales, quats=sc.quats,
                opacity_logits=sc.opacity_logits, sh=sc.sh)


def _gpu_loss_grad(scene, cam, target, recompute):
    from paper_2603_08997_amd import autograd as AG
    planes = to_dev(scene.to_planes()).requires_grad_(True)
    img = AG.render(planes, scene.n, scene.sh_degree, [cam], recompute=recompute)
    loss = AG.photometric_loss(img, to_dev(target.reshape(-1)), cam.width, cam.height)
    loss.backward()
    torch.cuda.synchronize()
    return float(loss.detach()), planes.grad.cpu().numpy()


def _check(scene, cam, target):
    loss_t, grad_t = _gpu_loss_grad(scene, cam, target, recompute=True)
    loss_k, grad_k = _gpu_loss_grad(scene, cam, target, recompute=False)
    # same forward; the backward sums per-tile contributions with float
    # atomics, whose order (and so the last bits) varies from run to run
    assert loss_t == loss_k
    assert rel_norm_err(grad_t, grad_k) <= 1e-5
    ref_loss, _, _, ref, _ = G.loss_and_grads(G.scene_dict(scene), scene.sh_degree, cam,
                                              R.RasterParams(), target.astype(np.float64))
    say(f"  loss gpu {loss_t:.7f} oracle {ref_loss:.7f}")
    assert abs(loss_t - ref_loss) <= 1e-5 * abs(ref_loss)
    got = _grad_groups(grad_t, scene.n, scene.sh_degree)
    for k in GROUPS:
        assert rel_norm_err(got[k], ref[k]) <= 1e-3, (k, rel_norm_err(got[k], ref[k]))
        assert rel_max_err(got[k], ref[k]) <= 1e-3, (k, rel_max_err(got[k], ref[k]))


def test_autograd_tiny_matches_oracle():
    require_gpu()
    sc = S.tiny_scene(S.SEED_TINY_RENDER, log_scale_mean=-2.2)
    tgt_scene = S.tiny_scene(S.SEED_TINY_TARGET, log_scale_mean=-2.2)
    cam = S.tetra_cameras()[0]
    with torch.no_grad():
        t = R.render(*[torch.as_tensor(np.asarray(a, np.float64)) for a in
                       (tgt_scene.means, tgt_scene.log_scales, tgt_scene.quats,
                        tgt_scene.opacity_logits, tgt_scene.sh)],
                     tgt_scene.sh_degree, cam, R.RasterParams())
    target = t["rgb"].numpy().reshape(3, cam.height, cam.width).astype(np.float32)
    say("autograd tiny")
    _check(sc, cam, target)


def test_autograd_dense_crop_matches_oracle():
    require_gpu()
    crop, cam = dense_crop()
    target = np.random.default_rng(21).uniform(0, 1, (3, cam.height, cam.width)).astype(np.float32)
    say(f"autograd dense crop: {crop.n} Gaussians, {cam.width}x{cam.height}")
    _check(crop, cam, target)


def test_autograd_dense_peak_memory():
    """Dense 6M view: the recomputing backward gives the same gradient (up to
    the order of the float atomics that sum per-tile contributions) and holds
    no forward workspace between the two passes."""
    require_gpu()
    from paper_2603_08997_amd import autograd as AG
    scene = S.dense_cluster_scene(S.SEED_SCENE, 6_000_000, 3)
    cam = S.hemisphere_cameras(S.SEED_CAMERAS, 1, 1600, 1060)[0]
    target = torch.rand(3 * cam.width * cam.height, device="cuda",
                        generator=torch.Generator(device="cuda").manual_seed(3))
    out = {}
    for recompute in (True, False):
        planes = to_dev(scene.to_planes()).requires_grad_(True)
        torch.cuda.synchronize()
        torch.cuda.reset_peak_memory_stats()
        base = torch.cuda.memory_allocated()
        img = AG.render(planes, scene.n, 3, [cam], capacity=200_000_000, recompute=recompute)
        loss = AG.photometric_loss(img, target, cam.width, cam.height)
        torch.cuda.synchronize()
        held = torch.cuda.memory_allocated() - base
        loss.backward()
        torch.cuda.synchronize()
        peak = torch.cuda.max_memory_allocated() - base
        out[recompute] = (float(loss.detach()), planes.grad.cpu().numpy(), held)
        say(f"  recompute={recompute}: loss {out[recompute][0]:.6f}, device memory held between "
            f"forward and backward {held / 2**30:.2f} GiB, peak {peak / 2**30:.2f} GiB "
            f"(above the parameters)")
        del planes, img, loss
        torch.cuda.empty_cache()
    assert out[True][0] == out[False][0]
    assert rel_norm_err(out[True][1], out[False][1]) <= 1e-5
    assert out[True][2] < out[False][2]
