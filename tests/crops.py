"""The dense-configuration crop: the 200 visible Gaussians whose projected
centres lie nearest the image centre of the dense 6M view, rendered alone in a
64x64 window around the centre (principal point shifted). Selection uses the
oracle's projection; the crop is an input for both the oracle pins and the
GPU parity test."""
from __future__ import annotations

import functools

import numpy as np
import torch

from oracle import render as R
from paper_2603_08997_amd import scenes as S

CROP_N = 200
CROP_WIN = 64


@functools.lru_cache(maxsize=1)
def dense_crop(n_total: int = 6_000_000):
    scene = S.dense_cluster_scene(S.SEED_SCENE, n_total, 3)
    cam = S.hemisphere_cameras(S.SEED_CAMERAS, 1, 1600, 1060)[0]
    arrs = [torch.as_tensor(np.asarray(a, np.float64)) for a in
            (scene.means, scene.log_scales, scene.quats, scene.opacity_logits, scene.sh)]
    with torch.no_grad():
        pr = R.project(*arrs, 3, cam, R.RasterParams())
    uv = pr["uv"].numpy()
    dist = np.hypot(uv[:, 0] - cam.width / 2.0, uv[:, 1] - cam.height / 2.0)
    ids = pr["ids"].numpy()[np.argsort(dist, kind="stable")[:CROP_N]]
    crop = scene.subset(np.sort(ids))
    win = cam.shifted(cam.cx - (cam.width / 2.0 - CROP_WIN / 2.0),
                      cam.cy - (cam.height / 2.0 - CROP_WIN / 2.0), CROP_WIN, CROP_WIN)
    return crop, win
