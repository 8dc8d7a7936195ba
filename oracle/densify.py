"""Oracle adaptive density control (FP64). Test infrastructure only.

Sec. 3 of the paper describes the densification phase that precedes the
phase SkipGS accelerates: periodically, Gaussians with a high view-space
positional gradient are cloned when their spatial extent is small and split
when it is large, and near-transparent Gaussians (opacity below a small
threshold) are pruned; after iteration T_d the set is fixed and the gate
takes over (Sec. 3, Algorithm 1).

The paper names the three operations and the opacity rule only. Readings
(the standard 3DGS adaptive density control, as parameters):

* view-space positional gradient of a Gaussian in one view: the norm of
  dL/d(u, v) expressed in normalised device units, where the image spans
  [-1, 1] on each axis: || (dL/du * W / 2, dL/dv * H / 2) ||; the statistic
  is its mean over the views (iterations) since the last densification in
  which the Gaussian was visible; a Gaussian densifies when the mean is at
  least grad_threshold (sum >= grad_threshold * count, count > 0);
* extent: the largest of the three scales; small when
  max log-scale <= log(percent_dense * scene_extent), else large;
* split: the Gaussian is replaced by two children whose centres are drawn
  from its own density, mu + R(q) diag(s) z with z ~ N(0, I) (the draws are
  inputs), with scales s / split_scale and every other parameter copied;
* clone: an exact copy is added;
* prune: a Gaussian whose opacity is below min_opacity produces nothing
  (neither itself nor a clone or children, which share its opacity);
* Adam moments: kept Gaussians keep theirs, new ones (clones, children)
  start at zero;
* output order: the kept Gaussians in index order, then the clones in index
  order, then the children (two per split Gaussian, in index order);
* decisions are taken in the precision the kernels use: the float32 log-scale
  and opacity logit against float32 thresholds formed in binary64 (so
  log-scale > float32(log(percent_dense * extent)) and logit <
  float32(log(m / (1 - m))), m = min_opacity), and the gradient test in
  binary64 on the float32 sum and the integer count.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from . import render as R


@dataclass
class DensifyParams:
    grad_threshold: float = 2e-4
    percent_dense: float = 0.01
    scene_extent: float = 5.0
    min_opacity: float = 0.005
    split_scale: float = 1.6

    def thresholds(self):
        """(gradient, log-scale, logit) thresholds as the kernels compare them."""
        f = np.float32
        g = float(f(self.grad_threshold))
        ls = float(f(math.log(float(f(self.percent_dense)) * float(f(self.scene_extent)))))
        mo = float(f(self.min_opacity))
        lg = float(f(math.log(mo / (1.0 - mo))))
        return g, ls, lg


def view_space_grad(du, dv, width: int, height: int):
    """The view-space positional gradient norm of one view (NDC units)."""
    du = np.asarray(du, np.float64)
    dv = np.asarray(dv, np.float64)
    return np.sqrt((du * 0.5 * width) ** 2 + (dv * 0.5 * height) ** 2)


def decisions(params, grad_sum, count, p: DensifyParams):
    """Per Gaussian: (keep, clone, split) booleans. ``params``: planar
    [F][>= n] float32 array; grad_sum float32, count int (length n)."""
    n = len(count)
    gt, lst, lgt = p.thresholds()
    ls = np.asarray(params[3:6, :n], np.float32).astype(np.float64)
    logit = np.asarray(params[10, :n], np.float32).astype(np.float64)
    g = np.asarray(grad_sum, np.float32).astype(np.float64)
    c = np.asarray(count, np.int64)
    prune = logit < lgt
    cand = (c > 0) & (g >= gt * c.astype(np.float64))
    big = ls.max(axis=0) > lst
    keep = ~prune & ~(cand & big)
    clone = ~prune & cand & ~big
    split = ~prune & cand & big
    return keep, clone, split


def densify(params, m, v, grad_sum, count, normals, p: DensifyParams):
    """One densification step. params, m, v: planar [F][>= n] arrays (the
    first n columns are the Gaussians); normals: (n, 2, 3) standard-normal
    draws for the two children of each Gaussian (used where it splits).
    Returns (params, m, v) of the new set, planar [F][n_out], float64."""
    n = len(count)
    P = np.asarray(params, np.float64)[:, :n]
    M = np.asarray(m, np.float64)[:, :n]
    V = np.asarray(v, np.float64)[:, :n]
    keep, clone, split = decisions(params, grad_sum, count, p)
    idx_k = np.nonzero(keep)[0]
    idx_c = np.nonzero(clone)[0]
    idx_s = np.nonzero(split)[0]
    F = P.shape[0]
    # children: centres mu + R diag(s) z, scales s / split_scale
    mu = torch.tensor(P[0:3, idx_s].T)
    ls = torch.tensor(P[3:6, idx_s].T)
    q = torch.tensor(P[6:10, idx_s].T)
    Rm = R.quat_to_rotation(q) if len(idx_s) else torch.zeros(0, 3, 3, dtype=torch.float64)
    s = torch.exp(ls)
    z = torch.tensor(np.asarray(normals, np.float64)[idx_s])          # (S, 2, 3)
    kids = np.zeros((F, 2 * len(idx_s)))
    for j in range(2):
        cj = mu + torch.einsum("nab,nb->na", Rm, s * z[:, j, :])
        blk = P[:, idx_s].copy()
        blk[0:3] = cj.numpy().T
        blk[3:6] = P[3:6, idx_s] - math.log(float(np.float32(p.split_scale)))
        kids[:, j::2] = blk
    out_p = np.concatenate([P[:, idx_k], P[:, idx_c], kids], axis=1)
    zeros = np.zeros((F, len(idx_c) + 2 * len(idx_s)))
    out_m = np.concatenate([M[:, idx_k], zeros], axis=1)
    out_v = np.concatenate([V[:, idx_k], zeros], axis=1)
    return out_p, out_m, out_v
