"""Pins of the oracle's adaptive density control (Sec. 3): the clone / split
/ prune rules on hand-built cases, the output order, split children against a
closed form and against the parent's density (sample moments checked with an
independent rotation), threshold boundaries, and the view-space gradient
statistic."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import densify as D

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")

F = 11 + 3   # SH degree 0


def _planes(n, rng):
    P = np.zeros((F, n), np.float32)
    P[0:3] = rng.normal(0, 1, (3, n))
    P[3:6] = rng.normal(-3, 0.3, (3, n))
    q = rng.normal(0, 1, (4, n))
    P[6:10] = q
    P[10] = rng.normal(1.0, 0.5, n)
    P[11:14] = rng.uniform(0, 1, (3, n))
    return P


def test_rules_counts_and_order():
    rng = np.random.default_rng(0)
    p = D.DensifyParams(grad_threshold=1e-3, percent_dense=0.01, scene_extent=5.0,
                        min_opacity=0.005)
    P = _planes(6, rng)
    small, big = math.log(0.01), math.log(0.2)   # max scale vs 0.05
    P[3:6, :] = small
    P[3, 2] = big                                  # Gaussian 2 is large
    P[4, 5] = big                                  # Gaussian 5 is large
    P[10, 3] = -8.0                                # opacity 3e-4: pruned
    P[10, 5] = -8.0
    g = np.array([0.0, 0.02, 0.02, 0.02, 0.0, 0.02], np.float32)
    c = np.array([3, 10, 10, 10, 0, 10])
    # 0: below threshold, kept; 1: clone; 2: split; 3: pruned (would clone);
    # 4: never visible, kept; 5: pruned (would split)
    keep, clone, split = D.decisions(P, g, c, p)
    assert keep.tolist() == [True, True, False, False, True, False]
    assert clone.tolist() == [False, True, False, False, False, False]
    assert split.tolist() == [False, False, True, False, False, False]
    m = rng.normal(0, 1, P.shape).astype(np.float32)
    v = rng.uniform(0, 1, P.shape).astype(np.float32)
    z = rng.normal(0, 1, (6, 2, 3))
    op, om, ov = D.densify(P, m, v, g, c, z, p)
    assert op.shape == (F, 3 + 1 + 2)
    # kept in index order, then the clone, then the two children
    assert np.array_equal(op[:, 0], P[:, 0]) and np.array_equal(op[:, 1], P[:, 1])
    assert np.array_equal(op[:, 2], P[:, 4]) and np.array_equal(op[:, 3], P[:, 1])
    for k in (4, 5):
        assert np.array_equal(op[6:, k], P[6:, 2].astype(np.float64))   # copied planes
        assert np.allclose(op[3:6, k], P[3:6, 2] - math.log(1.6), rtol=0, atol=1e-6)
    # moments: kept keep theirs, new ones start at zero
    assert np.array_equal(om[:, :3], m[:, [0, 1, 4]]) and np.array_equal(ov[:, :3], v[:, [0, 1, 4]])
    assert not om[:, 3:].any() and not ov[:, 3:].any()


def test_split_identity_rotation_closed_form():
    """q = (2, 0, 0, 0) (normalised to the identity): child = mu + s * z."""
    p = D.DensifyParams(grad_threshold=1e-3, percent_dense=0.001, scene_extent=1.0)
    P = np.zeros((F, 1), np.float32)
    P[0:3, 0] = (0.5, -1.0, 2.0)
    P[3:6, 0] = np.log([0.3, 0.1, 0.02])
    P[6:10, 0] = (2.0, 0.0, 0.0, 0.0)
    P[10, 0] = 2.0
    z = np.array([[[1.0, -2.0, 0.5], [0.0, 3.0, -1.0]]])
    op, _, _ = D.densify(P, P, P, np.array([1.0], np.float32), np.array([1]), z, p)
    s = np.exp(P[3:6, 0].astype(np.float64))
    for j in range(2):
        assert np.allclose(op[0:3, j], P[0:3, 0] + s * z[0, j], rtol=0, atol=1e-12)
        assert np.allclose(np.exp(op[3:6, j]), s / 1.6, rtol=1e-12)


def test_split_children_follow_parent_density():
    """Children of one anisotropic, rotated Gaussian: sample mean and
    covariance against mu and R diag(s^2) R^T, R from scipy's rotation."""
    rng = np.random.default_rng(3)
    n = 20000
    rot = Rotation.from_euler("zyx", [0.7, -0.4, 1.1])
    x, y, z, w = rot.as_quat()
    s = np.array([0.5, 0.2, 0.05])
    P = np.zeros((F, n), np.float32)
    P[0:3] = np.array([[1.0], [2.0], [-0.5]])
    P[3:6] = np.log(s)[:, None]
    P[6:10] = np.array([[w], [x], [y], [z]])
    P[10] = 3.0
    p = D.DensifyParams(grad_threshold=1e-3, percent_dense=0.001, scene_extent=1.0)
    zs = rng.normal(0, 1, (n, 2, 3))
    op, _, _ = D.densify(P, P, P, np.ones(n, np.float32), np.ones(n, np.int64), zs, p)
    kids = op[0:3].T
    assert kids.shape == (2 * n, 3)
    sig = rot.as_matrix() @ np.diag(s ** 2) @ rot.as_matrix().T
    assert np.allclose(kids.mean(0), [1.0, 2.0, -0.5], atol=4 * 0.5 / math.sqrt(2 * n))
    cov = np.cov(kids.T)
    assert np.linalg.norm(cov - sig) / np.linalg.norm(sig) < 0.03


def test_threshold_boundaries():
    p = D.DensifyParams(grad_threshold=2e-4, percent_dense=0.01, scene_extent=5.0,
                        min_opacity=0.005)
    gt, lst, lgt = p.thresholds()
    P = np.zeros((F, 6), np.float32)
    P[10] = 1.0
    P[3:6] = lst - 1.0
    g = np.zeros(6, np.float32)
    c = np.full(6, 4)
    g[0] = np.float32(gt) * np.float32(4)                        # exactly at the threshold
    g[1] = np.nextafter(g[0], np.float32(0))                      # just below
    g[2:] = g[0]
    P[3, 2] = lst                                                 # at the size limit: small
    P[3, 3] = np.nextafter(np.float32(lst), np.float32(np.inf))   # just above: large
    P[10, 4] = lgt                                                # at the opacity limit: kept
    P[10, 5] = np.nextafter(np.float32(lgt), np.float32(-np.inf))  # just below: pruned
    keep, clone, split = D.decisions(P, g, c, p)
    assert clone.tolist() == [True, False, True, False, True, False]
    assert split.tolist() == [False, False, False, True, False, False]
    assert keep.tolist() == [True, True, True, False, True, False]
    # thresholds: logit(min_opacity) and log(percent_dense * extent)
    assert abs(lgt - math.log(0.005 / 0.995)) < 1e-6
    assert abs(lst - math.log(0.05)) < 1e-6


def test_view_space_grad_closed_form():
    # a pixel-space gradient of (2 / W, 0) is one NDC unit
    assert D.view_space_grad(2.0 / 640, 0.0, 640, 480) == pytest.approx(1.0)
    assert D.view_space_grad(3.0 / 640 * 2, 4.0 / 480 * 2, 640, 480) == pytest.approx(5.0)
