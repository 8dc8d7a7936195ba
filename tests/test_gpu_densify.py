"""Adaptive density control (Sec. 3) through the C ABI against the oracle:
the clone / split / prune step (sizes, decisions and order bit-exact, copied
Gaussians and moments bit-exact, split children within FP32 rounding) on
ragged counts and both SH degrees, an output too small for the new set, the
view-space gradient statistic after a render backward on identical records,
and a short two-phase run (densification until T_d, then the gate)."""
import numpy as np
import pytest
import torch

from oracle import densify as OD
from oracle import render as R
from paper_2603_08997_amd import scenes as S
from tests.gpu_util import rel_max_err, require_gpu, say, sg, split_views, to_dev
from tests.sensitivity import decision_sensitive
from tests.test_gpu_stages import DECISION_REL, Stage, _oracle_composite, _records, _views

pytestmark = pytest.mark.gpu


def _inputs(n, sh_degree, seed):
    """Seeded parameters (mixture scene), moments, statistic and draws with a
    spread of outcomes: about a third below the gradient threshold, the rest
    split between small and large, some near-transparent."""
    rng = np.random.default_rng(seed)
    sc = S.mixture_scene(seed, n, sh_degree=sh_degree)
    P = sc.to_planes()
    F, stride = P.shape
    P[10, :n] = rng.normal(-1.0, 3.0, n).astype(np.float32)      # some below logit(0.005)
    m = rng.normal(0, 1e-3, (F, stride)).astype(np.float32)
    v = rng.uniform(0, 1e-6, (F, stride)).astype(np.float32)
    count = rng.integers(0, 12, n).astype(np.int32)
    g = (count * 2e-4 * rng.uniform(0.3, 2.0, n)).astype(np.float32)
    normals = rng.normal(0, 1, (n, 2, 3)).astype(np.float32)
    return P, m, v, g, count, normals


def _gpu_densify(dp, P, m, v, g, count, normals, n, sh_degree, out_stride):
    m_ = sg()
    F = P.shape[0]
    outs = [torch.full((F, out_stride), float("nan"), device="cuda") for _ in range(3)]
    ws = m_.alloc_bytes(max(m_.densify_workspace_size(n), 16))
    d_n = torch.zeros(1, dtype=torch.int64, device="cuda")
    m_.densify(dp, to_dev(P), n, sh_degree, to_dev(m), to_dev(v), to_dev(g), to_dev(count),
               to_dev(normals), *outs, ws, d_n)
    torch.cuda.synchronize()
    return int(d_n.item()), [o.cpu().numpy() for o in outs]


@pytest.mark.parametrize("n,deg", [(5000, 3), (777, 0), (1, 3)])
def test_densify_matches_oracle(n, deg):
    require_gpu()
    m_ = sg()
    P, m, v, g, count, normals = _inputs(n, deg, 60 + n)
    dp = m_.DensifyParams(grad_threshold=2e-4, percent_dense=0.01, scene_extent=2.0,
                          min_opacity=0.005)
    odp = OD.DensifyParams(grad_threshold=2e-4, percent_dense=0.01, scene_extent=2.0,
                           min_opacity=0.005)
    keep, clone, split = OD.decisions(P, g, count, odp)
    say(f"densify n={n} deg={deg}: keep {keep.sum()} clone {clone.sum()} split {split.sum()}")
    op, om, ov = OD.densify(P, m, v, g, count, normals, odp)
    n_out, (gp, gm, gv) = _gpu_densify(dp, P, m, v, g, count, normals, n, deg,
                                       S.padded_stride(2 * n))
    assert n_out == op.shape[1]
    K, Cn = int(keep.sum()), int(clone.sum())
    copies = slice(0, K + Cn)
    # kept and cloned Gaussians, and every moment: bit for bit
    assert np.array_equal(gp[:, copies], op[:, copies].astype(np.float32))
    assert np.array_equal(gm[:, :n_out], om.astype(np.float32))
    assert np.array_equal(gv[:, :n_out], ov.astype(np.float32))
    kids = slice(K + Cn, n_out)
    if n_out > K + Cn:
        # children: centres and log-scales within FP32 rounding, the rest copied
        assert rel_max_err(gp[0:3, kids], op[0:3, kids]) < 1e-5
        assert np.abs(gp[3:6, kids] - op[3:6, kids]).max() < 2e-6
        assert np.array_equal(gp[6:, kids], op[6:, kids].astype(np.float32))
    # nothing written past the new set
    assert np.isnan(gp[:, n_out:]).all()


def test_densify_output_too_small_writes_nothing():
    require_gpu()
    m_ = sg()
    n = 3000
    P, m, v, g, count, normals = _inputs(n, 3, 9)
    dp = m_.DensifyParams(scene_extent=2.0)
    odp = OD.DensifyParams(scene_extent=2.0)
    need = OD.densify(P, m, v, g, count, normals, odp)[0].shape[1]
    assert need > 64
    n_out, (gp, gm, gv) = _gpu_densify(dp, P, m, v, g, count, normals, n, 3, 64)
    assert n_out == need
    assert np.isnan(gp).all() and np.isnan(gm).all() and np.isnan(gv).all()
    n_out, _ = _gpu_densify(dp, P, m, v, g[:0], count[:0], normals[:0], 0, 3, 64)
    assert n_out == 0


def test_densify_stats_matches_oracle():
    """The statistic after a compositing backward on identical records (two
    views in one batch): counts exact, sums within the gradient tolerance;
    cotangents zero on the pixels the oracle calls decision-sensitive."""
    require_gpu()
    m_ = sg()
    cams = _views()
    n = 900
    recs, cat = _records(n, cams, 300, max_radius=14)
    rp = m_.RasterParams()
    orp = R.RasterParams()
    st = Stage(n, cams, rp, cat, 400_000)
    st.rasterize()
    assert st.flags == 0
    rng = np.random.default_rng(8)
    dls, gsum, cnt = [], np.zeros(n), np.zeros(n, np.int64)
    for vi, (rec, cam) in enumerate(zip(recs, cams)):
        comp = lambda rp_: _oracle_composite(rec, cam, rp_, n, vi)[0]
        _, sens = decision_sensitive(comp, orp, DECISION_REL, 1e-5)
        dl = rng.normal(0, 1, (3, cam.width * cam.height))
        dl[:, sens["last"]] = 0.0
        dls.append(dl)
        out, t = _oracle_composite(rec, cam, orp, n, vi, leaf=True)
        (out["rgb"] * torch.tensor(dl.astype(np.float32).astype(np.float64))).sum().backward()
        tx, ty = (cam.width + 15) // 16, (cam.height + 15) // 16
        x0, x1, y0, y1 = (a.numpy() for a in R.tile_rect(rec["u"].astype(np.float64),
                                                           rec["v"].astype(np.float64),
                                                           rec["extent"], 16, 16, tx, ty))
        vis = (x1 > x0) & (y1 > y0) & (rec["extent"][:, 0] >= 0)
        gv = OD.view_space_grad(t["u"].grad.numpy(), t["v"].grad.numpy(), cam.width, cam.height)
        gsum += np.where(vis, gv, 0.0)
        cnt += vis
    st.backward(np.concatenate([d.reshape(-1) for d in dls]).astype(np.float32))
    d_g = torch.zeros(n, device="cuda")
    d_c = torch.zeros(n, dtype=torch.int32, device="cuda")
    m_.densify_stats(cams, n, rp, st.ws, st.cap, d_g, d_c)
    m_.densify_stats(cams, n, rp, st.ws, st.cap, d_g, d_c)   # accumulates
    torch.cuda.synchronize()
    assert np.array_equal(d_c.cpu().numpy(), 2 * cnt)
    assert rel_max_err(d_g.cpu().numpy(), 2 * gsum) < 1e-3
    gate = torch.zeros(1, dtype=torch.int32, device="cuda")
    before = d_g.clone()
    m_.densify_stats(cams, n, rp, st.ws, st.cap, d_g, d_c, gate)   # closed gate: untouched
    torch.cuda.synchronize()
    assert torch.equal(before, d_g)


def test_two_phase_training():
    """Densification until T_d (clone / split / prune every 50 iterations on
    the 1,000-Gaussian scene), then gated training of the fixed set: the set
    changes, no status flag, the gate's backward budget holds."""
    require_gpu()
    m_ = sg()
    from paper_2603_08997_amd import train as T
    gt = S.tiny_scene(S.SEED_TINY_TARGET)
    init = S.tiny_scene(S.SEED_TINY_RENDER)
    cams = S.tetra_cameras()
    rp = m_.RasterParams()
    targets = T.render_targets(gt, cams, rp, 200_000)
    seq = S.view_sequence(S.SEED_VIEW_SEQUENCE, len(cams), 400)
    gate = m_.windowed_gate(len(cams))
    dp = m_.DensifyParams(grad_threshold=1e-4, percent_dense=0.01, scene_extent=4.0,
                          min_opacity=0.05)
    out = T.train_two_phase(init, cams, targets, rp, gate, dp, densify_until=200,
                            densify_every=50, post_iters=200, sequence=seq, log=say)
    say(f"  counts {out['counts']}, post backward {out['post_backward']}/{out['post_iterations']}")
    assert len(out["counts"]) == 5 and len(set(out["counts"])) > 1
    assert out["status_densify"] == 0 and out["status_post"] == 0
    assert out["post_iterations"] == 200
    assert out["post_backward"] >= 100          # >= 50 backward passes per window of 100
    loss = out["trainer"].mean_loss(range(len(cams)))
    assert np.isfinite(loss)
