"""Captured HIP graphs against eager launches and the oracle.

* A whole training iteration (sgs_view_sequence_next + sgs_train_iteration:
  render, loss, gate on the device, predicated backward and Adam) captured
  once and replayed over the device view sequence: each replay is checked
  against an eager execution of the same iteration from the same state (the
  eager run, a restore and a synchronisation sit between replays). Forward,
  loss and gate are bit-identical; parameters and moments too when the gate
  skips the backward, and within float-atomic reordering when it runs.
* A batched forward of views of different resolutions captured once: every
  replay equals the eager render bit for bit, and the image matches the
  oracle on every pixel the oracle does not call decision-sensitive."""
import numpy as np
import pytest
import torch

from oracle import render as R
from paper_2603_08997_amd import scenes as S
from tests.gpu_util import require_gpu, say, sg, to_dev
from tests.sensitivity import oracle_view_masks

pytestmark = pytest.mark.gpu


def _capture(fn):
    """A graph of fn(stream), captured on a side stream after one eager call
    there."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn(s.cuda_stream)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        fn(s.cuda_stream)
    torch.cuda.synchronize()
    return g


def test_training_iteration_graph_replays_match_eager():
    require_gpu()
    from paper_2603_08997_amd.train import Trainer, measure_capacity, render_targets
    m = sg()
    gt = S.mixture_scene(S.SEED_SCENE, 3000, sh_degree=1, log_scale_mean=-3.0)
    init = S.perturb(gt, S.SEED_INIT_PERTURB)
    cams = S.hemisphere_cameras(S.SEED_CAMERAS, 6, 96, 64)
    rp = m.RasterParams()
    cap = int(measure_capacity(gt, cams, rp) * 1.5) + 4096
    targets = render_targets(gt, cams, rp, cap)
    gp = m.GateParams(n_views=len(cams), warmup=2)
    seq = np.array([0, 3, 1, 4, 2, 5, 0, 3], np.int32)
    tr = Trainer(init, cams, targets, rp, gp, cap, gated=True, sequence=seq)
    graph = _capture(tr.step)   # two iterations of the sequence
    state = lambda: [tr.planes, tr.m, tr.v, tr.step_count, tr.gstate, tr.seq_pos]
    flips = 0
    for r in range(6):
        snap = [t.clone() for t in state()]
        tr.step()
        torch.cuda.synchronize()
        eager = {"rgb": tr.rgb.clone(), "loss": tr.loss.clone(), "gate": tr.gate.clone(),
                 "view": tr.view.clone(), "gstate": tr.gstate.clone(), "planes": tr.planes.clone(),
                 "m": tr.m.clone(), "v": tr.v.clone(), "step": tr.step_count.clone()}
        for t, s in zip(state(), snap):
            t.copy_(s)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        say(f"replay {r}: view {tr.view.item()} gate {tr.gate.item()} loss {tr.loss.item():.6f}")
        now = {"rgb": tr.rgb, "loss": tr.loss, "gate": tr.gate, "view": tr.view,
               "gstate": tr.gstate, "step": tr.step_count}
        for k, t in now.items():
            assert torch.equal(t, eager[k]), (r, k)
        for k, t in (("planes", tr.planes), ("m", tr.m), ("v", tr.v)):
            if tr.gate.item() == 0:
                assert torch.equal(t, eager[k]), (r, k)
            else:
                a, b = t.cpu().numpy(), eager[k].cpu().numpy()
                assert np.abs(a - b).max() <= 1e-5 * max(np.abs(b).max(), 1e-30), (r, k)
        flips += int(tr.gate.item() == 0)
    flags, _, _ = m.read_status(tr.ws)
    assert flags == 0
    say(f"  replays with the backward skipped: {flips} of 6")


def test_batched_forward_graph_replays_match_eager_and_oracle():
    require_gpu()
    m = sg()
    sc = S.mixture_scene(S.SEED_SCENE, 3000, sh_degree=3, log_scale_mean=-3.0)
    base = S.hemisphere_cameras(S.SEED_CAMERAS, 3, 96, 64)
    sizes = [(96, 64), (64, 48), (80, 80)]
    cams = [S.hemisphere_cameras(S.SEED_CAMERAS, 3, w, h)[k] for k, (w, h) in enumerate(sizes)]
    rp = m.RasterParams()
    planes = to_dev(sc.to_planes())
    cap = 400_000
    ws = m.alloc_bytes(m.forward_workspace_size(rp, sc.n, cams, cap)).zero_()
    m.clear_status(ws)
    px = sum(c.width * c.height for c in cams)
    eager = torch.zeros(3 * px, device="cuda")
    m.render_forward(planes, sc.n, 3, cams, rp, ws, cap, eager)
    torch.cuda.synchronize()
    assert m.read_status(ws)[0] == 0
    out = torch.zeros(3 * px, device="cuda")
    graph = _capture(lambda s: m.render_forward(planes, sc.n, 3, cams, rp, ws, cap, out,
                                                stream=torch.cuda.current_stream()))
    other = torch.zeros(3 * base[0].width * base[0].height, device="cuda")
    ws2 = m.alloc_bytes(m.forward_workspace_size(rp, sc.n, base[:1], cap)).zero_()
    for r in range(3):
        out.fill_(-1.0)
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), r
        # eager work of the program between replays
        m.render_forward(planes, sc.n, 3, base[:1], rp, ws2, cap, other)
        torch.cuda.synchronize()
    img = eager.cpu().numpy()
    off = 0
    for v, cam in enumerate(cams):
        n_px = cam.width * cam.height
        got = img[3 * off:3 * (off + n_px)].reshape(3, n_px)
        ref, colour, _ = oracle_view_masks(sc, cam, R.RasterParams(), 3e-5, 1e-5)
        ok = ~colour
        err = np.abs(got[:, ok] - ref[:, ok]).max() / max(np.abs(ref).max(), 1e-30)
        say(f"  view {v} {cam.width}x{cam.height}: rel max err {err:.2e}, "
            f"{int(colour.sum())} sensitive pixels")
        assert err <= 1e-5
        off += n_px
