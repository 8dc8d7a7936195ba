"""Parity of the loss (Eq. 6), the gate (Algorithm 1) and Adam with the oracle."""
import math

import numpy as np
import pytest
import torch

from oracle import adam as A
from oracle import gate as Gt
from oracle import loss as Lm
from tests.gpu_util import rel_max_err, rel_norm_err, require_gpu, say, sg, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape", [(64, 64), (83, 37), (1, 5), (250, 171)])
def test_loss_and_gradient_match_oracle(shape):
    require_gpu()
    m = sg()
    h, w = shape
    rng = np.random.default_rng(h * 1000 + w)
    x = rng.uniform(0, 1, (3, h, w)).astype(np.float32)
    y = np.clip(x + rng.normal(0, 0.15, x.shape), 0, 1).astype(np.float32)
    say(f"loss {shape}")
    ws = m.alloc_bytes(m.loss_workspace_size(w, h)).zero_()
    d_loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    dx, dy = to_dev(x), to_dev(y)
    m.photometric_loss(dx, dy, w, h, 0.2, ws, d_loss)
    dl = torch.zeros_like(dx)
    m.photometric_loss_backward(dx, dy, w, h, 0.2, ws, None, dl)
    torch.cuda.synchronize()
    L_ref, g_ref = Lm.photometric_loss_and_grad(x.astype(np.float64), y.astype(np.float64))
    assert abs(d_loss.item() - L_ref) <= 1e-5 * abs(L_ref)
    g = dl.cpu().numpy()
    g_ref = g_ref.numpy()
    assert rel_norm_err(g, g_ref) < 1e-4
    assert rel_max_err(g, g_ref) < 1e-4


def test_loss_is_bit_reproducible_and_gate_closed_backward_skips():
    require_gpu()
    m = sg()
    h, w = 97, 131
    rng = np.random.default_rng(0)
    x = to_dev(rng.uniform(0, 1, (3, h, w)).astype(np.float32))
    y = to_dev(rng.uniform(0, 1, (3, h, w)).astype(np.float32))
    ws = m.alloc_bytes(m.loss_workspace_size(w, h)).zero_()
    vals = []
    for _ in range(5):
        d = torch.zeros(1, device="cuda")
        m.photometric_loss(x, y, w, h, 0.2, ws, d)
        vals.append(d.item())
    assert len(set(vals)) == 1
    dl = torch.full_like(x, 3.0)
    gate = torch.zeros(1, dtype=torch.int32, device="cuda")
    m.photometric_loss_backward(x, y, w, h, 0.2, ws, gate, dl)
    torch.cuda.synchronize()
    assert bool((dl == 3.0).all())


def _gpu_gate_run(p, views, losses):
    m = sg()
    state = m.alloc_bytes(m.gate_state_size(p))
    m.gate_init(p, state)
    d_losses = to_dev(np.asarray(losses, np.float32))
    d_views = to_dev(np.asarray(views, np.int32))
    gates = torch.full((len(views),), -1, dtype=torch.int32, device="cuda")
    for t in range(len(views)):
        m.gate_update(p, state, d_views[t:t + 1], d_losses[t:t + 1], gates[t:t + 1])
    snap = m.gate_read(p, state)
    return gates.cpu().numpy(), snap


def _oracle_params(p):
    return Gt.GateParams(n_views=p.n_views, beta=p.beta, eps=p.eps, delta=p.delta, rho_lo=p.rho_lo,
                         warmup=p.warmup, window=p.window, calibrate=p.calibrate, budget=p.budget)


@pytest.mark.parametrize("preset", ["paper", "windowed", "no_budget", "short_warmup"])
def test_gate_replay_bit_exact(preset):
    require_gpu()
    m = sg()
    n_views = 12
    T = 1500
    if preset == "paper":
        p = m.paper_gate(n_views)
    elif preset == "windowed":
        p = m.windowed_gate(n_views)
    elif preset == "no_budget":
        p = m.GateParams(n_views=n_views, warmup=50, budget=False)
    else:
        p = m.GateParams(n_views=n_views, warmup=37, beta=0.8, delta=0.01)
    rng = np.random.default_rng(42)
    views = rng.integers(0, n_views, T)
    base = 0.3 * np.exp(-np.arange(T) / 800.0)
    losses = (base * (1 + 0.05 * rng.normal(size=T))).astype(np.float32)
    say(f"gate replay {preset}")
    g_gpu, snap = _gpu_gate_run(p, views, losses)
    st, res = Gt.run(_oracle_params(p), views, losses)
    assert list(g_gpu) == [r.g for r in res]
    assert snap["b"] == st.b and snap["t"] == st.t
    assert snap["warm_hits"] == st.warm_hits and snap["warm_count"] == st.warm_count
    assert snap["rho_min"] == st.rho_min and bool(snap["calibrated"]) == st.calibrated
    assert np.array_equal(snap["ema"], np.asarray(st.ema))        # bitwise binary64
    assert list(snap["has_ema"].astype(bool)) == st.has_ema
    assert snap["last_forced"] == res[-1].forced and snap["last_proposed"] == res[-1].proposed


def test_gate_nonfinite_loss():
    """W = 3. t=1: first sight, backward (b=1). t=2: NaN, skip. t=3: first
    sight of view 1, backward (b=2). t=4: inf, skip. t=5: s = 0.3/0.5 < 1, no
    warmup history so rho_min stays 0.5, rho = 2/4 is not below it: skip."""
    require_gpu()
    m = sg()
    p = m.GateParams(n_views=2, warmup=3)
    losses = np.array([0.5, np.nan, 0.4, np.inf, 0.3], np.float32)
    views = [0, 0, 1, 1, 0]
    g_gpu, snap = _gpu_gate_run(p, views, losses)
    st, res = Gt.run(_oracle_params(p), views, losses)
    assert list(g_gpu) == [r.g for r in res] == [1, 0, 1, 0, 0]
    assert snap["flags"] & m.STATUS_NONFINITE_LOSS
    assert np.array_equal(snap["ema"], np.asarray(st.ema))


def test_gate_out_of_range_view_is_flagged_and_not_an_iteration():
    """A device view index outside [0, n_views) leaves the state as it was
    (no clock tick, no count, no EMA change), gives g = 0 and sets the bad-view
    flag; the following iterations match the oracle run without it."""
    require_gpu()
    m = sg()
    p = m.GateParams(n_views=3, warmup=2)
    views = [0, 1, 7, 2, -1, 0, 1]
    losses = np.array([0.5, 0.4, 0.3, 0.45, 0.2, 0.49, 0.41], np.float32)
    g_gpu, snap = _gpu_gate_run(p, views, losses)
    keep = [i for i, v in enumerate(views) if 0 <= v < 3]
    st, res = Gt.run(_oracle_params(p), [views[i] for i in keep], losses[keep])
    assert [int(g_gpu[i]) for i in (2, 4)] == [0, 0]
    assert [int(g_gpu[i]) for i in keep] == [r.g for r in res]
    assert snap["t"] == st.t == 5 and snap["b"] == st.b
    assert snap["flags"] & m.STATUS_BAD_VIEW
    assert np.array_equal(snap["ema"], np.asarray(st.ema))


@pytest.mark.parametrize("n", [1, 100, 5000])
def test_adam_matches_oracle(n):
    require_gpu()
    m = sg()
    deg = 1
    F = 11 + 3 * 4
    stride = max(64, (n + 63) // 64 * 64)
    rng = np.random.default_rng(n)
    p = np.zeros((F, stride), np.float32)
    g = np.zeros((F, stride), np.float32)
    mm = np.zeros((F, stride), np.float32)
    vv = np.zeros((F, stride), np.float32)
    p[:, :n] = rng.normal(size=(F, n))
    lrs = np.array(m.default_lrs(deg), np.float64)
    dp, dg, dm, dv = (to_dev(a) for a in (p, g, mm, vv))
    step = torch.zeros(1, dtype=torch.int32, device="cuda")
    gate = torch.ones(1, dtype=torch.int32, device="cuda")
    ap = m.AdamParams(lr=tuple(lrs))
    ref_p, ref_m, ref_v = p.astype(np.float64), mm.astype(np.float64), vv.astype(np.float64)
    for k in range(1, 6):
        gk = np.zeros((F, stride), np.float32)
        gk[:, :n] = rng.normal(size=(F, n)) * 10.0 ** rng.uniform(-6, 0, (F, n))
        dg.copy_(to_dev(gk))
        gate.fill_(1 if k != 3 else 0)
        m.adam_step(ap, dp, dg, dm, dv, n, step, gate)
        torch.cuda.synchronize()
        # a closed gate leaves the gradient in place; an open one clears it
        assert bool((dg == to_dev(gk)).all()) if k == 3 else not bool(dg.any())
        if k != 3:
            kk = k if k < 3 else k - 1
            ref_p, ref_m, ref_v = A.adam_step(ref_p, gk, ref_m, ref_v, kk, lrs[:, None])
    torch.cuda.synchronize()
    assert step.item() == 4
    got_p = dp.cpu().numpy().astype(np.float64)
    upd = np.abs(ref_p - p)
    assert np.all(np.abs(got_p - ref_p) <= 1e-6 * np.abs(ref_p) + 1e-4 * upd + 1e-12)
    assert rel_max_err(dm.cpu().numpy(), ref_m) < 1e-5
    assert rel_max_err(dv.cpu().numpy(), ref_v) < 1e-5
