"""Pins for the oracle SkipGS gate (Algorithm 1, Eqs. 7-13): closed-form
backward counts, a hand-derived trace, warmup calibration and edge cases."""
import math

import numpy as np
import pytest

from oracle import gate as Gt


def _run(p, views, losses):
    st, res = Gt.run(p, views, losses)
    return st, [r.g for r in res], res


def test_constant_loss_cumulative_budget_closed_form():
    """Constant loss, one view, no warmup, rho_min = 0.5: every proposal after
    the first is a skip (s = L/(L + eps) < 1), so only the override runs backward
    and b_t = max(1, floor(t / 2))."""
    p = Gt.GateParams(n_views=1, beta=0.95, warmup=0, calibrate=False)
    st = Gt.init_state(p)
    for t in range(1, 1001):
        Gt.step(p, st, 0, 0.25)
        assert st.b == max(1, t // 2), t


def test_constant_loss_windowed_budget_fifty_per_window():
    p = Gt.windowed_preset(n_views=3)
    st = Gt.init_state(p)
    counts = []
    prev_b = 0
    for t in range(1, 1001):
        Gt.step(p, st, t % 3, 0.5)
        if t % 100 == 0:
            counts.append(st.b - prev_b)
            prev_b = st.b
    # the first window also holds the three first-sight backward passes
    assert counts[0] >= 50 and all(c == 50 for c in counts[1:]), counts


def test_increasing_loss_always_backward():
    p = Gt.GateParams(n_views=4, warmup=10)
    losses = np.linspace(0.1, 0.9, 200)
    views = np.arange(200) % 4
    st, g, _ = _run(p, views, losses)
    assert all(g) and st.b == 200


def test_without_budget_never_backward_on_constant_loss():
    p = Gt.GateParams(n_views=1, warmup=0, calibrate=False, budget=False)
    _, g, _ = _run(p, [0] * 50, [0.3] * 50)
    assert g == [1] + [0] * 49


def test_warmup_calibration():
    """W = 6 warmup iterations over views (0,1,0,1,0,1): the first sight of each
    view is not counted; of the 4 counted proposals, 1 is a backward (the loss
    rise at t = 4), so rho_hat = 1/4 and rho_min = 0.5 + 0.5 / 4 = 0.625."""
    p = Gt.GateParams(n_views=2, beta=0.5, warmup=6)
    views = [0, 1, 0, 1, 0, 1, 0]
    losses = [1.0, 1.0, 0.9, 1.2, 0.5, 0.5, 0.1]
    st, g, res = _run(p, views, losses)
    assert g[:6] == [1] * 6
    assert [r.proposed for r in res[:6]] == [1, 1, 0, 1, 0, 0]
    assert st.warm_count == 4 and st.warm_hits == 1
    assert st.calibrated and st.rho_min == 0.625
    # t = 7: rho = 6 / 6 = 1 >= 0.625 and s < 1 -> skip
    assert g[6] == 0


def test_hand_derived_trace():
    """beta = 0.5, W = 0, rho_min = 0.5, two views:
    t v  L    EMA before  s       proposal rho(t-1)   g  EMA after
    1 0  1.0  -           inf     1        0/1=0      1  1.0
    2 1  2.0  -           inf     1        1/1        1  2.0
    3 0  0.8  1.0         <1      0        2/2=1      0  0.9
    4 0  1.0  0.9         >1      1        2/3        1  0.95
    5 1  1.0  2.0         <1      0        3/4        0  1.5
    6 1  1.2  1.5         <1      0        3/5=0.6    0  1.35
    7 0  0.9  0.95        <1      0        3/6=0.5    0  0.925   (0.5 is not < 0.5)
    8 1  1.0  1.35        <1      0        3/7<0.5    1 (forced)  1.175
    """
    p = Gt.GateParams(n_views=2, beta=0.5, warmup=0, calibrate=False)
    views = [0, 1, 0, 0, 1, 1, 0, 1]
    losses = [1.0, 2.0, 0.8, 1.0, 1.0, 1.2, 0.9, 1.0]
    st, g, res = _run(p, views, losses)
    assert g == [1, 1, 0, 1, 0, 0, 0, 1]
    assert [r.forced for r in res] == [0, 0, 0, 0, 0, 0, 0, 1]
    assert st.b == 4 and st.t == 8
    f = lambda x: float(np.float32(x))
    assert st.ema[0] == pytest.approx(0.5 * (0.5 * (0.5 * f(1.0) + 0.5 * f(0.8)) + 0.5 * f(1.0)) + 0.5 * f(0.9), abs=1e-15)
    assert st.ema[1] == pytest.approx(0.5 * (0.5 * (0.5 * f(2.0) + 0.5 * f(1.0)) + 0.5 * f(1.2)) + 0.5 * f(1.0), abs=1e-15)


def test_score_uses_ema_before_update_and_delta_threshold():
    p = Gt.GateParams(n_views=1, beta=0.9, delta=0.02, warmup=0, calibrate=False, budget=False)
    st = Gt.init_state(p)
    Gt.step(p, st, 0, 1.0)
    r = Gt.step(p, st, 0, 1.015)     # within 2%: skip
    assert r.g == 0
    r = Gt.step(p, st, 0, 1.1)       # EMA now 0.9*1 + 0.1*1.015 = 1.0015; 1.1 > 1.02*1.0015
    assert r.g == 1
    assert st.ema[0] == pytest.approx(0.9 * (0.9 * 1.0 + 0.1 * float(np.float32(1.015))) + 0.1 * float(np.float32(1.1)))


def test_nonfinite_loss_keeps_ema_and_skips():
    p = Gt.GateParams(n_views=1, warmup=5)
    st = Gt.init_state(p)
    Gt.step(p, st, 0, 0.5)
    r = Gt.step(p, st, 0, math.nan)
    assert r.g == 0 and st.nonfinite and st.ema[0] == 0.5 and st.t == 2 and st.b == 1
    r = Gt.step(p, st, 0, math.inf)
    assert r.g == 0 and st.t == 3


def test_no_warmup_keeps_rho_lo():
    p = Gt.GateParams(n_views=2, warmup=0, rho_lo=0.5, calibrate=True)
    st, _, _ = _run(p, [0, 1] * 20, [0.4] * 40)
    assert st.rho_min == 0.5


def test_warmup_with_no_history_keeps_rho_lo():
    p = Gt.GateParams(n_views=10, warmup=5)
    st, _, _ = _run(p, [0, 1, 2, 3, 4, 5], [0.3] * 6)
    assert st.warm_count == 0 and st.rho_min == 0.5 and st.calibrated
