"""Oracle SkipGS backward gate (plain Python floats = IEEE binary64). Test
infrastructure only.

Algorithm 1 of the paper, one call per post-densification iteration t
(t = 1 at the first iteration after densification stops, Sec. 4):

1. deviation score s = L / (EMA_v + eps) if view v has an EMA, else +inf (Eq. 8);
2. skip test g = 1[s > 1] (Eq. 9);
3. cumulative backward ratio before this iteration rho = b / max(t - 1, 1) (Eq. 10);
4. warmup (t <= W): record g for calibration when the view already had an EMA,
   then force g = 1;
5. after warmup: at t = W + 1 calibrate once rho_min = rho_lo + (1 - rho_lo) rho_hat_W
   (Eqs. 12-13); if rho < rho_min force g = 1 (Eq. 11);
6. if g = 1 the backward and optimiser step run and b += 1;
7. EMA_v <- beta EMA_v + (1 - beta) L, unconditionally (Eq. 7).

Readings where the paper is silent:
* the first observation of a view sets its EMA to that loss;
* ``delta`` generalises the threshold of Eq. 9 to s > 1 + delta (delta = 0 is the
  paper; delta = 0.02 reads "skip when within 2% of the EMA" one-sidedly);
* ``window`` > 0 replaces the cumulative ratio by one over tumbling windows of
  that many iterations aligned at t = 1, window + 1, ...; the count and the
  iteration index restart at each window start;
* ``budget`` = False removes the override (the "w/o budget" ablation);
* a non-finite loss leaves the EMA unchanged and gives g = 0 (sticky flag);
* the loss arrives as float32 and is widened exactly to binary64.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class GateParams:
    n_views: int
    beta: float = 0.95
    eps: float = 1e-8
    delta: float = 0.0
    rho_lo: float = 0.5
    warmup: int = 500
    window: int = 0
    calibrate: bool = True
    budget: bool = True


def paper_preset(n_views: int) -> GateParams:
    """Sec. 5.1: W = 500, beta = 0.95, eps = 1e-8, rho_lo = 0.5, calibrated."""
    return GateParams(n_views=n_views, beta=0.95, eps=1e-8, delta=0.0, rho_lo=0.5,
                      warmup=500, window=0, calibrate=True, budget=True)


def windowed_preset(n_views: int) -> GateParams:
    """EMA decay 0.9, skip when within 2% of the EMA, at least 50% backward per
    100-iteration window, no warmup."""
    return GateParams(n_views=n_views, beta=0.9, eps=1e-8, delta=0.02, rho_lo=0.5,
                      warmup=0, window=100, calibrate=False, budget=True)


@dataclass
class GateState:
    ema: list
    has_ema: list
    t: int = 0
    b: int = 0
    t_w: int = 0
    b_w: int = 0
    warm_hits: int = 0
    warm_count: int = 0
    rho_min: float = 0.5
    calibrated: bool = False
    nonfinite: bool = False


def init_state(p: GateParams) -> GateState:
    return GateState(ema=[0.0] * p.n_views, has_ema=[False] * p.n_views, rho_min=p.rho_lo)


@dataclass
class GateResult:
    g: int
    proposed: int
    forced: int
    s: float
    rho: float


def step(p: GateParams, st: GateState, view: int, loss) -> GateResult:
    """One iteration of Algorithm 1; mutates ``st``."""
    L = float(np.float32(loss))
    st.t += 1
    t = st.t
    if p.window > 0 and (t - 1) % p.window == 0:
        st.t_w = 0
        st.b_w = 0
    st.t_w += 1

    if not math.isfinite(L):
        st.nonfinite = True
        return GateResult(0, 0, 0, math.nan, math.nan)

    had = st.has_ema[view]
    if had:
        s = L / (st.ema[view] + p.eps)
        g = 1 if s > 1.0 + p.delta else 0
    else:
        s = math.inf
        g = 1
    proposed = g

    if p.window > 0:
        rho = st.b_w / max(st.t_w - 1, 1)
    else:
        rho = st.b / max(t - 1, 1)

    if t <= p.warmup:
        if had:
            st.warm_count += 1
            st.warm_hits += g
        g = 1
    else:
        if p.calibrate and p.warmup > 0 and not st.calibrated:
            if st.warm_count > 0:
                rho_hat = st.warm_hits / st.warm_count
                st.rho_min = p.rho_lo + (1.0 - p.rho_lo) * rho_hat
            st.calibrated = True
        if p.budget and rho < st.rho_min:
            g = 1

    if g:
        st.b += 1
        st.b_w += 1
    if had:
        st.ema[view] = p.beta * st.ema[view] + (1.0 - p.beta) * L
    else:
        st.ema[view] = L
        st.has_ema[view] = True
    return GateResult(g, proposed, int(g and not proposed), s, rho)


def run(p: GateParams, views, losses) -> tuple[GateState, list]:
    st = init_state(p)
    out = [step(p, st, int(v), l) for v, l in zip(views, losses)]
    return st, out
