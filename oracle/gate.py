"""Oracle SkipGS backward gate (plain Python floats = IEEE binary64). Test
infrastructure only.

Sec. 4 of the paper (Algorithm 1; Eqs. 7-13) gates the backward pass of each
post-densification iteration t, counted from t = 1 once densification has
ended. Here the gate is split into what it observes, what it
decides and how its state moves:

* observation: the per-view deviation score of Eq. 8 against the EMA held
  before this iteration, and the backward ratio of Eq. 10 over the
  iterations before this one;
* decision (``decide``): a pure function of the score's proposal (Eq. 9),
  the phase (warmup or gated) and the budget test of Eq. 11 against the
  current floor;
* state: the warmup statistic and the one-time calibration of the floor
  (Eqs. 12-13), the backward count, and the EMA of Eq. 7, which moves on
  every iteration whatever the decision.

Readings where the paper is silent:
* the first observation of a view sets its EMA to that loss (the view is
  then backpropagated, its score being undefined);
* ``delta`` generalises the threshold of Eq. 9 to s > 1 + delta (delta = 0 is the
  paper; delta = 0.02 reads "skip when within 2% of the EMA" one-sidedly);
* the warmup statistic counts only views that already had an EMA;
* with no such view in the warmup the floor stays at rho_lo;
* ``window`` > 0 replaces the cumulative ratio by one over tumbling windows of
  that many iterations aligned at t = 1, window + 1, ...; the count and the
  iteration index restart at each window start;
* ``budget`` = False removes the override (the "w/o budget" ablation);
* a non-finite loss leaves the EMA unchanged and gives g = 0 (sticky flag);
* the loss arrives as float32 and is widened exactly to binary64.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

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
    t: int = 0              # iterations seen
    b: int = 0              # backward passes run
    t_w: int = 0            # iterations and backward passes in the current window
    b_w: int = 0
    warm_hits: int = 0      # warmup statistic: proposals to backpropagate ...
    warm_count: int = 0     # ... out of the warmup iterations that had a score
    rho_min: float = 0.5    # current budget floor
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


# --- observation -----------------------------------------------------------
def deviation_score(p: GateParams, st: GateState, view: int, L: float) -> float:
    """Eq. 8 against the EMA before this iteration; +inf for a view with no EMA."""
    if not st.has_ema[view]:
        return math.inf
    return L / (st.ema[view] + p.eps)


def backward_ratio(p: GateParams, st: GateState) -> float:
    """Eq. 10 over the iterations before the current one (of the current
    window when ``window`` > 0). Called after the clock has advanced."""
    if p.window > 0:
        return st.b_w / max(st.t_w - 1, 1)
    return st.b / max(st.t - 1, 1)


# --- decision --------------------------------------------------------------
def decide(proposal: int, in_warmup: bool, budget: bool, rho: float, rho_min: float) -> int:
    """g of one iteration: the warmup always backpropagates; afterwards the
    proposal of Eq. 9 stands unless the budget floor is enforced and the
    ratio is below it (Eq. 11)."""
    if in_warmup:
        return 1
    if budget and rho < rho_min:
        return 1
    return proposal


# --- state -----------------------------------------------------------------
def advance_clock(p: GateParams, st: GateState):
    st.t += 1
    if p.window > 0 and (st.t - 1) % p.window == 0:
        st.t_w, st.b_w = 0, 0
    st.t_w += 1


def calibrate_floor(p: GateParams, st: GateState):
    """Eqs. 12-13, once, at the first iteration after the warmup."""
    if st.calibrated or not p.calibrate or p.warmup <= 0:
        return
    if st.warm_count > 0:
        st.rho_min = p.rho_lo + (1.0 - p.rho_lo) * (st.warm_hits / st.warm_count)
    st.calibrated = True


def account(st: GateState, g: int):
    st.b += g
    st.b_w += g


def update_ema(p: GateParams, st: GateState, view: int, L: float):
    """Eq. 7 (the first observation initialises the EMA)."""
    if st.has_ema[view]:
        st.ema[view] = p.beta * st.ema[view] + (1.0 - p.beta) * L
    else:
        st.ema[view] = L
        st.has_ema[view] = True


def step(p: GateParams, st: GateState, view: int, loss) -> GateResult:
    """One post-densification iteration of the gate; mutates ``st``."""
    L = float(np.float32(loss))
    advance_clock(p, st)
    if not math.isfinite(L):
        st.nonfinite = True
        return GateResult(0, 0, 0, math.nan, math.nan)
    s = deviation_score(p, st, view, L)
    proposal = 1 if s > 1.0 + p.delta else 0       # +inf always proposes
    rho = backward_ratio(p, st)
    in_warmup = st.t <= p.warmup
    if in_warmup:
        if st.has_ema[view]:
            st.warm_count += 1
            st.warm_hits += proposal
    else:
        calibrate_floor(p, st)
    g = decide(proposal, in_warmup, p.budget, rho, st.rho_min)
    account(st, g)
    update_ema(p, st, view, L)
    return GateResult(g, proposal, int(g == 1 and proposal == 0), s, rho)


def run(p: GateParams, views, losses) -> tuple[GateState, list]:
    st = init_state(p)
    out = [step(p, st, int(v), l) for v, l in zip(views, losses)]
    return st, out
