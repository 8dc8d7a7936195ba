"""Oracle Adam step (FP64). Test infrastructure only.

The paper trains with the standard 3DGS optimiser, Adam (Sec. 3, Sec. 5.1),
and applies the update only when backward runs (Algorithm 1). Adam as defined
by Kingma and Ba, with bias correction:
    m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
    p <- p - lr * (m / (1 - b1^k)) / (sqrt(v / (1 - b2^k)) + eps)
where k counts executed steps. Readings: b1 = 0.9, b2 = 0.999, eps = 1e-15,
one learning rate per parameter plane.
"""
from __future__ import annotations

import numpy as np

BETA1 = 0.9
BETA2 = 0.999
EPS = 1e-15


def adam_step(p, g, m, v, k: int, lr, beta1=BETA1, beta2=BETA2, eps=EPS):
    """One update; arrays of equal shape (float64 copies are returned). ``lr``
    may be a scalar or broadcastable to p (per-plane rates)."""
    p = np.asarray(p, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** k)
    v_hat = v / (1.0 - beta2 ** k)
    p = p - np.asarray(lr, dtype=np.float64) * m_hat / (np.sqrt(v_hat) + eps)
    return p, m, v
