"""Pins for the oracle Adam step: the first-step closed form and agreement with
torch.optim.Adam in float64 over many steps."""
import numpy as np
import torch

from oracle import adam as A


def test_first_step_closed_form():
    rng = np.random.default_rng(0)
    p0 = rng.normal(size=100)
    g = rng.normal(size=100)
    lr = 1e-3
    p1, m, v = A.adam_step(p0, g, np.zeros(100), np.zeros(100), 1, lr)
    assert np.allclose(p1, p0 - lr * g / (np.abs(g) + A.EPS), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g, atol=1e-17) and np.allclose(v, 0.001 * g * g, atol=1e-20)


def test_matches_torch_adam_float64():
    rng = np.random.default_rng(1)
    p = rng.normal(size=(5, 40))
    lr = np.array([1.6e-4, 5e-3, 1e-3, 2.5e-2, 2.5e-3])[:, None]
    params = [torch.tensor(p[i].copy(), requires_grad=True) for i in range(5)]
    opts = [torch.optim.Adam([params[i]], lr=float(lr[i, 0]), betas=(A.BETA1, A.BETA2), eps=A.EPS)
            for i in range(5)]
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for k in range(1, 31):
        g = rng.normal(size=p.shape) * (1 + k)
        g[:, ::7] = 0.0
        p, m, v = A.adam_step(p, g, m, v, k, lr)
        for i in range(5):
            params[i].grad = torch.tensor(g[i])
            opts[i].step()
    ref = np.stack([q.detach().numpy() for q in params])
    assert np.abs(p - ref).max() < 1e-13
