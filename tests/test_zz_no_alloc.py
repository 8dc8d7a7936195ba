"""The workspace-free loss entry point (for callers that cannot allocate):
through the C ABI, bit-identical to sgs_photometric_loss on two calls in a
row, the second on a smaller image, and rejecting an image beyond its static
scratch before enqueueing anything."""
import numpy as np
import pytest
import torch

from tests.gpu_util import require_gpu, say, sg, to_dev

pytestmark = pytest.mark.gpu


def _images(seed, w, h):
    rng = np.random.default_rng(seed)
    x = rng.random((3, h, w), dtype=np.float32)
    y = np.clip(x + rng.normal(0, 0.1, x.shape).astype(np.float32), 0, 1)
    return to_dev(x.reshape(-1)), to_dev(y.reshape(-1))


def test_static_loss_matches_workspace_loss_twice():
    require_gpu()
    m = sg()
    for k, (w, h, lam) in enumerate([(1600, 1060, 0.2), (333, 217, 0.7)]):
        say(f"static loss call {k}: {w}x{h} lambda={lam}")
        x, y = _images(40 + k, w, h)
        ws = m.alloc_bytes(m.loss_workspace_size(w, h))
        ref = torch.full((1,), -1.0, device="cuda")
        got = torch.full((1,), -2.0, device="cuda")
        m.photometric_loss(x, y, w, h, lam, ws, ref)
        m.photometric_loss_static(x, y, w, h, lam, got)
        torch.cuda.synchronize()
        assert got.item() == ref.item(), (k, got.item(), ref.item())
        assert 0.0 < got.item() < 1.0


def test_static_loss_rejects_images_beyond_the_scratch():
    require_gpu()
    m = sg()
    w, h = 4097, 4096   # 257 x 256 tiles of 16x16 > 65536
    d = torch.zeros(1, device="cuda")
    with pytest.raises(m.SkipGSError) as e:
        m.photometric_loss_static(d, d, w, h, 0.2, d)
    assert e.value.status == 3 and "static scratch" in str(e.value)
