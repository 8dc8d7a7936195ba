"""The launch-shape tuner: it times every candidate (tile shape x LDS batch x
super-tile), picks the fastest, stores the choice and reuses it; and every
candidate renders the same image bit for bit (the launch shape changes how
the work is laid out, never the result)."""
import json

import numpy as np
import pytest
import torch

from paper_2603_08997_amd import scenes as S
from tests.gpu_util import require_gpu, say, sg, to_dev

pytestmark = pytest.mark.gpu


def test_tuner_picks_stores_and_reuses(tmp_path):
    require_gpu()
    m = sg()
    from paper_2603_08997_amd import tune as T
    sc = S.mixture_scene(S.SEED_SCENE, 3000, sh_degree=3, log_scale_mean=-3.0)
    cams = [S.hemisphere_cameras(S.SEED_CAMERAS, 2, 96, 64)[0],
            S.hemisphere_cameras(S.SEED_CAMERAS, 2, 80, 80)[1]]
    planes = to_dev(sc.to_planes())
    px = sum(c.width * c.height for c in cams)
    dl = torch.randn(3 * px, device="cuda", generator=torch.Generator(device="cuda").manual_seed(3))
    store = str(tmp_path / "tuned.json")
    rp, rec = T.tune(planes, sc.n, 3, cams, dl, store=store)
    assert not rec["reused"]
    n_cand = len(T.TILES) * len(T.BATCHES) * len(T.SUPER_TILES)
    assert len(rec["trials"]) == n_cand
    best = min(rec["trials"], key=lambda t: t["ms"])
    assert (rp.tile_w, rp.tile_h, rp.lds_batch, rp.super_tile) == \
        (best["tile_w"], best["tile_h"], best["lds_batch"], best["super_tile"])
    say(f"tuned {rec['choice']} {rec['ms']:.3f} ms")
    table = json.load(open(store))
    assert T.workload_key(sc.n, 3, cams) in table
    rp2, rec2 = T.tune(planes, sc.n, 3, cams, dl, store=store)
    assert rec2["reused"] and rp2 == rp
    # every candidate's image equals the default launch's bit for bit
    images = []
    for tr in rec["trials"]:
        r = m.RasterParams(tile_w=tr["tile_w"], tile_h=tr["tile_h"], lds_batch=tr["lds_batch"],
                           super_tile=tr["super_tile"])
        cap = 400_000
        ws = m.alloc_bytes(m.forward_workspace_size(r, sc.n, cams, cap)).zero_()
        out = torch.zeros(3 * px, device="cuda")
        m.render_forward(planes, sc.n, 3, cams, r, ws, cap, out)
        torch.cuda.synchronize()
        assert m.read_status(ws)[0] == 0
        images.append(out.cpu().numpy())
    for img in images[1:]:
        assert np.array_equal(img, images[0])
