"""Stage parity on identical float32 records: tile binning and sort (bit
exact), compositing forward (1e-5) and backward (1e-3) against the oracle."""
import numpy as np
import pytest
import torch

from oracle import render as R
from paper_2603_08997_amd import scenes as S
from tests.gpu_util import (region, rel_max_err, rel_norm_err, require_gpu, say, sg, split_views,
                            to_dev)

pytestmark = pytest.mark.gpu

TILES = [(16, 16), (8, 8), (32, 8)]


def _views():
    return [S.look_at_camera((3.0, 1.0, 1.0), 83, 61), S.look_at_camera((0.5, -3.0, 2.0), 48, 33)]


def _records(n, cams, seed, **kw):
    recs = [S.random_records(seed + v, n, c.width, c.height, **kw) for v, c in enumerate(cams)]
    cat = {k: np.concatenate([r[k] for r in recs]) for k in recs[0]}
    return recs, cat


class Stage:
    def __init__(self, n, cams, rp, cat, capacity):
        m = sg()
        self.m, self.n, self.cams, self.rp, self.cap = m, n, cams, rp, capacity
        self.ws = m.alloc_bytes(m.forward_workspace_size(rp, n, cams, capacity))
        self.ws.zero_()
        self.L = m.get_workspace_layout(rp, n, cams, capacity)
        d = {k: to_dev(v) for k, v in cat.items()}
        m.load_records(cams, n, rp, self.ws, capacity, d["u"], d["v"], d["depth"], d["extent"],
                       d["conic"], d["opacity"], d["rgb"])
        m.bin(cams, n, rp, self.ws, capacity)
        self.flags, self.vis, self.pairs = m.read_status(self.ws)
        self.kept = m.read_counters(self.ws)["pairs_kept"]

    def lists(self):
        P = self.kept
        kt = np.uint16 if self.L.pair_tile_bytes == 2 else np.uint32
        tiles = region(self.ws, self.L.pair_tile, P, kt).astype(np.uint32)
        ents = region(self.ws, self.L.pair_entry, P, np.uint32)
        ranges = region(self.ws, self.L.ranges, 2 * self.L.total_tiles, np.uint32).reshape(-1, 2)
        return tiles, ents, ranges

    def rasterize(self):
        px = sum(c.width * c.height for c in self.cams)
        self.rgb = torch.zeros(3 * px, dtype=torch.float32, device="cuda")
        self.m.rasterize(self.cams, self.n, self.rp, self.ws, self.cap, self.rgb)
        torch.cuda.synchronize()
        tf = region(self.ws, self.L.t_final, self.L.total_pixels, np.float32)
        nl = region(self.ws, self.L.n_last, self.L.total_pixels, np.uint32)
        return self.rgb.cpu().numpy(), tf, nl

    def backward(self, dl):
        self.m.rasterize_backward(self.cams, self.n, self.rp, self.ws, self.cap, to_dev(dl))
        torch.cuda.synchronize()
        return region(self.ws, self.L.accum, 12 * self.L.entries, np.float32).reshape(-1, 12)


def _oracle_bins(recs, cams, n, tw, th):
    keys, vals, ranges = [], [], []
    off = 0
    for v, (r, c) in enumerate(zip(recs, cams)):
        k, val, rg = R.bin_and_sort(r["u"], r["v"], r["depth"], r["extent"], v * n + np.arange(n),
                                    c.width, c.height, tw, th, tile_offset=off)
        base = sum(len(x) for x in keys)
        rg = np.where(rg[:, 1:2] > rg[:, 0:1], rg + base, 0)
        keys.append(k); vals.append(val); ranges.append(rg)
        off += ((c.width + tw - 1) // tw) * ((c.height + th - 1) // th)
    return np.concatenate(keys), np.concatenate(vals), np.concatenate(ranges)


@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("ties", [0.0, 0.4])
def test_binning_bit_exact(tile, ties):
    require_gpu()
    st = _check_binning(_views(), tile, ties, 1500, 100 + int(ties * 10))
    assert st.L.pair_tile_bytes == 2   # few tiles: uint16 tile keys


def test_binning_bit_exact_wide_tile_keys():
    """79,800 tiles (three 1600x1060 views, 8x8 tiles): uint32 tile keys."""
    require_gpu()
    cams = [S.look_at_camera(p, 1600, 1060) for p in ((3.0, 1.0, 1.0), (0.5, -3.0, 2.0),
                                                        (-2.0, 2.0, 1.5))]
    st = _check_binning(cams, (8, 8), 0.2, 1500, 131)
    assert st.L.pair_tile_bytes == 4


def _check_binning(cams, tile, ties, n, seed):
    m = sg()
    tw, th = tile
    recs, cat = _records(n, cams, seed, max_radius=20, tie_fraction=ties)
    say(f"binning tile={tile} ties={ties} n={n} views={len(cams)}")
    rp = m.RasterParams(tile_w=tw, tile_h=th)
    st = Stage(n, cams, rp, cat, 400_000)
    assert st.flags == 0
    keys, vals, ranges = _oracle_bins(recs, cams, n, tw, th)
    tiles, ents, granges = st.lists()
    # the pair count the capacity must cover is that of the box lists
    assert st.pairs == len(keys)
    assert st.kept <= st.pairs and len(ents) == st.kept
    # the GPU lists are the box lists less entries that fail the exact tile
    # test: per tile, a subsequence of the oracle's list that keeps every
    # entry able to contribute to a pixel of the tile, in the same order
    orp = R.RasterParams(tile_w=tw, tile_h=th)
    gtiles = (keys >> np.uint64(32)).astype(np.int64)
    assert np.array_equal(tiles.astype(np.int64),
                          np.repeat(np.arange(len(granges)), granges[:, 1] - granges[:, 0]))
    toff, dropped, dropped_dead, dead = 0, 0, 0, 0
    for v, (rec, cam) in enumerate(zip(recs, cams)):
        tx_n = (cam.width + tw - 1) // tw
        ty_n = (cam.height + th - 1) // th
        for t in range(toff, toff + tx_n * ty_n):
            lo, hi = ranges[t]
            olist = vals[lo:hi]
            glist = ents[granges[t][0]:granges[t][1]].astype(np.int64)
            assert np.all(gtiles[lo:hi] == t)
            keep = np.isin(olist, glist)
            assert np.array_equal(olist[keep], glist)          # ordered subsequence
            tx, ty = (t - toff) % tx_n, (t - toff) // tx_n
            for e, kept in zip(olist, keep):
                i = e - v * n
                live = R.tile_contributes(rec["u"][i], rec["v"][i], *rec["conic"][i],
                                          rec["opacity"][i], *rec["extent"][i], tx, ty, tw, th,
                                          cam.width, cam.height, orp)
                assert kept or not live, (t, e)
                dead += int(not live)
                dropped += int(not kept)
        toff += tx_n * ty_n
    say(f"  box pairs {len(vals)}, kept {len(ents)}, non-contributing {dead}, dropped {dropped}")
    assert dropped >= 0.5 * dead
    return st


def test_binning_empty_and_capacity_overflow():
    require_gpu()
    m = sg()
    cams = _views()
    n = 300
    recs, cat = _records(n, cams, 7, max_radius=15)
    cat["extent"][:] = -1                      # nothing visible
    st = Stage(n, cams, m.RasterParams(), cat, 1000)
    assert st.flags == 0 and st.vis == 0 and st.pairs == 0
    _, _, ranges = st.lists()
    assert not ranges.any()
    recs, cat = _records(n, cams, 8, max_radius=15)
    st = Stage(n, cams, m.RasterParams(), cat, 64)   # far too small
    assert st.flags & m.STATUS_PAIR_OVERFLOW
    assert st.pairs > 64


def _oracle_composite(rec, cam, rp, n, view, leaf=False):
    t = {k: torch.tensor(np.asarray(rec[k], np.float64), requires_grad=leaf)
         for k in ("u", "v", "conic", "opacity", "rgb")}
    uv = torch.stack([t["u"], t["v"]], 1)
    out = R.composite(uv, t["conic"], t["opacity"], t["rgb"], torch.tensor(rec["depth"], dtype=torch.float64),
                      torch.tensor(rec["extent"].astype(np.int64)), view * n + torch.arange(n),
                      cam.width, cam.height, rp)
    return out, t


@pytest.mark.parametrize("tile", TILES)
def test_raster_forward_and_backward_match_oracle(tile):
    require_gpu()
    _check_raster(tile)


def test_raster_nondefault_params_match_oracle():
    """alpha_min = 0 (no skip threshold: log2 alpha_min = -inf, no exact tile
    culling), alpha_max = 0.9 and t_min = 1e-3."""
    require_gpu()
    _check_raster((16, 16), alpha_min=0.0, alpha_max=0.9, t_min=1e-3)


def _check_raster(tile, **params):
    m = sg()
    tw, th = tile
    cams = _views()
    n = 900
    recs, cat = _records(n, cams, 300, max_radius=14)
    bg = (0.2, 0.4, 0.6)
    say(f"raster tile={tile} n={n} {params}")
    st = Stage(n, cams, m.RasterParams(tile_w=tw, tile_h=th, bg=bg, **params), cat, 400_000)
    rgb, tf, nl = st.rasterize()
    orp = R.RasterParams(tile_w=tw, tile_h=th, bg=bg, **params)
    _, ents, granges = st.lists()
    rng = np.random.default_rng(5)
    dls, flips_total = [], 0
    for v, (rec, cam, img, T, NL) in enumerate(zip(recs, cams, split_views(rgb, cams, 3),
                                                   split_views(tf, cams), split_views(nl, cams))):
        out, _ = _oracle_composite(rec, cam, orp, n, v)
        ref_img = out["rgb"].detach().numpy()
        # the GPU's last blended Gaussian: entry at position n_last - 1 of the
        # pixel's tile list
        px, py = R.pixel_grid(cam.width, cam.height)
        tiles_x = (cam.width + tw - 1) // tw
        toff = sum(((c.width + tw - 1) // tw) * ((c.height + th - 1) // th) for c in cams[:v])
        t = toff + (py.numpy() // th) * tiles_x + px.numpy() // tw
        nlv = NL.astype(np.int64)
        g_last = np.full(len(nlv), -1, np.int64)
        has = nlv > 0
        g_last[has] = ents[granges[t[has], 0].astype(np.int64) + nlv[has] - 1].astype(np.int64)
        flips = g_last != out["last"].numpy()
        flips_total += int(flips.sum())
        ok = ~flips
        assert flips.mean() < 1e-3
        assert rel_max_err(img.reshape(3, -1)[:, ok], ref_img[:, ok]) < 1e-5
        assert rel_max_err(T[ok], out["T_final"].detach().numpy()[ok]) < 1e-5
        dl = rng.normal(0, 1, (3, cam.width * cam.height))
        dl[:, flips] = 0.0
        dls.append(dl)
    say(f"  decision flips: {flips_total}")
    # backward on the same records, cotangents zero on flipped pixels
    dl_all = np.concatenate([d.reshape(-1) for d in dls]).astype(np.float32)
    acc = st.backward(dl_all)
    for v, (rec, cam) in enumerate(zip(recs, cams)):
        out, t = _oracle_composite(rec, cam, orp, n, v, leaf=True)
        (out["rgb"] * torch.tensor(dls[v].astype(np.float32).astype(np.float64))).sum().backward()
        a = acc[v * n:(v + 1) * n]
        pairs = [("u", a[:, 0], t["u"].grad), ("v", a[:, 1], t["v"].grad),
                 ("conic", a[:, 2:5], t["conic"].grad), ("opacity", a[:, 5], t["opacity"].grad),
                 ("rgb", np.stack([a[:, 6], a[:, 7], a[:, 8]], 1), t["rgb"].grad)]
        for name, got, ref in pairs:
            ref = ref.numpy()
            assert rel_norm_err(got, ref) < 1e-3, (v, name, rel_norm_err(got, ref))
            assert rel_max_err(got, ref) < 1e-3, (v, name, rel_max_err(got, ref))


def test_raster_backward_gate_closed_touches_nothing():
    require_gpu()
    m = sg()
    cams = _views()[:1]
    n = 200
    recs, cat = _records(n, cams, 11, max_radius=10)
    st = Stage(n, cams, m.RasterParams(), cat, 100_000)
    st.rasterize()
    acc_region = st.ws[st.L.accum:st.L.accum + 48 * n]
    acc_region.fill_(7)
    gate = torch.zeros(1, dtype=torch.int32, device="cuda")
    m.rasterize_backward(cams, n, st.rp, st.ws, st.cap,
                         torch.ones(3 * cams[0].width * cams[0].height, device="cuda"), gate)
    torch.cuda.synchronize()
    assert bool((acc_region == 7).all())
