"""Stage parity on identical float32 records: super-tile binning and sort and
the tile lists split from it (bit exact without the reach test; with it, an
ordered subsequence keeping every contributing entry), compositing forward
(1e-5) and backward (1e-3) against the oracle, with only pixels the oracle
itself calls decision-sensitive left out."""
import numpy as np
import pytest
import torch

from oracle import render as R
from paper_2603_08997_amd import scenes as S
from tests.gpu_util import (last_blended, tile_lists, region, rel_max_err, rel_norm_err,
                            require_gpu, say, sg, split_views, to_dev)
from tests.sensitivity import decision_sensitive

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
        cnt = m.read_counters(self.ws)
        self.kept, self.needed, self.items = cnt["pairs_kept"], cnt["pairs"], cnt["items"]

    def lists(self):
        """The sorted super-tile lists: super-tile index, tile rectangle
        inside the super-tile (x0, x1, y0, y1, last inclusive) and entry per
        pair, and the ranges."""
        P = self.kept
        raw = region(self.ws, self.L.sup_key, P, np.uint32).astype(np.int64)
        kb, rb = self.L.key_bits, self.L.rect_bits
        keys = raw & ((1 << kb) - 1)
        r = raw >> kb
        rect = np.stack([(r >> (k * rb)) & ((1 << rb) - 1) for k in range(4)], 1)
        self.rect = rect
        ents = region(self.ws, self.L.sup_entry, P, np.uint32)
        ranges = region(self.ws, self.L.sup_ranges, 2 * self.L.total_supers,
                        np.uint32).reshape(-1, 2)
        return keys, ents, ranges

    def rasterize(self):
        px = sum(c.width * c.height for c in self.cams)
        self.rgb = torch.zeros(3 * px, dtype=torch.float32, device="cuda")
        self.m.rasterize(self.cams, self.n, self.rp, self.ws, self.cap, self.rgb)
        torch.cuda.synchronize()
        self.flags = self.m.read_status(self.ws)[0]
        tf = region(self.ws, self.L.t_final, self.L.total_pixels, np.float32)
        nl = region(self.ws, self.L.n_last, self.L.total_pixels, np.uint32)
        return self.rgb.cpu().numpy(), tf, nl

    def backward(self, dl):
        self.m.rasterize_backward(self.cams, self.n, self.rp, self.ws, self.cap, to_dev(dl))
        torch.cuda.synchronize()
        return region(self.ws, self.L.accum, 12 * self.L.entries, np.float32).reshape(-1, 12)


def _tiles_of(cam, tw, th):
    return ((cam.width + tw - 1) // tw) * ((cam.height + th - 1) // th)


def _supers_of(cam, tw, th, S_):
    return (((cam.width + tw - 1) // tw + S_ - 1) // S_) * (((cam.height + th - 1) // th + S_ - 1) // S_)


def _oracle_super_lists(recs, cams, n, tw, th, S_):
    sups, vals, ranges = [], [], []
    off = 0
    for v, (r, c) in enumerate(zip(recs, cams)):
        k, val, rg = R.super_tile_lists(r["u"], r["v"], r["depth"], r["extent"],
                                        v * n + np.arange(n), c.width, c.height, tw, th, S_,
                                        super_offset=off)
        base = sum(len(x) for x in sups)
        rg = np.where(rg[:, 1:2] > rg[:, 0:1], rg + base, 0)
        sups.append(k); vals.append(val); ranges.append(rg)
        off += _supers_of(c, tw, th, S_)
    return np.concatenate(sups), np.concatenate(vals), np.concatenate(ranges)


def _oracle_rects(recs, cams, n, tw, th, S_, sups, vals):
    """Per pair: the entry's tile rectangle (oracle) inside the pair's
    super-tile, relative to its first tile, last column and row inclusive."""
    out = np.zeros((len(vals), 4), np.int64)
    soff = 0
    for v, (r, c) in enumerate(zip(recs, cams)):
        tx_n, ty_n = (c.width + tw - 1) // tw, (c.height + th - 1) // th
        sx_n = (tx_n + S_ - 1) // S_
        x0, x1, y0, y1 = (a.numpy() for a in R.tile_rect(r["u"].astype(np.float64),
                                                           r["v"].astype(np.float64), r["extent"],
                                                           tw, th, tx_n, ty_n))
        nsup = _supers_of(c, tw, th, S_)
        sel = np.nonzero((sups >= soff) & (sups < soff + nsup))[0]
        for k in sel:
            i = vals[k] - v * n
            s = sups[k] - soff
            ox, oy = (s % sx_n) * S_, (s // sx_n) * S_
            out[k] = (max(x0[i], ox) - ox, min(x1[i], ox + S_) - 1 - ox,
                      max(y0[i], oy) - oy, min(y1[i], oy + S_) - 1 - oy)
        soff += nsup
    return out


def _oracle_tile_lists(recs, cams, n, tw, th):
    """tile (global index) -> oracle tile list (entry indices)."""
    out, off = {}, 0
    for v, (r, c) in enumerate(zip(recs, cams)):
        _, val, rg = R.bin_and_sort(r["u"], r["v"], r["depth"], r["extent"],
                                    v * n + np.arange(n), c.width, c.height, tw, th)
        for t in range(len(rg)):
            out[off + t] = val[rg[t, 0]:rg[t, 1]]
        off += _tiles_of(c, tw, th)
    return out


@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("ties", [0.0, 0.4])
def test_binning_matches_oracle(tile, ties):
    require_gpu()
    st = _check_binning(_views(), tile, ties, 1500, 100 + int(ties * 10))
    assert st.L.rect_bits == 3   # super-tiles of 8 tiles


@pytest.mark.parametrize("tile,S_", [((16, 16), 8), ((8, 8), 3), ((32, 8), 1), ((16, 16), 2)])
def test_binning_bit_exact_without_reach_test(tile, S_):
    """alpha_min = 0 (no reach test): super-tile keys, entry order (float32
    depth, then index) and ranges equal the oracle's super-tile lists bit for
    bit, for several super-tile sizes (1: the tile lists themselves)."""
    require_gpu()
    _check_binning(_views(), tile, 0.3, 1200, 77, super_tile=S_, alpha_min=0.0)


def test_binning_bit_exact_wide_keys():
    """79,800 tiles of 8x8 in super-tiles of one tile (three 1600x1060 views):
    17-bit super-tile indices, no rectangle bits."""
    require_gpu()
    cams = [S.look_at_camera(p, 1600, 1060) for p in ((3.0, 1.0, 1.0), (0.5, -3.0, 2.0),
                                                        (-2.0, 2.0, 1.5))]
    st = _check_binning(cams, (8, 8), 0.2, 1500, 131, super_tile=1, alpha_min=0.0)
    assert st.L.key_bits == 17 and st.L.rect_bits == 0


def _check_binning(cams, tile, ties, n, seed, super_tile=8, alpha_min=None):
    m = sg()
    tw, th = tile
    recs, cat = _records(n, cams, seed, max_radius=20, tie_fraction=ties)
    extra = {} if alpha_min is None else {"alpha_min": alpha_min}
    say(f"binning tile={tile} S={super_tile} ties={ties} n={n} views={len(cams)} {extra}")
    # whole lists (no split prefix): the lists sgs_bin leaves are complete
    rp = m.RasterParams(tile_w=tw, tile_h=th, super_tile=super_tile, split_prefix=0, **extra)
    st = Stage(n, cams, rp, cat, 400_000)
    assert st.flags == 0
    sups, vals, ranges = _oracle_super_lists(recs, cams, n, tw, th, super_tile)
    keys, ents, granges = st.lists()
    # the pair count the capacity must cover is that of the box lists
    assert st.needed == len(vals)
    assert st.kept <= st.needed and len(ents) == st.kept
    assert np.array_equal(keys.astype(np.int64),
                          np.repeat(np.arange(len(granges)), granges[:, 1] - granges[:, 0]))
    if alpha_min == 0.0:
        # no reach test: bit-exact lists, and every key's rectangle is the
        # entry's tile rectangle clipped to the super-tile
        assert np.array_equal(keys.astype(np.int64), sups)
        assert np.array_equal(ents.astype(np.int64), vals)
        assert np.array_equal(granges.astype(np.int64), ranges)
        assert np.array_equal(st.rect, _oracle_rects(recs, cams, n, tw, th, super_tile, sups, vals))
        _check_tile_lists(st, recs, cams, n, tw, th, 0.0)
        return st
    # the GPU lists are the box lists less entries that cannot reach
    # alpha_min on the super-tile: per super-tile, an ordered subsequence of
    # the oracle's list that keeps every entry able to contribute to a pixel
    orp = R.RasterParams(tile_w=tw, tile_h=th, alpha_min=rp.alpha_min)
    soff, dropped, dead = 0, 0, 0
    for v, (rec, cam) in enumerate(zip(recs, cams)):
        sx_n = ((cam.width + tw - 1) // tw + super_tile - 1) // super_tile
        for sidx in range(soff, soff + _supers_of(cam, tw, th, super_tile)):
            lo, hi = ranges[sidx]
            olist = vals[lo:hi]
            glist = ents[granges[sidx][0]:granges[sidx][1]].astype(np.int64)
            keep = np.isin(olist, glist)
            assert np.array_equal(olist[keep], glist)          # ordered subsequence
            sx, sy = (sidx - soff) % sx_n, (sidx - soff) // sx_n
            x0, y0 = sx * super_tile * tw, sy * super_tile * th
            for e, kept in zip(olist, keep):
                i = e - v * n
                live = R.rect_contributes(rec["u"][i], rec["v"][i], *rec["conic"][i],
                                          rec["opacity"][i], *rec["extent"][i], x0,
                                          min(x0 + super_tile * tw, cam.width), y0,
                                          min(y0 + super_tile * th, cam.height), orp)
                assert kept or not live, (sidx, e)
                dead += int(not live)
                dropped += int(not kept)
        soff += _supers_of(cam, tw, th, super_tile)
    say(f"  super-tile pairs {len(vals)}, kept {len(ents)}, non-contributing {dead}, "
        f"dropped {dropped}")
    assert dropped >= 0.3 * dead
    _check_tile_lists(st, recs, cams, n, tw, th, rp.alpha_min)
    return st


def _check_tile_lists(st, recs, cams, n, tw, th, alpha_min):
    """The tile lists split from the super-tile lists: without the reach test
    the oracle's tile lists bit for bit; with it, per tile, an ordered
    subsequence of the oracle's list keeping every entry that can contribute
    to a pixel of the tile."""
    lists = tile_lists(st.ws, st.L)
    olists = _oracle_tile_lists(recs, cams, n, tw, th)
    orp = R.RasterParams(tile_w=tw, tile_h=th, alpha_min=alpha_min)
    assert st.items == sum(len(x) for x in lists.values())
    toff, dropped, dead = 0, 0, 0
    empty = np.zeros(0, np.int64)
    for v, (rec, cam) in enumerate(zip(recs, cams)):
        tx_n = (cam.width + tw - 1) // tw
        for t in range(toff, toff + _tiles_of(cam, tw, th)):
            ol, gl = olists[t], lists.get(t, empty)
            if alpha_min == 0.0:
                assert np.array_equal(gl, ol), t
                continue
            keep = np.isin(ol, gl)
            assert np.array_equal(ol[keep], gl), t
            tx, ty = (t - toff) % tx_n, (t - toff) // tx_n
            for e, kept in zip(ol, keep):
                i = e - v * n
                live = R.tile_contributes(rec["u"][i], rec["v"][i], *rec["conic"][i],
                                          rec["opacity"][i], *rec["extent"][i], tx, ty, tw, th,
                                          cam.width, cam.height, orp)
                assert kept or not live, (t, e)
                dead += int(not live)
                dropped += int(not kept)
        toff += _tiles_of(cam, tw, th)
    say(f"  tile-list entries {st.items}, non-contributing {dead}, dropped {dropped}")
    if alpha_min > 0.0:
        assert dropped >= 0.3 * dead
    return lists


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
    rgb, tf, nl = st.rasterize()
    assert st.flags == 0 and not nl.any() and np.all(tf == 1.0) and not rgb.any()
    recs, cat = _records(n, cams, 8, max_radius=15)
    st = Stage(n, cams, m.RasterParams(super_tile=1), cat, 64)   # far too small
    assert st.flags & m.STATUS_PAIR_OVERFLOW
    assert st.pairs > 64


def test_tile_list_overflow():
    """Capacity for the super-tile pairs but not for the tile lists (super-
    tiles of 8x8 small tiles hold few pairs while the tile lists are long):
    binning flags the overflow and reports the capacity the lists need; with
    that capacity the image equals the one rendered with ample storage."""
    require_gpu()
    m = sg()
    cams = [S.look_at_camera((3.0, 1.0, 1.0), 255, 255)]
    n = 20000
    recs, cat = _records(n, cams, 21, max_radius=24)
    rp = m.RasterParams(tile_w=8, tile_h=8, super_tile=8, lds_batch=32, split_prefix=0)
    probe = Stage(n, cams, rp, cat, 400_000)
    rgb_ref, _, _ = probe.rasterize()
    assert probe.flags == 0
    assert probe.needed < probe.items, (probe.needed, probe.items)
    st = Stage(n, cams, rp, cat, probe.needed)
    assert st.flags & m.STATUS_PAIR_OVERFLOW
    assert st.pairs == probe.items
    assert not tile_lists(st.ws, st.L)          # no partial lists
    st = Stage(n, cams, rp, cat, st.pairs)
    rgb, _, _ = st.rasterize()
    assert st.flags == 0
    assert np.array_equal(rgb, rgb_ref)


def _tile_need(nl, cams, tw, th):
    """Per tile (global index): the largest list position any of its pixels
    blends up to (n_last)."""
    need, off, poff = {}, 0, 0
    for cam in cams:
        tx_n = (cam.width + tw - 1) // tw
        ys, xs = np.divmod(np.arange(cam.width * cam.height), cam.width)
        t = off + (ys // th) * tx_n + xs // tw
        m = np.zeros(_tiles_of(cam, tw, th), np.int64)
        np.maximum.at(m, t - off, nl[poff:poff + cam.width * cam.height].astype(np.int64))
        need.update({off + k: int(x) for k, x in enumerate(m)})
        off += _tiles_of(cam, tw, th)
        poff += cam.width * cam.height
    return need


PREFIX = 2048


def _prefix_scene():
    # dense overlapping records in super-tiles of 8x8 small tiles: the
    # super-tile lists run to thousands of pairs; in the small second view
    # they are long enough to be cut by the prefix, and there some tiles
    # terminate within it while others need their whole lists
    cams = [S.look_at_camera((3.0, 1.0, 1.0), 255, 255), S.look_at_camera((0.5, -3.0, 2.0), 120, 90)]
    n = 40000
    recs, cat = _records(n, cams, 41, max_radius=24)
    return cams, n, recs, cat


def test_split_prefix_matches_whole_lists():
    """Tile lists split from 2048-pair prefixes of the long super-tile lists
    and completed on the device for the tiles that need more: image, T_final and
    last positions bit-identical to those of whole lists, the same work
    counters, every list after compositing a prefix of the whole list that
    covers the tile's blended entries (some strictly shorter), gradients equal
    up to the order of the float atomic additions."""
    require_gpu()
    m = sg()
    cams, n, recs, cat = _prefix_scene()
    base = dict(tile_w=8, tile_h=8, super_tile=8, lds_batch=32)
    say(f"split prefix: n={n} views={len(cams)} {base}")
    whole = Stage(n, cams, m.RasterParams(split_prefix=0, **base), cat, 3_000_000)
    w_rgb, w_tf, w_nl = whole.rasterize()
    pre = Stage(n, cams, m.RasterParams(split_prefix=PREFIX, **base), cat, 3_000_000)
    p_rgb, p_tf, p_nl = pre.rasterize()
    assert whole.flags == 0 and pre.flags == 0
    cw, cp = m.read_counters(whole.ws), m.read_counters(pre.ws)
    say(f"  whole: items {cw['items']}; prefix: items {cp['items']} + rest {cp['items_rest']}, "
        f"redo {cp['redo']}")
    assert cw["redo"] == 0 and cw["items_rest"] == 0
    assert cp["redo"] == 1 and cp["items"] < cw["items"]
    assert np.array_equal(p_rgb, w_rgb)
    assert np.array_equal(p_tf, w_tf)
    assert np.array_equal(p_nl, w_nl)
    for k in ("blended", "evaluated", "used"):
        assert cp[k] == cw[k], k
    lw, lp = tile_lists(whole.ws, whole.L), tile_lists(pre.ws, pre.L)
    need = _tile_need(w_nl, cams, 8, 8)
    empty = np.zeros(0, np.int64)
    cut = 0
    for t, wl in lw.items():
        pl = lp.get(t, empty)
        assert np.array_equal(pl, wl[:len(pl)]), t
        assert len(pl) >= need[t], t
        cut += int(len(pl) < len(wl))
    assert not set(lp) - set(lw)
    say(f"  tiles with a strict prefix list: {cut} of {len(lw)}")
    assert cut > 0
    rng = np.random.default_rng(3)
    dl = rng.normal(0, 1, len(w_rgb)).astype(np.float32)
    gw, gp = whole.backward(dl), pre.backward(dl)
    assert rel_max_err(gp, gw) < 1e-5, rel_max_err(gp, gw)


def test_split_rest_overflow():
    """Capacity for the prefix lists but not for the completing split: the
    compositing call flags the overflow and reports the capacity both splits
    need; with that capacity the image equals the whole-list image."""
    require_gpu()
    m = sg()
    cams, n, recs, cat = _prefix_scene()
    base = dict(tile_w=8, tile_h=8, super_tile=8, lds_batch=32)
    ref = Stage(n, cams, m.RasterParams(split_prefix=0, **base), cat, 3_000_000)
    rgb_ref, _, _ = ref.rasterize()
    rp = m.RasterParams(split_prefix=PREFIX, **base)
    probe = Stage(n, cams, rp, cat, 3_000_000)
    probe.rasterize()
    c = m.read_counters(probe.ws)
    total = c["items"] + c["items_rest"]
    cap = max(c["pairs"], c["items"])
    say(f"  pairs {c['pairs']} prefix items {c['items']} rest {c['items_rest']} cap {cap}")
    assert c["items_rest"] > 0 and cap < total
    st = Stage(n, cams, rp, cat, cap)
    assert st.flags == 0                       # the prefix lists fit
    st.rasterize()
    assert st.flags & m.STATUS_PAIR_OVERFLOW
    assert m.read_status(st.ws)[2] == total
    st = Stage(n, cams, rp, cat, total)
    rgb, _, _ = st.rasterize()
    assert st.flags == 0
    assert np.array_equal(rgb, rgb_ref)


def _oracle_composite(rec, cam, rp, n, view, leaf=False):
    t = {k: torch.tensor(np.asarray(rec[k], np.float64), requires_grad=leaf)
         for k in ("u", "v", "conic", "opacity", "rgb")}
    uv = torch.stack([t["u"], t["v"]], 1)
    out = R.composite(uv, t["conic"], t["opacity"], t["rgb"], torch.tensor(rec["depth"], dtype=torch.float64),
                      torch.tensor(rec["extent"].astype(np.int64)), view * n + torch.arange(n),
                      cam.width, cam.height, rp)
    return out, t


@pytest.mark.parametrize("tile,S_,B", [((16, 16), 8, 64), ((8, 8), 4, 32), ((32, 8), 2, 128),
                                       ((16, 16), 1, 256)])
def test_raster_forward_and_backward_match_oracle(tile, S_, B):
    require_gpu()
    _check_raster(tile, super_tile=S_, lds_batch=B)


def test_raster_nondefault_params_match_oracle():
    """alpha_min = 0 (no skip threshold: log2 alpha_min = -inf, no reach
    test), alpha_max = 0.9 and t_min = 1e-3."""
    require_gpu()
    _check_raster((16, 16), alpha_min=0.0, alpha_max=0.9, t_min=1e-3)


DECISION_REL = 3e-5


def _check_raster(tile, super_tile=8, lds_batch=64, **params):
    m = sg()
    tw, th = tile
    cams = _views()
    n = 900
    recs, cat = _records(n, cams, 300, max_radius=14)
    bg = (0.2, 0.4, 0.6)
    say(f"raster tile={tile} S={super_tile} B={lds_batch} n={n} {params}")
    st = Stage(n, cams, m.RasterParams(tile_w=tw, tile_h=th, bg=bg, super_tile=super_tile,
                                       lds_batch=lds_batch, **params), cat, 400_000)
    rgb, tf, nl = st.rasterize()
    assert st.flags == 0
    orp = R.RasterParams(tile_w=tw, tile_h=th, bg=bg, **params)
    lists = _check_tile_lists(st, recs, cams, n, tw, th, orp.alpha_min)
    rng = np.random.default_rng(5)
    dls, excl_total = [], 0
    toff = 0
    for v, (rec, cam, img, T, NL) in enumerate(zip(recs, cams, split_views(rgb, cams, 3),
                                                   split_views(tf, cams), split_views(nl, cams))):
        comp = lambda rp_: _oracle_composite(rec, cam, rp_, n, v)[0]
        out, sens = decision_sensitive(comp, orp, DECISION_REL, 1e-5)
        ref_img = out["rgb"].detach().numpy()
        px, py = R.pixel_grid(cam.width, cam.height)
        t = toff + (py.numpy() // th) * ((cam.width + tw - 1) // tw) + px.numpy() // tw
        g_last = last_blended(lists, NL.astype(np.int64), t)
        ok_last = ~sens["last"]
        # no unexplained mismatch: the last blended Gaussian agrees on every
        # pixel the oracle does not call decision-sensitive
        assert np.array_equal(g_last[ok_last], out["last"].numpy()[ok_last]), v
        ok = ~sens["colour"]
        assert rel_max_err(img.reshape(3, -1)[:, ok], ref_img[:, ok]) < 1e-5
        assert rel_max_err(T[ok], out["T_final"].detach().numpy()[ok]) < 1e-5
        excl_total += int(sens["last"].sum())
        assert sens["last"].mean() < 1e-2
        dl = rng.normal(0, 1, (3, cam.width * cam.height))
        dl[:, sens["last"]] = 0.0
        dls.append(dl)
        toff += _tiles_of(cam, tw, th)
    say(f"  decision-sensitive pixels (oracle): {excl_total}")
    # backward on the same records, cotangents zero on sensitive pixels
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
