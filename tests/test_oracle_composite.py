"""Pins for the oracle's compositing (Eqs. 4-5) and tile binning: brute-force
unsorted compositing, closed forms and invariants."""
import math

import numpy as np
import pytest
import torch

from oracle import render as R
from paper_2603_08997_amd import scenes as S

DT = torch.float64


def _records(seed, n, w, h, **kw):
    rec = S.random_records(seed, n, w, h, **kw)
    t = lambda x: torch.tensor(np.asarray(x, np.float64))
    return dict(uv=t(np.stack([rec["u"], rec["v"]], 1)), conic=t(rec["conic"]),
                opacity=t(rec["opacity"]), rgb=t(rec["rgb"]), depth=t(rec["depth"]),
                extent=torch.tensor(rec["extent"].astype(np.int64)), ids=torch.arange(n)), rec


def _brute_force_pixel(x, y, rec, rp):
    """Eq. 4 at one pixel with no sort: T_i is the product over the active
    Gaussians that precede i in (depth, index), computed pairwise."""
    rp = rp.as_f32()
    n = len(rec["u"])
    px, py = x + 0.5, y + 0.5
    alpha = {}
    for i in range(n):
        u, v = float(rec["u"][i]), float(rec["v"][i])
        rx, ry = (int(x) for x in rec["extent"][i])
        if abs(px - u) > rx or abs(py - v) > ry:
            continue
        a, b, c = (float(z) for z in rec["conic"][i])
        dx, dy = px - u, py - v
        pw = -0.5 * (a * dx * dx + c * dy * dy) - b * dx * dy
        if pw > 0:
            continue
        al = min(rp.alpha_max, float(rec["opacity"][i]) * math.exp(pw))
        if al < rp.alpha_min:
            continue
        alpha[i] = al
    key = lambda i: (float(rec["depth"][i]), i)
    col = np.zeros(3)
    T_final = 1.0
    nb = 0
    for i, ai in alpha.items():
        Ti = 1.0
        for j, aj in alpha.items():
            if key(j) < key(i):
                Ti *= (1.0 - aj)
        if Ti * (1.0 - ai) >= rp.t_min:
            col += np.asarray(rec["rgb"][i], np.float64) * ai * Ti
            T_final *= (1.0 - ai)
            nb += 1
    col += np.asarray(rp.bg) * T_final
    return col, T_final, nb


@pytest.mark.parametrize("rp", [R.RasterParams(bg=(0.1, 0.2, 0.3)), R.smooth_params(bg=(0.0, 0.5, 1.0)),
                                R.RasterParams(t_min=0.3)])
@pytest.mark.parametrize("ties", [0.0, 0.3])
def test_sorted_compositing_equals_brute_force(rp, ties):
    w, h = 20, 14
    t, rec = _records(21, 60, w, h, max_radius=9, tie_fraction=ties)
    out = R.composite(t["uv"], t["conic"], t["opacity"], t["rgb"], t["depth"], t["extent"], t["ids"],
                      w, h, rp)
    img = out["rgb"].numpy().reshape(3, h, w)
    T = out["T_final"].numpy().reshape(h, w)
    nb = out["n_blended"].numpy().reshape(h, w)
    for y in range(h):
        for x in range(w):
            col, Tf, n = _brute_force_pixel(x, y, rec, rp)
            assert np.allclose(img[:, y, x], col, rtol=0, atol=1e-13)
            assert abs(T[y, x] - Tf) < 1e-13
            assert nb[y, x] == n


def test_weights_and_final_transmittance_sum_to_one():
    """With white colours and black background C(p) = sum_i alpha'_i T_i, and the
    telescoping product gives sum_i alpha'_i T_i + T_final = 1."""
    w, h = 32, 24
    t, _ = _records(4, 300, w, h, max_radius=12)
    t["rgb"] = torch.ones_like(t["rgb"])
    for rp in (R.RasterParams(), R.smooth_params()):
        out = R.composite(t["uv"], t["conic"], t["opacity"], t["rgb"], t["depth"], t["extent"],
                          t["ids"], w, h, rp)
        wsum = out["rgb"][0].numpy()
        assert np.all(wsum <= 1 + 1e-12)
        assert np.abs(wsum + out["T_final"].numpy() - 1.0).max() < 1e-12


def test_final_transmittance_is_product_over_blended():
    w, h = 16, 16
    t, rec = _records(5, 40, w, h, max_radius=10)
    rp = R.RasterParams()
    out = R.composite(t["uv"], t["conic"], t["opacity"], t["rgb"], t["depth"], t["extent"], t["ids"],
                      w, h, rp)
    assert (out["T_final"] >= R.f32(rp.t_min)).all()
    assert (out["T_final"] <= 1.0).all()


def test_two_gaussians_at_their_centre_closed_form():
    """Both centred on pixel (5, 5): alpha' = opacity there, so
    C = c1 o1 + c2 o2 (1 - o1) + bg (1 - o1)(1 - o2) with 1 the nearer one."""
    uv = torch.tensor([[5.5, 5.5], [5.5, 5.5]], dtype=DT)
    conic = torch.tensor([[0.5, 0.1, 0.4], [0.3, 0.0, 0.3]], dtype=DT)
    o = torch.tensor([0.6, 0.7], dtype=DT)
    rgb = torch.tensor([[1.0, 0.0, 0.2], [0.0, 1.0, 0.4]], dtype=DT)
    bg = (0.25, 0.5, 0.75)
    rp = R.RasterParams(bg=bg)
    for depth, near in (([1.0, 2.0], 0), ([3.0, 2.0], 1)):
        out = R.composite(uv, conic, o, rgb, torch.tensor(depth, dtype=DT),
                          torch.tensor([[4, 4], [4, 4]]), torch.arange(2), 11, 11, rp, px=[5], py=[5])
        far = 1 - near
        o1, o2 = [0.6, 0.7][near], [0.6, 0.7][far]
        c1, c2 = rgb[near].numpy(), rgb[far].numpy()
        expect = c1 * o1 + c2 * o2 * (1 - o1) + np.asarray(R.RasterParams(bg=bg).as_f32().bg) * (1 - o1) * (1 - o2)
        assert np.allclose(out["rgb"][:, 0].numpy(), expect, atol=1e-15)
        assert out["T_final"].item() == pytest.approx((1 - o1) * (1 - o2), abs=1e-15)


def test_equal_depth_ties_break_by_index():
    uv = torch.tensor([[3.5, 3.5], [3.5, 3.5]], dtype=DT)
    conic = torch.tensor([[0.5, 0.0, 0.5]] * 2, dtype=DT)
    o = torch.tensor([0.5, 0.5], dtype=DT)
    rgb = torch.tensor([[1.0, 0, 0], [0, 1.0, 0]], dtype=DT)
    out = R.composite(uv, conic, o, rgb, torch.tensor([2.0, 2.0], dtype=DT),
                      torch.tensor([[3, 3], [3, 3]]), torch.tensor([7, 3]), 8, 8, R.RasterParams(),
                      px=[3], py=[3])
    # index 3 (green) is in front of index 7 (red)
    assert np.allclose(out["rgb"][:, 0].numpy(), [0.25, 0.5, 0.0], atol=1e-15)
    assert out["last"].item() == 7


def test_depths_equal_in_float32_tie_and_break_by_index():
    """The depth key is the float32 camera depth: Gaussian 3 lies 5e-9 behind
    Gaussian 7 in binary64, but both depths round to the same float32 value,
    so they tie and the lower index (3, green) is composited first."""
    assert np.float32(2.0 + 5e-9) == np.float32(2.0) and 2.0 + 5e-9 > 2.0
    uv = torch.tensor([[3.5, 3.5], [3.5, 3.5]], dtype=DT)
    conic = torch.tensor([[0.5, 0.0, 0.5]] * 2, dtype=DT)
    o = torch.tensor([0.5, 0.5], dtype=DT)
    rgb = torch.tensor([[1.0, 0, 0], [0, 1.0, 0]], dtype=DT)
    depth = torch.tensor([2.0, 2.0 + 5e-9], dtype=DT)
    out = R.composite(uv, conic, o, rgb, depth, torch.tensor([[3, 3], [3, 3]]),
                      torch.tensor([7, 3]), 8, 8, R.RasterParams(), px=[3], py=[3])
    assert np.allclose(out["rgb"][:, 0].numpy(), [0.25, 0.5, 0.0], atol=1e-15)
    assert out["last"].item() == 7
    # one float32 step apart, the nearer one is in front whatever the index
    depth = torch.tensor([float(np.nextafter(np.float32(2.0), np.float32(3.0))), 2.0], dtype=DT)
    out = R.composite(uv, conic, o, rgb, depth, torch.tensor([[3, 3], [3, 3]]),
                      torch.tensor([3, 7]), 8, 8, R.RasterParams(), px=[3], py=[3])
    assert np.allclose(out["rgb"][:, 0].numpy(), [0.25, 0.5, 0.0], atol=1e-15)
    assert out["last"].item() == 3


def test_single_isotropic_splat_closed_form():
    """One isotropic Gaussian on the optical axis at depth d: its screen
    covariance is ((f s / d)^2 + h) I, so alpha'(p) = o exp(-|p - c|^2 / (2 sigma^2))
    and C(p) = rgb alpha' + bg (1 - alpha') wherever the pixel is within the
    cut-off square and no threshold applies."""
    cam = S.look_at_camera((0.0, -3.0, 0.5), 48, 40)
    Rc = cam.R.astype(np.float64)
    tcam = cam.t.astype(np.float64)
    C = -Rc.T @ tcam
    mean = C + 2.5 * Rc[2]
    d = (Rc @ mean + tcam)[2]
    s, o_logit, dc = 0.02, 0.4, 0.8
    rp = R.smooth_params(bg=(0.1, 0.2, 0.3), jac_clamp=0.0)
    out = R.render(np.array([mean]), np.log([[s, s, s]]), np.array([[1.0, 0, 0, 0]]), np.array([o_logit]),
                   np.full((1, 1, 3), dc), 0, cam, rp)
    sig2 = (cam.fx * s / d) ** 2 + R.f32(rp.dilation)
    o = 1 / (1 + math.exp(-o_logit))
    rgb = dc / (2 * math.sqrt(math.pi)) + 0.5
    r = math.ceil(3 * math.sqrt(sig2))
    u0 = cam.fx * (Rc[0] @ mean + tcam[0]) / d + cam.cx
    v0 = cam.fy * (Rc[1] @ mean + tcam[1]) / d + cam.cy
    img = out["rgb"].detach().numpy().reshape(3, cam.height, cam.width)
    bg = np.asarray(rp.as_f32().bg)
    for y in range(cam.height):
        for x in range(cam.width):
            dx, dy = x + 0.5 - u0, y + 0.5 - v0
            if abs(dx) <= r and abs(dy) <= r:
                a = o * math.exp(-(dx * dx + dy * dy) / (2 * sig2))
                expect = rgb * a + bg * (1 - a)
            else:
                expect = bg
            assert np.allclose(img[:, y, x], expect, rtol=1e-7, atol=1e-12)


def test_bins_cover_exactly_the_rect_and_sort_by_depth_then_index():
    w, h, tw, th = 53, 37, 16, 8
    rec = S.random_records(9, 80, w, h, max_radius=15, tie_fraction=0.25)
    keys, vals, ranges = R.bin_and_sort(rec["u"], rec["v"], rec["depth"], rec["extent"], np.arange(80),
                                        w, h, tw, th, tile_offset=0)
    tx_n, ty_n = (w + tw - 1) // tw, (h + th - 1) // th
    dbits = R.float32_bits(rec["depth"])
    # tile membership: the tile's half-open box intersects the closed square
    for t in range(tx_n * ty_n):
        tx, ty = t % tx_n, t // tx_n
        expect = []
        for i in range(80):
            u, v = float(rec["u"][i]), float(rec["v"][i])
            rx, ry = (int(x) for x in rec["extent"][i])
            if (u + rx >= tx * tw and u - rx < (tx + 1) * tw and v + ry >= ty * th and v - ry < (ty + 1) * th):
                expect.append(i)
        s, e = ranges[t]
        got = list(vals[s:e])
        assert sorted(got) == expect
        # order: ascending depth, ties by index
        assert got == sorted(expect, key=lambda i: (int(dbits[i]), i))
        assert all((int(k) >> 32) == t for k in keys[s:e])
    assert np.all(np.diff(keys.astype(np.float64)) >= 0)


@pytest.mark.parametrize("S_", [1, 2, 3, 8])
def test_super_tile_list_is_the_depth_ordered_union_of_its_tile_lists(S_):
    """Each super-tile list holds, once each and in (float32 depth, index)
    order, exactly the Gaussians of the lists of its tiles; every tile list
    is the subsequence of its super-tile's list whose rectangles contain the
    tile; with super-tiles of one tile the lists are the tile lists."""
    w, h, tw, th = 75, 41, 8, 8
    rec = S.random_records(17, 120, w, h, max_radius=12, tie_fraction=0.3)
    ids = np.arange(120)
    _, tvals, tranges = R.bin_and_sort(rec["u"], rec["v"], rec["depth"], rec["extent"], ids, w, h,
                                       tw, th)
    sups, svals, sranges = R.super_tile_lists(rec["u"], rec["v"], rec["depth"], rec["extent"],
                                              ids, w, h, tw, th, S_)
    tx_n, ty_n = (w + tw - 1) // tw, (h + th - 1) // th
    sx_n = (tx_n + S_ - 1) // S_
    dbits = R.float32_bits(rec["depth"])
    key = lambda i: (int(dbits[i]), int(i))
    x0, x1, y0, y1 = (a.numpy() for a in R.tile_rect(rec["u"].astype(np.float64),
                                                       rec["v"].astype(np.float64), rec["extent"],
                                                       tw, th, tx_n, ty_n))
    for sidx in range(len(sranges)):
        sx, sy = sidx % sx_n, sidx // sx_n
        members = set()
        for ty in range(sy * S_, min((sy + 1) * S_, ty_n)):
            for tx in range(sx * S_, min((sx + 1) * S_, tx_n)):
                t = ty * tx_n + tx
                tl = list(tvals[tranges[t, 0]:tranges[t, 1]])
                members |= set(tl)
                sl = list(svals[sranges[sidx, 0]:sranges[sidx, 1]])
                inside = [i for i in sl if x0[i] <= tx < x1[i] and y0[i] <= ty < y1[i]]
                assert inside == tl
        got = list(svals[sranges[sidx, 0]:sranges[sidx, 1]])
        assert got == sorted(members, key=key)
        assert np.all(sups[sranges[sidx, 0]:sranges[sidx, 1]] == sidx)
    if S_ == 1:
        assert np.array_equal(svals, tvals) and np.array_equal(sranges, tranges)


def test_tile_lists_contain_every_overlapping_gaussian():
    """Every Gaussian overlapping a pixel is in the list of that pixel's tile,
    so compositing over tile lists equals compositing over all Gaussians."""
    w, h, tw, th = 40, 30, 8, 8
    rec = S.random_records(13, 120, w, h, max_radius=11)
    keys, vals, ranges = R.bin_and_sort(rec["u"], rec["v"], rec["depth"], rec["extent"], np.arange(120),
                                        w, h, tw, th)
    tx_n = (w + tw - 1) // tw
    for y in range(h):
        for x in range(w):
            t = (y // th) * tx_n + x // tw
            lst = set(vals[ranges[t, 0]:ranges[t, 1]].tolist())
            for i in range(120):
                if abs(x + 0.5 - rec["u"][i]) <= rec["extent"][i, 0] and abs(y + 0.5 - rec["v"][i]) <= rec["extent"][i, 1]:
                    assert i in lst


def test_image_independent_of_tile_shape_in_full_render():
    sc = S.tiny_scene(0, 300, log_scale_mean=-2.5)
    cam = S.tetra_cameras(width=50, height=38)[2]
    imgs = []
    for tw, th in ((8, 8), (16, 16), (32, 8)):
        rp = R.RasterParams(tile_w=tw, tile_h=th)
        out = R.render(sc.means, sc.log_scales, sc.quats, sc.opacity_logits, sc.sh, 0, cam, rp)
        imgs.append(out["rgb"].detach().numpy())
    assert np.array_equal(imgs[0], imgs[1]) and np.array_equal(imgs[0], imgs[2])


def test_overlap_box_contains_every_pixel_that_can_pass_alpha_min():
    """Eq. 5 evaluated directly on the whole 3-sigma square: every pixel where
    o exp(P) >= alpha_min lies in the overlap box, and the box is never larger
    than the square."""
    sc = S.mixture_scene(2, 3000, sh_degree=0, log_scale_mean=-2.8)
    cam = S.look_at_camera((3.0, -2.0, 2.5), 160, 120)
    rp = R.RasterParams()
    pr = R.project(sc.means, sc.log_scales, sc.quats, sc.opacity_logits, sc.sh, 0, cam, rp)
    amin = R.f32(rp.alpha_min)
    uv = pr["uv"].detach().numpy()
    con = pr["conic"].detach().numpy()
    o = pr["opacity"].detach().numpy()
    r = pr["radius"].numpy()
    ext = pr["extent"].numpy()
    assert np.all(ext <= r[:, None]) and np.all(ext >= 0)
    assert (ext < r[:, None]).any()          # the box does cut the square
    checked = 0
    for i in range(0, len(r), 7):
        ri = int(r[i])
        if ri > 40:
            continue
        off = np.arange(-ri, ri + 1, dtype=np.float64)
        px = np.floor(uv[i, 0]) + 0.5 + off
        py = np.floor(uv[i, 1]) + 0.5 + off
        dx = px[None, :] - uv[i, 0]
        dy = py[:, None] - uv[i, 1]
        a, b, c = con[i]
        P = -0.5 * (a * dx * dx + c * dy * dy) - b * dx * dy
        passes = (o[i] * np.exp(P) >= amin) & (np.abs(dx) <= ri) & (np.abs(dy) <= ri)
        inbox = (np.abs(dx) <= ext[i, 0]) & (np.abs(dy) <= ext[i, 1])
        assert not (passes & ~inbox).any(), i
        checked += 1
    assert checked > 100


def test_dropping_non_contributing_entries_changes_no_pixel_of_the_tile():
    """tile_contributes false => the Gaussian takes no part in any pixel of
    the tile: compositing the tile's pixels without those Gaussians gives the
    same result; and a Gaussian it calls contributing does get blended
    somewhere in the tile (with thresholds that cannot stop compositing)."""
    w, h, tw, th = 40, 29, 8, 8
    rec = S.random_records(31, 300, w, h, max_radius=14)
    rp = R.RasterParams(tile_w=tw, tile_h=th)
    n = len(rec["u"])
    uv = torch.tensor(np.stack([rec["u"], rec["v"]], 1), dtype=torch.float64)
    con = torch.tensor(rec["conic"], dtype=torch.float64)
    op = torch.tensor(rec["opacity"], dtype=torch.float64)
    col = torch.tensor(rec["rgb"], dtype=torch.float64)
    dep = torch.tensor(rec["depth"], dtype=torch.float64)
    ext = torch.tensor(rec["extent"].astype(np.int64))
    no_stop = R.RasterParams(tile_w=tw, tile_h=th, t_min=0.0)
    dead_total = 0
    for ty in range((h + th - 1) // th):
        for tx in range((w + tw - 1) // tw):
            xs = np.arange(tx * tw, min((tx + 1) * tw, w))
            ys = np.arange(ty * th, min((ty + 1) * th, h))
            px, py = [a.reshape(-1) for a in np.meshgrid(xs, ys)]
            live = np.array([R.tile_contributes(rec["u"][i], rec["v"][i], *rec["conic"][i],
                                                rec["opacity"][i], *rec["extent"][i], tx, ty,
                                                tw, th, w, h, rp) for i in range(n)])
            dead_total += int((~live).sum())
            ids = torch.arange(n)
            full = R.composite(uv, con, op, col, dep, ext, ids, w, h, rp, px=px, py=py)
            k = torch.as_tensor(np.nonzero(live)[0])
            part = R.composite(uv[k], con[k], op[k], col[k], dep[k], ext[k], ids[k], w, h, rp,
                               px=px, py=py)
            assert torch.equal(full["rgb"], part["rgb"])
            assert torch.equal(full["last"], part["last"])
            for i in k[:8].tolist():
                # a live Gaussian alone (no termination) blends at some pixel
                s1 = slice(i, i + 1)
                one = R.composite(uv[s1], con[s1], op[s1], col[s1], dep[s1], ext[s1], ids[s1],
                                  w, h, no_stop, px=px, py=py)
                assert int(one["n_blended"].sum()) >= 1, (tx, ty, i)
    assert dead_total > 0
