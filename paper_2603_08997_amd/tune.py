"""Launch-shape tuner: picks the tile shape, the LDS batch (list entries per
compositing batch) and the super-tile edge for a workload by timing one
forward + backward of its views with each candidate, stores the choice in a
JSON file keyed by the device, the Gaussian count, the SH degree and the view
sizes, and returns the stored choice on later calls.

The candidates change how the work is laid out, never the image or the
gradients (the compositing order is the lists' depth order in every case).
"""
from __future__ import annotations

import dataclasses
import itertools
import json
import os
import time

import torch

from . import skipgs as sk

TILES = ((16, 16), (32, 8), (8, 8))
BATCHES = (32, 64, 128, 256)
SUPER_TILES = (4, 8)


def default_store() -> str:
    return os.environ.get("SGS_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "skipgs", "tuned.json"))


def workload_key(n: int, sh_degree: int, cams) -> str:
    dev = torch.cuda.get_device_name(torch.cuda.current_device())
    views = ",".join(f"{c.width}x{c.height}" for c in cams)
    return f"{dev}|n={n}|sh={sh_degree}|views={views}"


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(path: str, table: dict) -> None:
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _capacity(planes, n, sh_degree, cams, rp) -> int:
    """Pair capacity the views need (probing until no overflow)."""
    cap = 1 << 16
    out = torch.empty(3 * sum(c.width * c.height for c in cams), device=planes.device)
    for _ in range(4):
        ws = sk.alloc_bytes(sk.forward_workspace_size(rp, n, cams, cap))
        sk.clear_status(ws)
        sk.render_forward(planes, n, sh_degree, cams, rp, ws, cap, out)
        flags, _, need = sk.read_status(ws)
        del ws
        if not flags & sk.STATUS_PAIR_OVERFLOW:
            return int(need * 1.05) + 4096
        cap = int(need * 1.25) + 4096
    raise RuntimeError("pair capacity probe did not converge")


def time_candidate(planes, n, sh_degree, cams, dl, rp, reps: int = 3) -> float:
    """Mean ms of one forward + backward of all views in one launch each."""
    cap = _capacity(planes, n, sh_degree, cams, rp)
    ws = sk.alloc_bytes(sk.forward_workspace_size(rp, n, cams, cap))
    sk.clear_status(ws)
    rgb = torch.empty(3 * sum(c.width * c.height for c in cams), device=planes.device)
    grads = torch.zeros_like(planes)

    def step():
        sk.render_forward(planes, n, sh_degree, cams, rp, ws, cap, rgb)
        sk.render_backward(planes, n, sh_degree, cams, rp, ws, cap, dl, None, grads)

    step()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        step()
    b.record()
    torch.cuda.synchronize()
    if sk.read_status(ws)[0]:
        raise RuntimeError("status flags set while tuning")
    return a.elapsed_time(b) / reps


def tune(planes, n: int, sh_degree: int, cams, dl, store: str | None = None,
         base: sk.RasterParams | None = None, retune: bool = False, log=None):
    """The fastest candidate for this workload (RasterParams) and the tuning
    record (stored or fresh). ``dl``: a cotangent of the views' images."""
    store = default_store() if store is None else store
    key = workload_key(n, sh_degree, cams)
    table = _load(store)
    base = base or sk.RasterParams()
    if not retune and key in table:
        rec = table[key]
        ch = rec["choice"]
        return dataclasses.replace(base, tile_w=ch["tile_w"], tile_h=ch["tile_h"],
                                   lds_batch=ch["lds_batch"], super_tile=ch["super_tile"]), \
            dict(rec, reused=True)
    t0 = time.perf_counter()
    trials = []
    for (tw, th), bsz, st in itertools.product(TILES, BATCHES, SUPER_TILES):
        rp = dataclasses.replace(base, tile_w=tw, tile_h=th, lds_batch=bsz, super_tile=st)
        ms = time_candidate(planes, n, sh_degree, cams, dl, rp)
        trials.append({"tile_w": tw, "tile_h": th, "lds_batch": bsz, "super_tile": st, "ms": ms})
        if log is not None:
            log(f"tune {tw}x{th} B{bsz} S{st}: {ms:.3f} ms")
        torch.cuda.empty_cache()
    best = min(trials, key=lambda t: t["ms"])
    rec = {"choice": {k: best[k] for k in ("tile_w", "tile_h", "lds_batch", "super_tile")},
           "ms": best["ms"], "trials": trials, "seconds": time.perf_counter() - t0}
    table[key] = rec
    _save(store, table)
    return dataclasses.replace(base, **rec["choice"]), dict(rec, reused=False)
