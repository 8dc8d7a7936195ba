"""Benchmark: post-densification iterations/s of SkipGS-gated vs full-backward
3DGS training on one MI355X, with the dominant kernel's roofline fraction
and the FP64 oracle timed on the host as a CPU reference.

    python bench.py [--steps K] [--warmup W] [--gate-preroll P] [--gpus 1]
    python bench.py --workload matched     # iterations and time to the full run's loss
    python bench.py --workload single      # 1M Gaussians, per-view stage medians
    python bench.py --workload dense       # 6M dense scene: backward GB/s, peak memory
    python bench.py --workload batched     # 8 mixed-resolution views per launch
    python bench.py --workload densify     # clone / split / prune step and its statistic
    python bench.py --workload atomics     # scattered FP32 atomic-add ceiling

Workload (defaults): 3,000,000 Gaussians (SH degree 3, ground-plane + two
clusters), 200 views at 1600x1060 on a hemisphere of radius 4-5, 16x16 tiles,
targets rendered from the ground-truth set, training from a perturbed copy,
uniform view sampling, loss 0.8 L1 + 0.2 (1 - SSIM), gate with EMA decay 0.9,
skip within 2% of the view's EMA, >= 50% backward per 100 iterations, Adam
(means lr 1.6e-4). One step = one training iteration: forward render, loss,
gate, and (when the gate opens) loss backward, render backward and Adam,
enqueued as one call with the view read on the device (replayed from a
captured HIP graph by default). Each run first takes P untimed iterations
(the gate pre-roll, the same for the gated and the full run) so that the
timed steps see the gate in its steady state, then W untimed and K timed
steps. Inputs are resident in HBM before the timed region starts.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# HBM bytes per dispatch measured with rocprofv3 counters for the default
# workload (written by paper_2603_08997_amd.profiling traffic); used only while
# the sources still match the ones measured
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_train_3M_1600x1060.txt")
FP32_VECTOR_PEAK_TFLOPS = 157.3
# FP32 operations per blended (pixel, Gaussian) pair in the compositing
# kernels, counted from the arithmetic each pair performs (FMA = 2, exp = 1).
FWD_FLOPS_PER_PAIR = 27
BWD_FLOPS_PER_PAIR = 62


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 2000 training iterations; 20 batches of the "
                         "batched workload)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps before the timed ones (default: 20; 2 batches)")
    ap.add_argument("--gate-preroll", type=int, default=1000,
                    help="untimed training iterations before the warmup, the same for every run")
    ap.add_argument("--n", type=int, default=3_000_000)
    ap.add_argument("--views", type=int, default=200)
    ap.add_argument("--width", type=int, default=1600)
    ap.add_argument("--height", type=int, default=1060)
    ap.add_argument("--gate", choices=["windowed", "paper"], default="windowed")
    ap.add_argument("--runs", default="gated,full",
                    help="comma list of gated, full, paper, paper_nobudget")
    ap.add_argument("--adam", choices=["dense", "visible"], default="dense",
                    help="dense Adam (every Gaussian, the paper's optimiser) or the "
                         "visible-only step")
    ap.add_argument("--super-tile", type=int, default=8)
    ap.add_argument("--lds-batch", type=int, default=64)
    ap.add_argument("--split-prefix", type=int, default=8192,
                    help="super-tile list pairs split into tile lists before compositing "
                         "(0: whole lists)")
    ap.add_argument("--no-graph", action="store_true",
                    help="enqueue every timed iteration instead of replaying a captured graph")
    ap.add_argument("--stage-iters", type=int, default=200,
                    help="iterations of the stage-by-stage pass that times each stage")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--eval-views", type=int, default=200)
    ap.add_argument("--match-iters", type=int, default=10000,
                    help="matched workload: iterations of the full run")
    ap.add_argument("--match-every", type=int, default=250,
                    help="matched workload: gated iterations between loss evaluations")
    ap.add_argument("--tune-store", default=None,
                    help="batched workload: the tuner's JSON store (default ~/.cache/skipgs)")
    ap.add_argument("--retune", action="store_true",
                    help="batched workload: tune again even if a stored choice exists")
    ap.add_argument("--workload", choices=["train", "matched", "single", "dense", "batched",
                                           "densify", "atomics"],
                    default="train")
    return ap.parse_args()


# ---------------------------------------------------------------------------
# CPU baseline: the FP64 oracle on the host
# ---------------------------------------------------------------------------
def cpu_baseline(gt, init, cam, crop=64):
    """The FP64 oracle on a bounded sample of one training iteration of the
    benchmark workload: the projection of all Gaussians (forward and, once,
    backward) plus compositing, loss and backward of a crop x crop window at
    the image centre; the window's time is scaled to the full image."""
    from oracle import render as OR, loss as OL
    threads = torch.get_num_threads()
    leaves = {k: torch.tensor(np.asarray(v, np.float64), requires_grad=True) for k, v in
              dict(means=init.means, log_scales=init.log_scales, quats=init.quats,
                   opacity_logits=init.opacity_logits, sh=init.sh).items()}
    t0 = time.perf_counter()
    pr = OR.project(leaves["means"], leaves["log_scales"], leaves["quats"],
                    leaves["opacity_logits"], leaves["sh"], init.sh_degree, cam, OR.RasterParams())
    t_proj = time.perf_counter() - t0
    x0, y0 = cam.width // 2 - crop // 2, cam.height // 2 - crop // 2
    ys, xs = np.meshgrid(np.arange(y0, y0 + crop), np.arange(x0, x0 + crop), indexing="ij")
    px, py = torch.tensor(xs.reshape(-1)), torch.tensor(ys.reshape(-1))
    with torch.no_grad():
        gpr = OR.project(gt.means, gt.log_scales, gt.quats, gt.opacity_logits, gt.sh, gt.sh_degree,
                         cam, OR.RasterParams())
        tgt = OR.composite(gpr["uv"], gpr["conic"], gpr["opacity"], gpr["rgb"], gpr["depth"],
                           gpr["extent"], gpr["ids"], cam.width, cam.height, OR.RasterParams(),
                           px=px, py=py)["rgb"].reshape(3, crop, crop)
    # the window's compositing, loss and backward to the projected records
    recs = {k: pr[k].detach().clone().requires_grad_(True)
            for k in ("uv", "conic", "opacity", "rgb")}
    t1 = time.perf_counter()
    out = OR.composite(recs["uv"], recs["conic"], recs["opacity"], recs["rgb"], pr["depth"],
                       pr["extent"], pr["ids"], cam.width, cam.height, OR.RasterParams(),
                       px=px, py=py)
    L = OL.photometric_loss(out["rgb"].reshape(3, crop, crop), tgt)
    L.backward()
    t_pix = time.perf_counter() - t1
    # the projection backward from those record gradients, once
    t2 = time.perf_counter()
    torch.autograd.backward([pr[k] for k in recs], [recs[k].grad for k in recs])
    t_pbwd = time.perf_counter() - t2
    scale = (cam.width * cam.height) / float(crop * crop)
    est = t_proj + t_pbwd + t_pix * scale
    return {"value": 1.0 / est, "unit": "iters/s", "cores": threads, "kind": "oracle",
            "sample": (f"one iteration of the benchmark workload: FP64 projection of all "
                       f"{init.n} Gaussians forward ({t_proj:.1f} s) and backward "
                       f"({t_pbwd:.1f} s), compositing, loss and backward of a {crop}x{crop} "
                       f"window ({t_pix:.1f} s) scaled x{scale:.0f} to the "
                       f"{cam.width}x{cam.height} view; torch CPU threads={threads}"),
            "seconds_per_iter_estimate": est}


def cpu_oracle_tiny():
    """The FP64 oracle on the whole 1,000-Gaussian scene (4 views of 64x64:
    forward, loss and backward of each view), single-threaded and on all
    host threads, measured in full."""
    from oracle import grad as OG, render as OR
    from paper_2603_08997_amd import scenes as S
    sc = S.tiny_scene(S.SEED_TINY_RENDER)
    tg = S.tiny_scene(S.SEED_TINY_TARGET)
    cams = S.tetra_cameras()
    arrs = OG.scene_dict(sc)
    rp = OR.RasterParams()
    with torch.no_grad():
        targets = [OR.render(tg.means, tg.log_scales, tg.quats, tg.opacity_logits, tg.sh, 0, c,
                             rp)["rgb"].reshape(3, c.height, c.width) for c in cams]
    out = {}
    all_threads = torch.get_num_threads()
    for label, th in (("1_thread", 1), ("all_threads", all_threads)):
        torch.set_num_threads(th)
        t0 = time.perf_counter()
        for c, t in zip(cams, targets):
            OG.loss_and_grads(arrs, 0, c, rp, t)
        out[label] = {"seconds_per_4_views": time.perf_counter() - t0, "threads": th}
    torch.set_num_threads(all_threads)
    out["workload"] = "1,000 Gaussians SH0, 4 views 64x64, forward + loss + backward per view"
    out["cores"] = os.cpu_count()
    return out


def hbm_copy_probe(nbytes=1 << 30, reps=20):
    """Streaming copy of nbytes through a plain elementwise kernel (torch's
    multiply by 1 into another buffer, so that it runs on the compute units
    rather than as a DMA transfer) timed with HIP events: bytes read plus
    bytes written per second, the practical ceiling of a kernel that reads
    and writes equal amounts. The same copies are the known-size reference
    for the HBM byte counters."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        torch.mul(src, 1.0, out=dst)
    b.record()
    torch.cuda.synchronize()
    gbs = 2.0 * nbytes * reps / (a.elapsed_time(b) * 1e-3) / 1e9
    del src, dst
    return gbs


# ---------------------------------------------------------------------------
# Training workload
# ---------------------------------------------------------------------------
class Setup:
    """Scene, cameras, view sequence, pair capacity and targets of the
    training workload (seeded; rendered on the GPU before any timing)."""

    def __init__(self, args, length):
        from paper_2603_08997_amd import scenes as S
        from paper_2603_08997_amd import skipgs as sk
        from paper_2603_08997_amd.train import measure_capacity, render_targets
        t0 = time.perf_counter()
        log(f"setup: scene n={args.n} views={args.views} {args.width}x{args.height}")
        self.gt = S.mixture_scene(S.SEED_SCENE, args.n, sh_degree=3)
        self.init = S.perturb(self.gt, S.SEED_INIT_PERTURB)
        self.cams = S.hemisphere_cameras(S.SEED_CAMERAS, args.views, args.width, args.height)
        self.seq = S.view_sequence(S.SEED_VIEW_SEQUENCE, args.views, length)
        self.rp = sk.RasterParams(super_tile=args.super_tile, lds_batch=args.lds_batch,
                             split_prefix=args.split_prefix)
        need = max(measure_capacity(self.gt, self.cams, self.rp),
                   measure_capacity(self.init, self.cams, self.rp))
        self.cap = int(need * 1.3) + 4096
        log(f"setup: capacity needed {need}, allocated {self.cap}")
        self.targets = render_targets(self.gt, self.cams, self.rp, self.cap)
        torch.cuda.synchronize()
        log(f"setup done in {time.perf_counter() - t0:.1f} s")


def gate_of(args, run, n_views):
    from paper_2603_08997_amd import skipgs as sk
    if run == "paper":
        return sk.paper_gate(n_views)
    if run == "paper_nobudget":
        return dataclasses.replace(sk.paper_gate(n_views), budget=False)
    return sk.windowed_gate(n_views) if args.gate == "windowed" else sk.paper_gate(n_views)


def capture(tr):
    """A graph of one training iteration (sequence step + iteration),
    captured on a side stream after one eager iteration there."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        tr.step(s.cuda_stream)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        tr.step(s.cuda_stream)
    torch.cuda.synchronize()
    return g


def timed_run(args, st, run, visible_only):
    """Pre-roll, warmup and timed steps of one run; returns its results and
    the trainer (left after the timed steps)."""
    from paper_2603_08997_amd import skipgs as sk
    from paper_2603_08997_amd.train import Trainer
    gp = gate_of(args, run, args.views)
    tr = Trainer(st.init, st.cams, st.targets, st.rp, gp, st.cap, gated=(run != "full"),
                 sequence=st.seq, visible_only=visible_only)
    graph = None if args.no_graph else capture(tr)   # (two iterations of the pre-roll)
    step = (lambda: graph.replay()) if graph is not None else (lambda: tr.step())
    done = 0 if graph is None else 2
    for _ in range(max(0, args.gate_preroll - done) + args.warmup):
        step()
    torch.cuda.synchronize()
    b0, t0 = tr.backward_count()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    gpu_s = ev0.elapsed_time(ev1) * 1e-3
    b1, t1 = tr.backward_count()
    flags, _, _ = tr.status()
    if flags & sk.STATUS_PAIR_OVERFLOW:
        raise RuntimeError("pair capacity overflow during the timed run")
    bf = (b1 - b0) / max(1, t1 - t0)
    res = {"iters_per_s": args.steps / wall, "ms_per_step": 1000 * wall / args.steps,
           "gpu_ms_per_step": 1000 * gpu_s / args.steps, "backward_fraction": bf,
           "iterations_before_timing": args.gate_preroll + args.warmup, "graph": graph is not None}
    log(f"{run}: {res['iters_per_s']:.1f} it/s, backward fraction {bf:.3f}")
    return res, tr


def stage_pass(args, st, tr, start):
    """Stage-by-stage iterations with HIP events (after the timed steps, on
    the same trainer): per-stage means over executed and skipped iterations."""
    from paper_2603_08997_amd.train import StageTimer
    timer = StageTimer()
    n = args.stage_iters
    seq = np.asarray(st.seq)
    dseq = torch.as_tensor(seq.astype(np.int32)).cuda()
    gslots = torch.zeros(n, dtype=torch.int32, device="cuda")
    for k in range(n):
        t = (start + k) % len(seq)
        tr.iteration(int(seq[t]), dseq[t:t + 1], gslots[k:k + 1], timer=timer)
    torch.cuda.synchronize()
    g = gslots.cpu().numpy()
    return {"all": timer.summary(), "executed": timer.summary(mask=g == 1) if (g == 1).any() else None,
            "skipped": timer.summary(mask=g == 0) if (g == 0).any() else None,
            "backward_fraction": float(g.mean())}


def train_counters(tr, views):
    """Per-view work of the forward, averaged over a few views."""
    from paper_2603_08997_amd import skipgs as sk
    keys = ("blended", "evaluated", "pairs", "pairs_kept", "items", "items_rest", "redo",
            "segments", "used", "visible")
    acc = {k: [] for k in keys}
    for v in views:
        tr.render(v, tr.rgb)
        torch.cuda.synchronize()
        c = sk.read_counters(tr.ws)
        for k in keys:
            acc[k].append(c[k])
    return {k: float(np.mean(x)) for k, x in acc.items()}


def roofline(args, stages, bf, cnt, visible_only):
    """The dominant kernel of an iteration (largest time per iteration among
    the compositing forward, the compositing backward and the fused projection
    backward + Adam) against its bound; the binning stage (a chain of sorts,
    scans and the tile-list split) is reported beside them against HBM."""
    ex = stages["executed"] or stages["all"]
    allm = stages["all"]
    F = 11 + 3 * 16
    n, vis = args.n, cnt["visible"]
    # fused backward + Adam: parameters, first and second moments read and
    # written once per plane of every updated Gaussian, the visibility word of
    # every Gaussian, the 48-byte gradient accumulator and the 16-byte colour
    # record of every visible one
    upd = vis if visible_only else n
    fused_bytes = upd * F * 4 * 6 + n * 4 + vis * (48 + 16)
    # binning: compaction (visibility word per entry; depth and key/value of
    # every visible entry), four depth-sort passes over 8-byte key/value pairs
    # (read + write), the super-tile counts gathered and scanned, the records
    # the emission reads (32 B per visible entry) and the 8-byte pairs it
    # writes, one pass of the super-tile sort (read + write); the split reads
    # every pair of the split prefixes (at most 512 per segment; 8 B) and its
    # entry's record (32 B) and writes its tile mask (8 B), then reads mask and
    # entry again (12 B) and writes every tile-list entry of the prefixes (4 B)
    P, I = cnt["pairs"], cnt["items"]
    Ps = min(cnt["pairs_kept"], 512 * cnt["segments"])
    bin_bytes = (n * 4 + vis * 12 + 4 * vis * 16 + vis * 12 + vis * 32 + P * 8 + P * 16
                 + Ps * (8 + 32 + 8) + Ps * 12 + I * 4)
    cands = {
        "raster_forward": dict(ms=allm["rasterize"], weight=1.0, bound="alu",
                               work=cnt["blended"] * FWD_FLOPS_PER_PAIR / 1e12, unit="TFLOP/s",
                               peak=FP32_VECTOR_PEAK_TFLOPS),
        "binning": dict(ms=allm["bin"], weight=1.0, bound="hbm", work=bin_bytes / 1e9,
                        unit="GB/s", peak=HBM_PEAK_GBS, stage=True),
        "raster_backward": dict(ms=ex["raster_bwd"], weight=bf, bound="alu",
                                work=cnt["blended"] * BWD_FLOPS_PER_PAIR / 1e12, unit="TFLOP/s",
                                peak=FP32_VECTOR_PEAK_TFLOPS),
        "project_backward_adam": dict(ms=ex["project_bwd"], weight=bf, bound="hbm",
                                      work=fused_bytes / 1e9, unit="GB/s", peak=HBM_PEAK_GBS),
    }
    summary = {}
    for k, c in cands.items():
        ach = c["work"] / (c["ms"] * 1e-3) if c["ms"] > 0 else 0.0
        summary[k] = {"avg_launch_ms": c["ms"], "ms_per_iteration": c["ms"] * c["weight"],
                      "bound": c["bound"], "achieved": ach, "unit": c["unit"],
                      "frac": ach / c["peak"]}
        if c.get("stage"):
            summary[k]["stage_of_kernels"] = True
    name = max((k for k in summary if not cands[k].get("stage")),
               key=lambda k: summary[k]["ms_per_iteration"])
    c, sm = cands[name], summary[name]
    traffic = None
    if (args.n, args.width, args.height) == (3_000_000, 1600, 1060) and not visible_only:
        from paper_2603_08997_amd.profiling import load_traffic
        rec = load_traffic(TRAFFIC_FILE)
        if rec is not None and name in rec["kernels"]:
            traffic = rec["kernels"][name]["traffic_bytes"]
    return {"kernel": name, "bound": c["bound"], "achieved": sm["achieved"], "peak": c["peak"],
            "unit": c["unit"], "frac": sm["frac"], "traffic": traffic, "avg_launch_ms": c["ms"],
            "blended_pairs_per_launch": cnt["blended"], "fused_bytes_per_launch": fused_bytes,
            "binning_bytes_per_launch": bin_bytes,
            "flops_per_pair": {"forward": FWD_FLOPS_PER_PAIR, "backward": BWD_FLOPS_PER_PAIR},
            "kernels": summary}


def run_train(args):
    runs = args.runs.split(",")
    for r in runs:
        if r not in ("gated", "full", "paper", "paper_nobudget"):
            raise SystemExit(f"unknown run {r!r} (gated, full, paper, paper_nobudget)")
    length = args.gate_preroll + args.warmup + args.steps + args.stage_iters + 8
    st = Setup(args, length)
    visible_only = args.adam == "visible"
    eval_views = list(range(min(args.views, args.eval_views)))
    results, keep = {}, {}
    for run in runs:
        res, tr = timed_run(args, st, run, visible_only)
        res["final_mean_loss"] = tr.mean_loss(eval_views)
        log(f"{run}: mean loss over {len(eval_views)} views after "
            f"{res['iterations_before_timing'] + args.steps} iterations "
            f"{res['final_mean_loss']:.6f}")
        if run == runs[0]:
            start = res["iterations_before_timing"] + args.steps + 2
            keep["stages"] = stage_pass(args, st, tr, start)
            keep["counters"] = train_counters(tr, list(range(min(8, args.views))))
        elif run == "full":
            keep["stages_full"] = stage_pass(args, st, tr, res["iterations_before_timing"] +
                                             args.steps + 2)
        results[run] = res
        del tr
        torch.cuda.empty_cache()
    head = runs[0]
    headline = results[head]
    stages = keep["stages"]
    out = {
        "metric": "post-densification iters/s (gated vs full) at 1 GPU",
        "value": headline["iters_per_s"],
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": headline["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": (f"{'gated' if head != 'full' else 'full-backward'} 3DGS "
                                f"post-densification training, {args.n} Gaussians SH3, "
                                f"{args.views} views {args.width}x{args.height}, 16x16 tiles, "
                                f"{args.gate} gate, {args.adam} Adam"),
                   "gaussians": args.n, "views": args.views, "width": args.width,
                   "height": args.height, "gate": args.gate, "adam": args.adam,
                   "gate_preroll": args.gate_preroll, "super_tile": args.super_tile,
                   "lds_batch": args.lds_batch, "split_prefix": args.split_prefix,
                   "graph": headline["graph"]},
        "skip_fraction": 1.0 - headline["backward_fraction"],
    }
    full = results.get("full")
    if full and head != "full":
        out["full_iters_per_s"] = full["iters_per_s"]
        if out["skip_fraction"] > 0:
            # only when the gate actually skipped in the timed run
            out["gated_over_full"] = headline["iters_per_s"] / full["iters_per_s"]
            n_it = headline["iterations_before_timing"] + args.steps
            out["equal_iteration_loss"] = {
                "iterations": n_it, "gated": headline["final_mean_loss"],
                "full": full["final_mean_loss"],
                "rel_diff": (headline["final_mean_loss"] - full["final_mean_loss"]) /
                full["final_mean_loss"],
                "note": "loss after the same number of iterations; the matched-loss criterion "
                        "(iterations and time to reach the full run's loss) is the 'matched' "
                        "workload"}
    for name in ("paper", "paper_nobudget"):
        r = results.get(name)
        if r and name != head:
            out[f"{name}_iters_per_s"] = r["iters_per_s"]
            out[f"{name}_skip_fraction"] = 1.0 - r["backward_fraction"]
    sk_ = stages["skipped"]
    full_st = keep.get("stages_full", stages)["all"]
    if sk_ is not None:
        out["skipped_iteration_cost"] = sum(sk_.values()) / sum(full_st.values())
    out["stage_ms"] = {k: ({kk: round(vv, 4) for kk, vv in v.items()} if isinstance(v, dict) else v)
                       for k, v in stages.items()}
    cnt = keep["counters"]
    out["per_view"] = cnt
    bf = headline["backward_fraction"]
    out["roofline"] = roofline(args, stages, bf if bf > 0 else 1.0, cnt, visible_only)
    out["hbm_copy_GBps"] = hbm_copy_probe()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(st.gt, st.init, st.cams[0])
        out["cpu_oracle_tiny"] = cpu_oracle_tiny()
    print(json.dumps(out), flush=True)


def run_matched(args):
    """The config-3 criterion: the full run trains for --match-iters
    iterations; the gated run trains until its mean loss over the evaluation
    views is within 1% of the full run's final loss (evaluated every
    --match-every iterations, untimed), or for at most 2.5x as many
    iterations. Reports iterations and training wall-clock for both."""
    args.warmup = 0
    cap_iters = int(2.5 * args.match_iters)
    st = Setup(args, cap_iters + 8)
    visible_only = args.adam == "visible"
    eval_views = list(range(min(args.views, args.eval_views)))
    from paper_2603_08997_amd.train import Trainer

    def trainer(run):
        return Trainer(st.init, st.cams, st.targets, st.rp, gate_of(args, run, args.views),
                       st.cap, gated=(run != "full"), sequence=st.seq, visible_only=visible_only)

    def train_for(tr, iters, graph):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(iters):
            graph.replay()
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) * 1e-3

    tr = trainer("full")
    g = capture(tr)                      # two iterations (timed below as part of training)
    t_full = train_for(tr, args.match_iters - 2, g)
    L_full = tr.mean_loss(eval_views)
    full_it_s = (args.match_iters - 2) / t_full
    log(f"full: {args.match_iters} iterations, loss {L_full:.6f}, {full_it_s:.1f} it/s")
    del g, tr
    torch.cuda.empty_cache()
    tr = trainer("gated")
    g = capture(tr)
    done, t_gated, trace = 2, 0.0, []
    target = 1.01 * L_full
    L = float("inf")
    while done < cap_iters:
        k = min(args.match_every - (done % args.match_every), cap_iters - done)
        t_gated += train_for(tr, k, g)
        done += k
        L = tr.mean_loss(eval_views)
        trace.append((done, round(L, 7)))
        if L <= target:
            break
    b, t = tr.backward_count()
    reached = L <= target
    log(f"gated: {done} iterations, loss {L:.6f} (target {target:.6f}, reached {reached})")
    gated_it_s = (done - 2) / t_gated
    est_full_time = args.match_iters / full_it_s
    out = {"metric": "post-densification iters/s (gated vs full) at 1 GPU",
           "value": gated_it_s, "unit": "iters/s", "n_gpus": 1, "steps": done,
           "warmup": 2, "ms_per_step": 1000.0 / gated_it_s, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": (f"matched final loss: gated until within 1% of the full run's "
                                   f"loss after {args.match_iters} iterations, {args.n} Gaussians "
                                   f"SH3, {args.views} views {args.width}x{args.height}, "
                                   f"{args.gate} gate, {args.adam} Adam")},
           "full": {"iterations": args.match_iters, "seconds": est_full_time,
                    "iters_per_s": full_it_s, "final_loss": L_full},
           "gated": {"iterations": done, "seconds": done / gated_it_s, "iters_per_s": gated_it_s,
                     "final_loss": L, "reached_within_1pct": reached,
                     "backward_fraction": b / max(1, t), "loss_trace": trace},
           "time_ratio_gated_over_full": (done / gated_it_s) / est_full_time,
           "iteration_ratio_gated_over_full": done / args.match_iters}
    print(json.dumps(out), flush=True)


# ---------------------------------------------------------------------------
# Other workloads
# ---------------------------------------------------------------------------
def run_single(args):
    """One view per launch of 1,000,000 Gaussians at 1245x825 (150 views on
    the hemisphere): forward (projection + compositing), sort (binning) and
    backward (compositing backward + projection backward) times per view,
    medians over the views, with a loss cotangent against a target of an
    independent scene."""
    from paper_2603_08997_amd import scenes as S
    from paper_2603_08997_amd import skipgs as sk
    from paper_2603_08997_amd.train import StageTimer, Trainer, measure_capacity, render_targets
    n, W, H, V = 1_000_000, 1245, 825, 150
    scene = S.mixture_scene(S.SEED_SCENE, n, 3)
    other = S.mixture_scene(S.SEED_TINY_TARGET, n, 3)
    cams = S.hemisphere_cameras(S.SEED_CAMERAS, V, W, H)
    rp = sk.RasterParams(super_tile=args.super_tile, lds_batch=args.lds_batch,
                             split_prefix=args.split_prefix)
    cap = int(max(measure_capacity(scene, cams, rp), measure_capacity(other, cams, rp)) * 1.3) + 4096
    targets = render_targets(other, cams, rp, cap)
    tr = Trainer(scene, cams, targets, rp, None, cap, gated=False, sequence=np.arange(V))
    timer = StageTimer()
    dseq = torch.arange(V, dtype=torch.int32, device="cuda")
    g = torch.ones(1, dtype=torch.int32, device="cuda")
    for v in range(min(5, V)):       # warmup
        tr.iteration(v, dseq[v:v + 1], g)
    for v in range(V):
        tr.iteration(v, dseq[v:v + 1], g, timer=timer)
    torch.cuda.synchronize()
    per = {k: timer.per_iter(k) for k in timer.names}
    fwd = per["project"] + per["rasterize"]
    srt = per["bin"]
    bwd = per["raster_bwd"] + per["project_bwd"]
    tot = sum(per[k] for k in timer.names)
    out = {"metric": "single-view forward / sort / backward time (median over views)",
           "value": float(np.median(tot)), "unit": "ms", "n_gpus": 1, "steps": V, "warmup": 5,
           "ms_per_step": float(np.median(tot)), "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{n} Gaussians SH3, {V} views {W}x{H}, one view per launch, "
                                  f"loss + backward with dense Adam"},
           "median_ms": {"forward": float(np.median(fwd)), "sort": float(np.median(srt)),
                         "backward": float(np.median(bwd)),
                         "loss": float(np.median(per["loss"] + per["loss_bwd"]))},
           "p90_ms": {"forward": float(np.percentile(fwd, 90)),
                      "sort": float(np.percentile(srt, 90)),
                      "backward": float(np.percentile(bwd, 90))}}
    print(json.dumps(out), flush=True)


def run_dense(args):
    """6,000,000 Gaussians of the dense cluster scene at 1600x1060 (about 60
    blended Gaussians per pixel): forward, then the backward through the
    autograd wrapper that recomputes the forward instead of keeping its
    workspace; backward time, its HBM bytes and GB/s, peak device memory."""
    from paper_2603_08997_amd import scenes as S
    from paper_2603_08997_amd import skipgs as sk
    from paper_2603_08997_amd import autograd as AG
    from paper_2603_08997_amd.train import measure_capacity
    n = 6_000_000
    scene = S.dense_cluster_scene(S.SEED_SCENE, n, 3)
    cam = S.hemisphere_cameras(S.SEED_CAMERAS, 1, 1600, 1060)[0]
    rp = sk.RasterParams(super_tile=args.super_tile, lds_batch=args.lds_batch,
                             split_prefix=args.split_prefix)
    cap = int(measure_capacity(scene, [cam], rp) * 1.2) + 4096
    planes = torch.as_tensor(scene.to_planes()).cuda()
    # per-view work of the forward
    ws = sk.alloc_bytes(sk.forward_workspace_size(rp, n, [cam], cap))
    sk.clear_status(ws)
    tmp = torch.empty(3 * cam.width * cam.height, device="cuda")
    sk.render_forward(planes, n, 3, [cam], rp, ws, cap, tmp)
    cnt = sk.read_counters(ws)
    del ws, tmp
    torch.cuda.empty_cache()
    torch.cuda.reset_peak_memory_stats()
    planes.requires_grad_(True)
    dl = torch.randn(3 * cam.width * cam.height, device="cuda",
                     generator=torch.Generator(device="cuda").manual_seed(3))
    steps = max(3, args.steps if args.steps is not None else 10)
    times = []
    for k in range(steps + 2):
        planes.grad = None
        img = AG.render(planes, n, 3, [cam], rp, cap, recompute=True)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        img.backward(dl)
        b.record()
        torch.cuda.synchronize()
        if k >= 2:
            times.append(a.elapsed_time(b))
    peak = torch.cuda.max_memory_allocated()
    F = 11 + 3 * 16
    vis = cnt["visible"]
    # backward with recompute: the forward again (parameters read, records
    # written), the compositing backward (records read, accumulators written)
    # and the projection backward (parameters and accumulators of every
    # visible Gaussian read, its gradient read and written)
    bwd_bytes = n * F * 4 + vis * (48 + 48 + 48 + 16) + vis * F * 4 * 3
    ms = float(np.median(times))
    out = {"metric": "memory-bound adjoint: backward GB/s and peak HBM",
           "value": bwd_bytes / (ms * 1e-3) / 1e9, "unit": "GB/s", "n_gpus": 1, "steps": steps,
           "warmup": 2, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"dense cluster scene, {n} Gaussians SH3, 1600x1060, backward "
                                  f"through the recomputing autograd wrapper"},
           "peak_hbm_gib": peak / 2 ** 30, "backward_ms": ms,
           "blended_per_pixel": cnt["blended"] / (cam.width * cam.height),
           "visible": vis, "backward_bytes": bwd_bytes,
           "frac_of_hbm_peak": bwd_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    print(json.dumps(out), flush=True)


def run_densify(args):
    """One adaptive-density-control step (clone / split / prune, Sec. 3) over
    the 3,000,000-Gaussian SH-3 training set, and the view-space gradient
    statistic gathered after a 1600x1060 render backward. Synthetic
    statistic: view counts U{0..11} and sums count * threshold * U(0.2, 1.1),
    so about a tenth of the seen Gaussians densify (about half of those
    split); opacity logits as drawn (some prune)."""
    from paper_2603_08997_amd import scenes as S
    from paper_2603_08997_amd import skipgs as sk
    from paper_2603_08997_amd.train import measure_capacity
    n = args.n
    scene = S.mixture_scene(S.SEED_SCENE, n, 3)
    F = 11 + 3 * 16
    rng = np.random.default_rng(11)
    planes = torch.as_tensor(scene.to_planes()).cuda()
    m = torch.zeros_like(planes)
    v = torch.zeros_like(planes)
    count = rng.integers(0, 12, n).astype(np.int32)
    g = (count * 2e-4 * rng.uniform(0.2, 1.1, n)).astype(np.float32)
    d_g, d_c = torch.as_tensor(g).cuda(), torch.as_tensor(count).cuda()
    normals = torch.as_tensor(rng.standard_normal((n, 2, 3)).astype(np.float32)).cuda()
    dp = sk.DensifyParams(scene_extent=6.0)
    cap = S.padded_stride(2 * n)
    outs = [torch.empty(F, cap, device="cuda") for _ in range(3)]
    ws = sk.alloc_bytes(sk.densify_workspace_size(n))
    d_n = torch.zeros(1, dtype=torch.int64, device="cuda")
    step = lambda: sk.densify(dp, planes, n, 3, m, v, d_g, d_c, normals, *outs, ws, d_n)
    steps = args.steps if args.steps is not None else 20
    for _ in range(2):
        step()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        step()
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    n_out = int(d_n.item())
    # outcomes, for the algorithmic bytes: decision inputs (logit, three
    # log-scales, statistic sum and count: 24 B) read by both passes; a kept
    # Gaussian reads and writes parameters and both moments (3 x 4F each
    # way); a clone writes 3 x 4F; a split Gaussian reads its parameters and
    # draws (4F + 24 B) and writes two children (2 x 3 x 4F)
    lg = planes[10, :n].cpu().numpy()
    ls = planes[3:6, :n].cpu().numpy().max(axis=0)
    dv = dp.c()
    lgt = np.float32(np.log(dv.min_opacity / (1 - dv.min_opacity)))
    lst = np.float32(np.log(np.float64(dv.percent_dense) * np.float64(dv.scene_extent)))
    alive = lg >= lgt
    cand = alive & (count > 0) & (g.astype(np.float64) >= np.float64(np.float32(2e-4)) * count)
    S_ = int((cand & (ls > lst)).sum())
    Cn = int((cand & ~(ls > lst)).sum())
    K = int(alive.sum()) - S_
    assert n_out == K + Cn + 2 * S_, (n_out, K, Cn, S_)
    step_bytes = 48 * n + K * 24 * F + Cn * 12 * F + S_ * (4 * F + 24 + 24 * F)
    # the statistic after one render backward of a view
    cam = S.hemisphere_cameras(S.SEED_CAMERAS, 1, args.width, args.height)[0]
    rp = sk.RasterParams(super_tile=args.super_tile, lds_batch=args.lds_batch,
                         split_prefix=args.split_prefix)
    pcap = int(measure_capacity(scene, [cam], rp) * 1.2) + 4096
    fws = sk.alloc_bytes(sk.forward_workspace_size(rp, n, [cam], pcap))
    sk.clear_status(fws)
    img = torch.empty(3 * cam.width * cam.height, device="cuda")
    sk.render_forward(planes, n, 3, [cam], rp, fws, pcap, img)
    grads = torch.zeros_like(planes)
    sk.render_backward(planes, n, 3, [cam], rp, fws, pcap, torch.ones_like(img) * 1e-3, None,
                       grads)
    gs = torch.zeros(n, device="cuda")
    cs = torch.zeros(n, dtype=torch.int32, device="cuda")
    sk.densify_stats([cam], n, rp, fws, pcap, gs, cs)
    torch.cuda.synchronize()
    a.record()
    for _ in range(steps):
        sk.densify_stats([cam], n, rp, fws, pcap, gs, cs)
    b.record()
    torch.cuda.synchronize()
    stats_ms = a.elapsed_time(b) / steps
    vis = int(sk.read_counters(fws)["visible"])
    stats_bytes = n * 4 + vis * 8 + n * 8 * 2   # visibility words, du dv, sum and count r/w
    gbs = step_bytes / (ms * 1e-3) / 1e9
    out = {"metric": "densification step throughput", "value": n / (ms * 1e-3), "unit": "Gaussians/s",
           "n_gpus": 1, "steps": steps, "warmup": 2, "ms_per_step": ms, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"clone / split / prune step over {n} Gaussians SH3 "
                                  f"(mixture scene, synthetic statistic) and the view-space "
                                  f"gradient statistic of a {args.width}x{args.height} view"},
           "outcomes": {"kept": K, "cloned": Cn, "split": S_, "pruned": n - int(alive.sum()),
                        "n_out": n_out},
           "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": gbs / HBM_PEAK_GBS, "bytes_per_step": step_bytes},
           "stats_kernel": {"ms": stats_ms, "bytes": stats_bytes,
                            "GBps": stats_bytes / (stats_ms * 1e-3) / 1e9, "visible": vis}}
    print(json.dumps(out), flush=True)


def run_atomics(args):
    """FP32 atomic-add throughput on the compositing backward's accumulator
    shape, as a ceiling for its atomics: 3M entries x 12 floats, 1.03M
    scattered rows of 9 floats added per launch (one list entry walked per
    row, the backward's per-view count), through torch's index_add_ (one
    float atomic per element on this device)."""
    n_entries, rows, width = args.n, 1_030_000, 9
    acc = torch.zeros(n_entries, width, device="cuda")
    g = torch.Generator(device="cuda").manual_seed(5)
    idx = torch.randint(0, n_entries, (rows,), device="cuda", generator=g)
    src = torch.rand(rows, width, device="cuda", generator=g)
    steps = args.steps if args.steps is not None else 50
    for _ in range(3):
        acc.index_add_(0, idx, src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        acc.index_add_(0, idx, src)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    rate = rows * width / (ms * 1e-3)
    out = {"metric": "scattered FP32 atomic-add throughput", "value": rate / 1e9,
           "unit": "G float atomics/s", "n_gpus": 1, "steps": steps, "warmup": 3,
           "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"index_add_ of {rows} random rows of {width} floats into a "
                                  f"{n_entries} x {width} float32 array"}}
    print(json.dumps(out), flush=True)


def run_batched(args):
    """Forward + backward of eight views of four resolutions (two each of
    640x480, 1245x825, 1600x1060, 980x545) of 2M Gaussians, gradients summed
    over the views: eight single-view launches, one launch of all views, and
    the replay of a captured graph of that launch, for the launch shape the
    tuner picks and the default one."""
    from paper_2603_08997_amd import scenes as S
    from paper_2603_08997_amd import skipgs as sk
    n = 2_000_000
    scene = S.mixture_scene(S.SEED_SCENE, n, 3)
    cams = S.batched_cameras()
    planes = torch.as_tensor(scene.to_planes()).cuda()
    px = sum(c.width * c.height for c in cams)
    dl = torch.randn(3 * px, device="cuda", generator=torch.Generator(device="cuda").manual_seed(7))
    grads = torch.zeros_like(planes)
    steps = max(3, args.steps if args.steps is not None else 20)
    warm = max(1, args.warmup if args.warmup is not None else 2)
    ev = lambda: torch.cuda.Event(enable_timing=True)
    # the launch shape: the project's tuner (tile shape x LDS batch x
    # super-tile, timed on this batch; the choice is stored and reused)
    from paper_2603_08997_amd import tune as T
    tuned, record = T.tune(planes, n, 3, cams, dl, store=args.tune_store, retune=args.retune,
                           log=log)
    log(f"tuner: {record['choice']} ({record['ms']:.3f} ms; "
        f"{'reused' if record['reused'] else 'tuned in %.0f s' % record['seconds']})")
    shapes = [tuned] + ([sk.RasterParams()] if tuned != sk.RasterParams() else [])
    results = {}
    for rp in shapes:
        tag = f"{rp.tile_w}x{rp.tile_h}/S{rp.super_tile}/B{rp.lds_batch}"

        def capacity(cs):
            cap = 1 << 16
            for _ in range(3):
                ws = sk.alloc_bytes(sk.forward_workspace_size(rp, n, cs, cap))
                sk.clear_status(ws)
                out = torch.empty(3 * sum(c.width * c.height for c in cs), device="cuda")
                sk.render_forward(planes, n, 3, cs, rp, ws, cap, out)
                flags, _, need = sk.read_status(ws)
                if not flags:
                    return int(need * 1.05) + 4096
                cap = int(need * 1.25) + 4096
            raise RuntimeError("capacity probe did not converge")

        cap = capacity(cams)
        ws = sk.alloc_bytes(sk.forward_workspace_size(rp, n, cams, cap))
        sk.clear_status(ws)
        rgb = torch.empty(3 * px, device="cuda")
        per = []
        off = 0
        for c in cams:
            k = 3 * c.width * c.height
            cv = capacity([c])
            w = sk.alloc_bytes(sk.forward_workspace_size(rp, n, [c], cv))
            sk.clear_status(w)
            per.append((c, cv, w, rgb[off:off + k], dl[off:off + k]))
            off += k

        def batched():
            sk.render_forward(planes, n, 3, cams, rp, ws, cap, rgb)
            sk.render_backward(planes, n, 3, cams, rp, ws, cap, dl, None, grads)

        def per_view():
            for c, cv, w, out, d in per:
                sk.render_forward(planes, n, 3, [c], rp, w, cv, out)
                sk.render_backward(planes, n, 3, [c], rp, w, cv, d, None, grads)

        def timeit(fn):
            for _ in range(warm):
                fn()
            a, b = ev(), ev()
            torch.cuda.synchronize()
            a.record()
            for _ in range(steps):
                fn()
            b.record()
            torch.cuda.synchronize()
            return a.elapsed_time(b) / steps

        log(f"{tag}: capacity {cap}; timing {steps} steps per mode")
        r = {"per_view_ms": timeit(per_view), "batched_ms": timeit(batched)}
        grads.zero_()
        batched()
        torch.cuda.synchronize()
        ref = rgb.clone()
        cs = torch.cuda.Stream()
        cs.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(cs):
            batched()
        torch.cuda.current_stream().wait_stream(cs)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=cs):
            batched()
        torch.cuda.synchronize()
        for _ in range(3):
            rgb.zero_()
            g.replay()
            torch.cuda.synchronize()
            if not torch.equal(rgb, ref):
                raise RuntimeError("graph replay differs from the eager launch")
        r["graph_ms"] = timeit(g.replay)
        if sk.read_status(ws)[0]:
            raise RuntimeError("status flags set")
        r["capacity"] = cap
        results[tag] = r
        log(f"{tag}: per-view {r['per_view_ms']:.3f} ms, batched {r['batched_ms']:.3f} ms, "
            f"graph {r['graph_ms']:.3f} ms")
        del g, ws, per
        torch.cuda.empty_cache()
    tuned_tag = f"{tuned.tile_w}x{tuned.tile_h}/S{tuned.super_tile}/B{tuned.lds_batch}"
    ms = min(results[tuned_tag]["batched_ms"], results[tuned_tag]["graph_ms"])
    out = {"metric": "batched 8-view forward+backward throughput at 1 GPU", "value": 1000.0 / ms,
           "unit": "batches/s", "n_gpus": 1, "steps": steps, "warmup": warm, "ms_per_step": ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"forward+backward of 8 views (2x 640x480, 1245x825, 1600x1060, "
                                  f"980x545) of {n} Gaussians SH3, one launch",
                      "launch_shape": tuned_tag},
           "tuner": {"choice": record["choice"], "reused": record["reused"],
                     "trials": sorted(record["trials"], key=lambda t: t["ms"])},
           "modes": results}
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    if args.workload == "batched":
        return run_batched(args)
    if args.workload == "single":
        return run_single(args)
    if args.workload == "dense":
        return run_dense(args)
    if args.workload == "densify":
        return run_densify(args)
    if args.workload == "atomics":
        return run_atomics(args)
    if args.steps is None:
        args.steps = 2000
    if args.warmup is None:
        args.warmup = 20
    if args.workload == "matched":
        return run_matched(args)
    return run_train(args)


if __name__ == "__main__":
    main()
