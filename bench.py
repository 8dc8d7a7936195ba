"""Benchmark: post-densification iterations/s of SkipGS-gated vs full-backward
3DGS training on one MI355X, with the dominant kernel's roofline fraction
and the FP64 oracle timed on the host as a CPU reference.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
    python bench.py --workload batched     # 8 mixed-resolution views per launch

Workload (defaults): 3,000,000 Gaussians (SH degree 3, ground-plane + two
clusters), 200 views at 1600x1060 on a hemisphere of radius 4-5, 16x16 tiles,
targets rendered from the ground-truth set, training from a perturbed copy,
uniform view sampling, loss 0.8 L1 + 0.2 (1 - SSIM), gate with EMA decay 0.9,
skip within 2% of the view's EMA, >= 50% backward per 100 iterations, Adam
(means lr 1.6e-4); 10,000 timed iterations per run (gated, then full). One
step = one training iteration: forward render, loss, gate, and (when the gate
opens) loss backward, render backward and Adam. Inputs are resident in HBM
before the timed region starts.
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
                    help="timed steps (default: 10000 iterations of the training workload, "
                         "20 batches of the batched one)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps first (default: 20 iterations, 2 batches)")
    ap.add_argument("--n", type=int, default=3_000_000)
    ap.add_argument("--views", type=int, default=200)
    ap.add_argument("--width", type=int, default=1600)
    ap.add_argument("--height", type=int, default=1060)
    ap.add_argument("--gate", choices=["windowed", "paper"], default="windowed")
    ap.add_argument("--runs", default="gated,full",
                    help="comma list of gated, full, paper, paper_nobudget")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-stage-events", action="store_true")
    ap.add_argument("--eval-views", type=int, default=200)
    ap.add_argument("--workload", choices=["train", "batched"], default="train",
                    help="train: gated vs full training (the headline); batched: forward + "
                         "backward of 8 mixed-resolution views of 2M Gaussians, per-view "
                         "launches vs one batched launch vs graph replay, per tile shape")
    return ap.parse_args()


def cpu_baseline(gt, init, cam, crop=24):
    """The FP64 oracle on a bounded sample of one iteration: projection of all
    Gaussians (with autograd) plus compositing, loss and backward for a
    crop x crop pixel window at the image centre; the per-pixel part is
    scaled to the full image."""
    from oracle import render as OR, loss as OL
    threads = torch.get_num_threads()
    arr = {k: torch.tensor(np.asarray(v, np.float64), requires_grad=True) for k, v in
           dict(means=init.means, log_scales=init.log_scales, quats=init.quats,
                opacity_logits=init.opacity_logits, sh=init.sh).items()}
    t0 = time.perf_counter()
    pr = OR.project(arr["means"], arr["log_scales"], arr["quats"], arr["opacity_logits"], arr["sh"],
                    init.sh_degree, cam, OR.RasterParams())
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
    t1 = time.perf_counter()
    out = OR.composite(pr["uv"], pr["conic"], pr["opacity"], pr["rgb"], pr["depth"], pr["extent"],
                       pr["ids"], cam.width, cam.height, OR.RasterParams(), px=px, py=py)
    L = OL.photometric_loss(out["rgb"].reshape(3, crop, crop), tgt)
    t_pix = time.perf_counter() - t1
    t2 = time.perf_counter()
    L.backward()
    t_bwd = time.perf_counter() - t2
    scale = (cam.width * cam.height) / float(crop * crop)
    # projection runs once per iteration; compositing and its share of the
    # backward scale with the pixel count
    est = t_proj + (t_pix + t_bwd) * scale
    return {"value": 1.0 / est, "unit": "iters/s", "cores": threads, "kind": "oracle",
            "sample": (f"one view: FP64 projection of all {init.n} Gaussians with autograd "
                       f"({t_proj:.1f} s) + compositing, loss and backward of a {crop}x{crop} "
                       f"window ({t_pix + t_bwd:.1f} s) scaled x{scale:.0f} to the full "
                       f"{cam.width}x{cam.height} view; torch CPU threads={threads}"),
            "seconds_per_iter_estimate": est}


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


def run_batched(args):
    """Forward + backward of eight views of four resolutions (two each of
    640x480, 1245x825, 1600x1060, 980x545) of 2M Gaussians, gradients summed
    over the views: eight single-view launches, one launch of all views, and
    the replay of a captured graph of that launch, for each tile shape."""
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
    results = {}
    for tw, th in ((16, 16), (8, 8), (32, 8)):
        rp = sk.RasterParams(tile_w=tw, tile_h=th)
        # capacities: whole batch and each view, sized by one probe launch
        def capacity(cs):
            ws = sk.alloc_bytes(sk.forward_workspace_size(rp, n, cs, 1 << 16))
            sk.clear_status(ws)
            out = torch.empty(3 * sum(c.width * c.height for c in cs), device="cuda")
            sk.render_forward(planes, n, 3, cs, rp, ws, 1 << 16, out)
            return int(sk.read_status(ws)[2] * 1.02) + 4096
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

        log(f"tiles {tw}x{th}: capacity {cap} pairs; timing {steps} steps per mode")
        r = {"per_view_ms": timeit(per_view), "batched_ms": timeit(batched)}
        # graph of the batched launch, replayed; the first replay's image must
        # equal the eager one
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
        flags = sk.read_status(ws)[0]
        if flags:
            raise RuntimeError(f"status flags {flags}")
        r["pairs"] = cap
        results[f"{tw}x{th}"] = r
        log(f"tiles {tw}x{th}: per-view {r['per_view_ms']:.3f} ms, batched {r['batched_ms']:.3f} ms, "
            f"graph {r['graph_ms']:.3f} ms")
        del g, ws, per
        torch.cuda.empty_cache()
    best = min(results, key=lambda k: min(results[k]["batched_ms"], results[k]["graph_ms"]))
    ms = min(results[best]["batched_ms"], results[best]["graph_ms"])
    out = {"metric": "batched 8-view forward+backward throughput at 1 GPU", "value": 1000.0 / ms,
           "unit": "batches/s", "n_gpus": 1, "steps": steps, "warmup": warm, "ms_per_step": ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"forward+backward of 8 views (2x 640x480, 1245x825, 1600x1060, "
                                  f"980x545) of {n} Gaussians SH3, one launch", "best_tiles": best},
           "modes": results}
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the sharding design is in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batched":
        torch.cuda.set_device(0)
        return run_batched(args)
    if args.steps is None:
        args.steps = 10000
    if args.warmup is None:
        args.warmup = 20
    from paper_2603_08997_amd import scenes as S
    from paper_2603_08997_amd import skipgs as sk
    from paper_2603_08997_amd.train import StageTimer, Trainer, measure_pairs, render_targets

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t_setup = time.perf_counter()
    log(f"setup: scene n={args.n} views={args.views} {args.width}x{args.height}")
    gt = S.mixture_scene(S.SEED_SCENE, args.n, sh_degree=3)
    init = S.perturb(gt, S.SEED_INIT_PERTURB)
    cams = S.hemisphere_cameras(S.SEED_CAMERAS, args.views, args.width, args.height)
    seq = S.view_sequence(S.SEED_VIEW_SEQUENCE, args.views, args.warmup + args.steps)
    rp = sk.RasterParams()
    pairs = max(measure_pairs(gt, cams, rp), measure_pairs(init, cams, rp))
    cap = int(pairs * 1.3) + 4096
    log(f"setup: max pairs per view {pairs}, capacity {cap}")
    targets = render_targets(gt, cams, rp, cap)
    torch.cuda.synchronize()
    log(f"setup done in {time.perf_counter() - t_setup:.1f} s")
    gate = sk.windowed_gate(args.views) if args.gate == "windowed" else sk.paper_gate(args.views)
    eval_views = list(range(min(args.views, args.eval_views)))

    results = {}
    for run in args.runs.split(","):
        if run not in ("gated", "full", "paper", "paper_nobudget"):
            raise SystemExit(f"unknown run {run!r} (gated, full, paper, paper_nobudget)")
        # paper: the gate with the paper's own settings (decay 0.95, no
        # tolerance, 500 warmup iterations, calibrated cumulative budget);
        # paper_nobudget: the same without the minimum-backward budget (the
        # "w/o budget" row of the paper's ablation, Table 4)
        if run == "paper":
            gp = sk.paper_gate(args.views)
        elif run == "paper_nobudget":
            gp = dataclasses.replace(sk.paper_gate(args.views), budget=False)
        else:
            gp = gate
        tr = Trainer(init, cams, targets, rp, gp, cap, gated=(run != "full"))
        gslots = torch.zeros(args.warmup + args.steps, dtype=torch.int32, device=dev)
        for t in range(args.warmup):
            tr.iteration(int(seq[t]), gslots[t:t + 1])
        timer = None if args.no_stage_events else StageTimer()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for t in range(args.warmup, args.warmup + args.steps):
            tr.iteration(int(seq[t]), gslots[t:t + 1], timer=timer)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        flags, vis, _ = tr.status()
        if flags & sk.STATUS_PAIR_OVERFLOW:
            raise RuntimeError("pair capacity overflow during the timed run")
        g = gslots[args.warmup:].cpu().numpy()
        res = {"iters_per_s": args.steps / dt, "ms_per_step": 1000 * dt / args.steps,
               "backward_fraction": float(g.mean()), "seconds": dt}
        if timer is not None:
            res["stage_ms_all"] = timer.summary()
            res["stage_ms_executed"] = timer.summary(mask=g == 1)
            res["stage_ms_skipped"] = timer.summary(mask=g == 0) if (g == 0).any() else None
        log(f"{run}: {res['iters_per_s']:.1f} it/s, backward fraction {res['backward_fraction']:.3f}")
        res["final_mean_loss"] = tr.mean_loss(eval_views)
        log(f"{run}: final mean loss over {len(eval_views)} views {res['final_mean_loss']:.6f}")
        results[run] = res
        res["_trainer"] = tr
        res["_timer"] = timer

    gated = results.get("gated")
    full = results.get("full")
    headline = gated or full

    # dominant kernel: of the compositing forward, the compositing backward
    # and the fused projection backward + Adam, the one with the largest
    # time per iteration in the headline run (backward kernels weighted by
    # the fraction of iterations that run them)
    roof = None
    tr = headline["_trainer"]
    timer = headline["_timer"]
    if timer is not None:
        # per-view counters, averaged over 8 views
        blended, evaluated, pairs, visible = [], [], [], []
        for v in range(min(8, args.views)):
            tr.render(v, tr.rgb)
            torch.cuda.synchronize()
            cnt = sk.read_counters(tr.ws)
            blended.append(cnt["blended"])
            evaluated.append(cnt["evaluated"])
            pairs.append(cnt["pairs"])
            visible.append(cnt["visible"])
        blended = float(np.mean(blended))
        vis = float(np.mean(visible))
        ex = headline["stage_ms_executed"]
        allm = headline["stage_ms_all"]
        bf = headline["backward_fraction"]
        F = 11 + 3 * 16
        # algorithmic HBM bytes of one fused launch: parameters, first and
        # second moments read and written once per plane of every Gaussian,
        # the visibility word of every Gaussian, and the 48-byte gradient
        # accumulator plus the 16-byte colour record of every visible one
        fused_bytes = args.n * (F * 4 * 6 + 4) + vis * (48 + 16)
        cands = {
            "raster_forward": dict(ms=allm["rasterize"], weight=1.0, bound="alu",
                                   work=blended * FWD_FLOPS_PER_PAIR / 1e12, unit="TFLOP/s",
                                   peak=FP32_VECTOR_PEAK_TFLOPS),
            "raster_backward": dict(ms=ex["raster_bwd"], weight=bf, bound="alu",
                                    work=blended * BWD_FLOPS_PER_PAIR / 1e12, unit="TFLOP/s",
                                    peak=FP32_VECTOR_PEAK_TFLOPS),
            "project_backward_adam": dict(ms=ex["project_bwd"], weight=bf, bound="hbm",
                                          work=fused_bytes / 1e9, unit="GB/s",
                                          peak=HBM_PEAK_GBS),
        }
        summary = {}
        for k, c in cands.items():
            ach = c["work"] / (c["ms"] * 1e-3) if c["ms"] > 0 else 0.0
            summary[k] = {"avg_launch_ms": c["ms"], "ms_per_iteration": c["ms"] * c["weight"],
                          "bound": c["bound"], "achieved": ach, "unit": c["unit"],
                          "frac": ach / c["peak"]}
        name = max(summary, key=lambda k: summary[k]["ms_per_iteration"])
        c, sm = cands[name], summary[name]
        traffic = None
        if (args.n, args.width, args.height) == (3_000_000, 1600, 1060):
            from paper_2603_08997_amd.profiling import load_traffic
            rec = load_traffic(TRAFFIC_FILE)
            if rec is not None and name in rec["kernels"]:
                traffic = rec["kernels"][name]["traffic_bytes"]
        roof = {"kernel": name, "bound": c["bound"], "achieved": sm["achieved"], "peak": c["peak"],
                "unit": c["unit"], "frac": sm["frac"], "traffic": traffic,
                "avg_launch_ms": c["ms"], "blended_pairs_per_launch": blended,
                "evaluated_pairs_per_launch": float(np.mean(evaluated)),
                "tile_pairs_per_view": float(np.mean(pairs)), "visible_per_view": vis,
                "fused_bytes_per_launch": fused_bytes,
                "flops_per_pair": {"forward": FWD_FLOPS_PER_PAIR, "backward": BWD_FLOPS_PER_PAIR},
                "kernels": summary}

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
        "config": {"workload": (f"gated 3DGS post-densification training, {args.n} Gaussians SH3, "
                                f"{args.views} views {args.width}x{args.height}, 16x16 tiles, "
                                f"{args.gate} gate"),
                   "gaussians": args.n, "views": args.views, "width": args.width,
                   "height": args.height, "gate": args.gate},
    }
    if gated and full:
        out["full_iters_per_s"] = full["iters_per_s"]
        out["gated_over_full"] = gated["iters_per_s"] / full["iters_per_s"]
        out["skip_fraction"] = 1.0 - gated["backward_fraction"]
        out["final_loss_gated"] = gated["final_mean_loss"]
        out["final_loss_full"] = full["final_mean_loss"]
        out["final_loss_rel_diff"] = (gated["final_mean_loss"] - full["final_mean_loss"]) / \
            full["final_mean_loss"]
        if gated.get("stage_ms_skipped") and full.get("stage_ms_all"):
            c = sum(gated["stage_ms_skipped"].values()) / sum(full["stage_ms_all"].values())
            out["skipped_iteration_cost"] = c
    for name in ("paper", "paper_nobudget"):
        r = results.get(name)
        if not r:
            continue
        out[f"{name}_iters_per_s"] = r["iters_per_s"]
        out[f"{name}_skip_fraction"] = 1.0 - r["backward_fraction"]
        out[f"final_loss_{name}"] = r["final_mean_loss"]
        if full:
            out[f"{name}_over_full"] = r["iters_per_s"] / full["iters_per_s"]
            out[f"final_loss_{name}_rel_diff"] = (r["final_mean_loss"] -
                                                  full["final_mean_loss"]) / full["final_mean_loss"]
    for k, r in results.items():
        out[f"stages_{k}"] = {kk: (round(vv, 4) if isinstance(vv, float) else vv)
                              for kk, vv in r.get("stage_ms_executed", {}).items()}
    if roof is not None:
        out["roofline"] = roof
    out["hbm_copy_GBps"] = hbm_copy_probe()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(gt, init, cams[0])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
