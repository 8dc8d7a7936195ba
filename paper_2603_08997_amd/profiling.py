"""Summaries of rocprofv3 output for the kernel profiles kept with the
sources, and the measured HBM traffic the benchmark reports.

    # per-iteration kernel table from a kernel trace (--kernel-trace --stats -f csv)
    python -m paper_2603_08997_amd.profiling kernels DIR --title T --command C --out FILE

    # HBM bytes per dispatch from two counter runs (--pmc FETCH_SIZE, --pmc WRITE_SIZE),
    # scaled by what the same counters read for a copy of known size
    python -m paper_2603_08997_amd.profiling traffic FETCH_DIR WRITE_DIR --copy-bytes B \\
        --command C --out FILE

The traffic file records a digest of the sources the kernels are built
from; the benchmark reports the traffic only while that digest matches.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import re
import statistics

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)

# Kernels whose traffic the benchmark may report: the benchmark's name for
# each, and the start of the name the trace shows.
TRAFFIC_KERNELS = {"project_backward_adam": "project_backward_adam_kernel",
                   "raster_backward": "raster_backward_kernel",
                   "raster_forward": "raster_forward_kernel",
                   "emit": "emit_kernel",
                   "split_count": "split_count_kernel",
                   "split_write": "split_write_kernel"}
COPY_KERNEL = "MulFunctor"


def source_digest() -> str:
    """sha256 over the kernel sources, the public header and the build flags."""
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(PKG, "csrc", "*"))) + [
        os.path.join(ROOT, "include", "skipgs.h"), os.path.join(PKG, "build.py")]
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def short_name(n: str) -> str:
    n = n.replace("void ", "").replace("sgs::(anonymous namespace)::", "")
    return n.split("(")[0]


def _rows(path):
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def kernels_table(d: str, iterations: int = 40, marker: str = "project_kernel",
                  require: str = "raster_backward") -> str:
    """Markdown table: time per iteration of each kernel over the last
    `iterations` iterations of the trace that launch `require` (an iteration
    starts at each launch of `marker`; iterations without `require`, such as
    evaluation renders, are left out), then rocprofv3's own per-kernel
    statistics."""
    trace = sorted(_rows(os.path.join(d, "run_kernel_trace.csv")),
                   key=lambda r: int(r["Start_Timestamp"]))
    names = [short_name(r["Kernel_Name"]) for r in trace]
    starts = [i for i, n in enumerate(names) if n.startswith(marker)] + [len(trace)]
    spans = [(a, b) for a, b in zip(starts, starts[1:])
             if any(names[i].startswith(require) for i in range(a, b))]
    if len(spans) < iterations:
        raise SystemExit("trace too short for the requested iterations")
    spans = spans[-iterations:]
    agg = collections.defaultdict(list)
    wall = 0.0
    for a, b in spans:
        for r, n in zip(trace[a:b], names[a:b]):
            agg[n].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
        last = max(i for i in range(a, b) if not names[i].startswith("__amd"))
        wall += (int(trace[last]["End_Timestamp"]) - int(trace[a]["Start_Timestamp"])) / 1e3
    out = ["| kernel | us/iter | launches/iter | us/launch |", "|---|---|---|---|"]
    tot = 0.0
    for n, v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        per = sum(v) / iterations
        tot += per
        if per >= 1.0:
            out.append(f"| `{n}` | {per:.1f} | {len(v) / iterations:.1f} | {sum(v) / len(v):.1f} |")
    out.append(f"| **sum of kernel time** | {tot:.1f} | | |")
    out.append(f"| **first kernel start to last kernel end, per iteration** | "
               f"{wall / iterations:.1f} | | |")
    out += ["", "rocprofv3 statistics over the whole run (all dispatches, setup included):", "",
            "| kernel | calls | average us | min us | max us |", "|---|---|---|---|---|"]
    stats = _rows(os.path.join(d, "run_kernel_stats.csv"))
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:16]:
        out.append(f"| `{short_name(r['Name'])}` | {r['Calls']} | "
                   f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                   f"{float(r['MaxNs']) / 1e3:.1f} |")
    return "\n".join(out)


def _counter_means(d: str, counter: str) -> dict:
    vals = collections.defaultdict(list)
    for r in _rows(os.path.join(d, "run_counter_collection.csv")):
        if r["Counter_Name"] != counter:
            continue
        n = r["Kernel_Name"]
        key = COPY_KERNEL if COPY_KERNEL in n else short_name(n)
        if key == COPY_KERNEL:
            key = f"{COPY_KERNEL}:{r['Grid_Size']}"
        vals[key].append(float(r["Counter_Value"]))
    return {k: statistics.mean(v) for k, v in vals.items()}


def traffic(fetch_dir: str, write_dir: str, copy_bytes: int) -> dict:
    """Per-dispatch HBM bytes of the kernels in TRAFFIC_KERNELS: the mean
    FETCH_SIZE and WRITE_SIZE (KiB) of their dispatches, each scaled by the
    ratio of the known bytes a plain copy moves to what the same counter reads
    for it (the copy reads and writes copy_bytes)."""
    fetch = _counter_means(fetch_dir, "FETCH_SIZE")
    write = _counter_means(write_dir, "WRITE_SIZE")
    copies = [k for k in fetch if k.startswith(COPY_KERNEL)]
    if not copies:
        raise SystemExit("no copy kernel dispatches in the counter runs")
    ck = max(copies, key=lambda k: int(k.split(":")[1]))
    f_fetch = copy_bytes / (fetch[ck] * 1024.0)
    f_write = copy_bytes / (write[ck] * 1024.0)
    out = {"copy_kernel_fetch_kib": fetch[ck], "copy_kernel_write_kib": write[ck],
           "copy_bytes": copy_bytes, "fetch_scale": f_fetch, "write_scale": f_write,
           "kernels": {}}
    for k, prefix in TRAFFIC_KERNELS.items():
        m = [n for n in fetch if n.startswith(prefix)]
        if not m:
            continue
        n = m[0]
        fb = fetch[n] * 1024.0 * f_fetch
        wb = write.get(n, 0.0) * 1024.0 * f_write
        out["kernels"][k] = {"name": n, "fetch_kib": fetch[n], "write_kib": write.get(n, 0.0),
                             "fetch_bytes": fb, "write_bytes": wb, "traffic_bytes": fb + wb}
    return out


def issue(pmc_dir: str, trace_dir: str | None, simds: int, clock_ghz: float) -> dict:
    """VALU issue utilisation per kernel from a counter run (SQ_INSTS_VALU ...):
    sum of VALU instructions x 4 cycles (a wave64 instruction on a 16-lane SIMD)
    / sum of (duration x clock x SIMDs). Durations are the counter run's own
    dispatch timestamps, or, with `trace_dir`, those of a kernel trace of the
    same command (the k-th launch of each kernel in both)."""
    counts = collections.defaultdict(list)
    durs = collections.defaultdict(list)
    seen = set()
    for r in sorted(_rows(os.path.join(pmc_dir, "run_counter_collection.csv")),
                    key=lambda r: int(r["Dispatch_Id"])):
        name = short_name(r["Kernel_Name"])
        counts[(name, r["Counter_Name"])].append(float(r["Counter_Value"]))
        if trace_dir is None and r["Dispatch_Id"] not in seen:
            seen.add(r["Dispatch_Id"])
            durs[name].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9)
    if trace_dir is not None:
        for r in sorted(_rows(os.path.join(trace_dir, "run_kernel_trace.csv")),
                        key=lambda r: int(r["Start_Timestamp"])):
            durs[short_name(r["Kernel_Name"])].append(
                (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9)
    out = {}
    for (name, ctr), vals in counts.items():
        if ctr != "SQ_INSTS_VALU" or name not in durs:
            continue
        k = min(len(vals), len(durs[name]))
        busy = sum(durs[name][:k]) * clock_ghz * 1e9 * simds
        rec = {"dispatches": k, "valu_instructions_per_dispatch": sum(vals[:k]) / k,
               "seconds_per_dispatch": sum(durs[name][:k]) / k,
               "valu_issue_utilisation": sum(vals[:k]) * 4 / busy}
        for other in ("SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM"):
            if (name, other) in counts:
                rec[other.lower() + "_per_dispatch"] = sum(counts[(name, other)][:k]) / k
        out[name] = rec
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    k = sub.add_parser("kernels")
    k.add_argument("dir")
    k.add_argument("--title", required=True)
    k.add_argument("--about", default="")
    k.add_argument("--command", required=True)
    k.add_argument("--iterations", type=int, default=40)
    k.add_argument("--out", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("fetch_dir")
    t.add_argument("write_dir")
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--command", required=True)
    t.add_argument("--out", required=True)
    i = sub.add_parser("issue")
    i.add_argument("pmc_dir")
    i.add_argument("--trace-dir", default=None)
    i.add_argument("--simds", type=int, default=1024)
    i.add_argument("--clock-ghz", type=float, default=2.4)
    i.add_argument("--command", required=True)
    i.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "issue":
        res = issue(a.pmc_dir, a.trace_dir, a.simds, a.clock_ghz)
        lines = [f"{k}: {v['valu_issue_utilisation']:.1%} VALU issue over {v['dispatches']} "
                 f"dispatches ({v['valu_instructions_per_dispatch'] / 1e6:.1f}M VALU "
                 f"instructions, {v['seconds_per_dispatch'] * 1e6:.1f} us each)"
                 for k, v in sorted(res.items())]
        text = ("VALU issue utilisation (rocprofv3 SQ_INSTS_VALU per dispatch over the "
                "dispatch's duration; wave64 VALU = 4 cycles on a 16-lane SIMD, "
                f"{a.simds} SIMDs at {a.clock_ghz} GHz)\n\n" + "\n".join(lines) +
                "\n\nCommand (repository root, one MI355X):\n\n    " + a.command + "\n\n" +
                f"Source digest: `{source_digest()}`\n\n" + json.dumps(res, indent=1) + "\n")
        with open(a.out, "w") as fh:
            fh.write(text)
        print(text)
        return
    if a.cmd == "kernels":
        body = kernels_table(a.dir, a.iterations)
        text = (f"# {a.title}\n\n{a.about}\n\nCommand (repository root, one MI355X):\n\n"
                f"    {a.command}\n\nSource digest: `{source_digest()}`\n\n{body}\n")
    else:
        res = traffic(a.fetch_dir, a.write_dir, a.copy_bytes)
        res["source_digest"] = source_digest()
        res["command"] = a.command
        lines = [f"{k}: fetch {v['fetch_bytes'] / 1e9:.3f} GB + write {v['write_bytes'] / 1e9:.3f}"
                 f" GB = {v['traffic_bytes'] / 1e9:.3f} GB per dispatch"
                 for k, v in res["kernels"].items()]
        text = ("HBM traffic per dispatch (rocprofv3 FETCH_SIZE and WRITE_SIZE, scaled by a copy "
                "of known size)\n\n" + "\n".join(lines) + "\n\n" + json.dumps(res, indent=1) + "\n")
    with open(a.out, "w") as fh:
        fh.write(text)
    print(text)


def load_traffic(path: str) -> dict | None:
    """The traffic record in `path` if its source digest matches the current
    sources, else None."""
    try:
        with open(path) as fh:
            text = fh.read()
    except OSError:
        return None
    m = re.search(r"\{.*\}", text, re.S)
    if not m:
        return None
    rec = json.loads(m.group(0))
    return rec if rec.get("source_digest") == source_digest() else None


if __name__ == "__main__":
    main()
