"""Helpers for the rocprofv3 measurements behind the benchmark's roofline.

``python -m paper_2502_17632_amd.profiling copy`` runs a plain device copy of
known size (the calibration of the FETCH_SIZE / WRITE_SIZE counters: the
bytes the counters report for a copy, divided by the bytes it must move).

``python -m paper_2502_17632_amd.profiling summarize ...`` reduces the CSV
files rocprofv3 wrote (kernel statistics or per-dispatch counters) to the
few figures the profile summaries keep.  Neither touches the library.
"""
from __future__ import annotations

import argparse
import csv
import glob
import os
import re
import sys
from collections import defaultdict


def run_copy(mib: int, reps: int):
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {reps} x {n * 4} bytes", flush=True)


def _csv(pattern: str):
    files = sorted(glob.glob(pattern, recursive=True))
    if not files:
        raise FileNotFoundError(pattern)
    rows = []
    for f in files:
        with open(f) as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def counter_per_dispatch(pmc_dir: str, counter: str, kernel_regex: str):
    """Mean, min, max of `counter` summed over each dispatch of the kernels
    whose name matches `kernel_regex`, and the dispatch count."""
    rows = _csv(os.path.join(pmc_dir, "**", "*counter_collection.csv"))
    per = defaultdict(float)
    rx = re.compile(kernel_regex)
    for r in rows:
        if r.get("Counter_Name") != counter or not rx.search(r.get("Kernel_Name", "")):
            continue
        per[r["Dispatch_Id"]] += float(r["Counter_Value"])
    vals = list(per.values())
    if not vals:
        return None
    return {"dispatches": len(vals), "mean": sum(vals) / len(vals), "min": min(vals),
            "max": max(vals)}


def kernel_stats(stats_dir: str, kernel_regex: str):
    rows = _csv(os.path.join(stats_dir, "**", "*kernel_stats.csv"))
    rx = re.compile(kernel_regex)
    out = []
    for r in rows:
        if rx.search(r["Name"]):
            out.append({"name": r["Name"], "calls": int(r["Calls"]),
                        "avg_us": float(r["AverageNs"]) / 1e3,
                        "min_us": float(r["MinNs"]) / 1e3, "max_us": float(r["MaxNs"]) / 1e3,
                        "percent": float(r["Percentage"])})
    return out


def counters_summary(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, kernel_regex,
                     copy_bytes, source, title, commands):
    """Text summary of the HBM traffic of one kernel: its FETCH_SIZE and
    WRITE_SIZE per dispatch (KiB), each scaled by what the counter reads for
    a copy of `copy_bytes` bytes (bytes moved / bytes reported), and the
    sha256 of the kernel's source so that a later change invalidates it."""
    import hashlib
    f = counter_per_dispatch(fetch_dir, "FETCH_SIZE", kernel_regex)
    w = counter_per_dispatch(write_dir, "WRITE_SIZE", kernel_regex)
    cf = counter_per_dispatch(copy_fetch_dir, "FETCH_SIZE", "copyBuffer|copy")
    cw = counter_per_dispatch(copy_write_dir, "WRITE_SIZE", "copyBuffer|copy")
    fs = copy_bytes / (cf["max"] * 1024.0)
    ws = copy_bytes / (cw["max"] * 1024.0)
    traffic = f["mean"] * 1024.0 * fs + w["mean"] * 1024.0 * ws
    sha = hashlib.sha256(open(source, "rb").read()).hexdigest()
    lines = [f"# {title}", "# commands (from the repository root on the GPU host):"]
    lines += [f"#   {c}" for c in commands]
    lines += [
        f"kernel_regex = {kernel_regex}",
        f"source = {os.path.relpath(source, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))}",
        f"filter_hip_sha256 = {sha}",
        f"dispatches = {f['dispatches']}",
        f"fetch_size_kib_per_dispatch = {f['mean']:.2f}",
        f"write_size_kib_per_dispatch = {w['mean']:.2f}",
        f"copy_bytes = {copy_bytes}",
        f"copy_fetch_size_kib = {cf['max']:.2f}",
        f"copy_write_size_kib = {cw['max']:.2f}",
        f"fetch_scale = {fs:.4f}",
        f"write_scale = {ws:.4f}",
        f"fetch_bytes_per_launch = {f['mean'] * 1024.0 * fs:.0f}",
        f"write_bytes_per_launch = {w['mean'] * 1024.0 * ws:.0f}",
        f"traffic_bytes_per_launch = {traffic:.0f}",
    ]
    return "\n".join(lines) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("copy", help="device copy of known size")
    c.add_argument("--mib", type=int, default=512)
    c.add_argument("--reps", type=int, default=5)
    s = sub.add_parser("summarize", help="reduce rocprofv3 CSV output")
    s.add_argument("--pmc-dir")
    s.add_argument("--stats-dir")
    s.add_argument("--counter", default="FETCH_SIZE")
    s.add_argument("--kernel", default=".")
    t = sub.add_parser("traffic", help="write the counter summary of one kernel")
    t.add_argument("--fetch-dir", required=True)
    t.add_argument("--write-dir", required=True)
    t.add_argument("--copy-fetch-dir", required=True)
    t.add_argument("--copy-write-dir", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--copy-mib", type=int, default=512)
    t.add_argument("--source", required=True)
    t.add_argument("--title", required=True)
    t.add_argument("--command", action="append", default=[])
    t.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "traffic":
        text = counters_summary(a.fetch_dir, a.write_dir, a.copy_fetch_dir, a.copy_write_dir,
                                a.kernel, a.copy_mib << 20, a.source, a.title, a.command)
        with open(a.out, "w") as fh:
            fh.write(text)
        print(text)
        return 0
    if a.cmd == "copy":
        run_copy(a.mib, a.reps)
        return 0
    if a.pmc_dir:
        print(a.counter, counter_per_dispatch(a.pmc_dir, a.counter, a.kernel))
    if a.stats_dir:
        for k in kernel_stats(a.stats_dir, a.kernel):
            print(k)
    return 0


if __name__ == "__main__":
    sys.exit(main())
