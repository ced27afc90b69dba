#!/usr/bin/env python3
"""Benchmark of the GiFt hot path on one MI355X.

One step = the whole hot path on the large synthetic workload (2,000,000
movable + 20,000 fixed cells, 2,100,000 nets, pins 2 + Zipf(2.2) capped at
1000, 90% index-local; nets above 16 cells star-expanded): netlist -> graph
build (dedupe, expansion, CSR sort/merge, degrees, normalisation) and the
multi-order filter (sigma 4, orders 1, 2, 4, 8, 16, equal weights, 2 signal
columns, float32 storage).  The netlist and the signal are resident in HBM
before the timed region starts.

Prints one JSON line.  ``value`` is filter work per second of whole step:
sum over the 16 SpMM passes of (stored entries + diagonal) x columns,
divided by the step time.  The roofline object describes the dominant
kernel, the non-final SpMM pass, timed per launch with HIP events on its own
stream by the library's profiler during the timed steps.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "filter nnz·cols/s + achieved HBM GB/s vs peak; p50/p99 request latency"
COUNTERS = os.path.join(ROOT, "profiles", "spmm_large_f32_counters.txt")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def host_cpu():
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def counter_traffic():
    """HBM bytes per SpMM launch measured with rocprofv3 counters, if they were
    taken on the current kernel source."""
    src = os.path.join(ROOT, "paper_2502_17632_amd", "csrc", "filter.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    try:
        kv = {}
        for line in open(COUNTERS):
            if "=" in line and not line.startswith("#"):
                k, v = line.strip().split("=", 1)
                kv[k.strip()] = v.strip()
        if kv.get("filter_hip_sha256") == sha:
            return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        pass
    return None


def filter_work(info, passes, cols):
    """(nnz + R) * cols for every pass but the last, (nnz_cells + N) * cols for
    the last one (which computes the cell rows only)."""
    full = (info["nnz"] + info["num_rows"]) * cols
    return full * (passes - 1) + (info["nnz_cells"] + info["num_cells"]) * cols


def filter_bytes(nnz, rows, nnz_cells, cells, cols, passes, num_terms, storage):
    """Algorithmic bytes of the whole filter: per pass row_ptr, col and values
    of the rows it covers, their diagonal, every signal row read once and the
    rows written; the last pass reads the saved iterates of the other terms
    and writes the float32 output instead of an iterate."""
    bt = {"f32": 4, "bf16": 2, "f16": 2, "f64": 8}[storage]
    ba = 8 if storage == "f64" else 4

    def one(r, z, fin):
        b = 4 * (r + 1) + (4 + bt) * z + ba * r + bt * cols * rows
        if not fin:
            return b + bt * cols * r
        return b + (num_terms - 1) * bt * cols * r + 4 * cols * r
    return one(rows, nnz, False) * (passes - 1) + one(cells, nnz_cells, True)


def bench_batched(gift, W, torch, storage, reps=10):
    """64 designs (log-uniform 10k-300k movable cells, the medium generator,
    per-design seeds), 8 columns each (4 placements), sigma 4, orders
    1, 2, 4, 8, equal weights: the per-design path (64 filter calls) against
    one tuned batch replaying its captured launch sequence."""
    import numpy as np
    orders = [1, 2, 4, 8]
    terms = ([4.0] * 4, orders, [0.25] * 4)
    sizes = W.batch_sizes(64)
    log(f"[bench] batched {storage}: generating 64 designs")
    nls = [W.sized(n, seed=1000 + i) for i, n in enumerate(sizes)]
    xs = [torch.tensor(W.make_signal(nl, W.BATCH_NOISE, seed=1000 + i), dtype=torch.float32,
                       device="cuda") for i, nl in enumerate(nls)]
    graphs = [gift.build_graph(nl.num_cells, nl.net_ptr, nl.pin_cell, star_threshold=16,
                               storage=storage, sigmas=[4.0]) for nl in nls]
    infos = [g.info() for g in graphs]
    nnz_cells = 0
    for g, nl in zip(graphs, nls):
        rp, _, _, _ = g.export()
        nnz_cells += int(rp[nl.num_cells])
    nnz = sum(i["nnz"] for i in infos)
    rows = sum(i["num_rows"] for i in infos)
    cells = sum(i["num_cells"] for i in infos)
    work = ((nnz + rows) * (max(orders) - 1) + (nnz_cells + cells)) * 8
    nbytes = filter_bytes(nnz, rows, nnz_cells, cells, 8, max(orders), len(orders), storage)
    torch.cuda.synchronize()

    def timed(fn):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / reps
        return e0.elapsed_time(e1) / reps, wall

    ys_alone = [torch.empty_like(x) for x in xs]

    def alone():
        for g, x, y in zip(graphs, xs, ys_alone):
            gift.filter_placement(g, *terms, x, out=y)
    ms_alone, wall_alone = timed(alone)

    t0 = time.perf_counter()
    b = gift.Batch(graphs, *terms, num_cols=8, tune=1)
    create_s = time.perf_counter() - t0
    ys = [torch.empty_like(x) for x in xs]
    ms_batch, wall_batch = timed(lambda: b.run(xs, ys))
    torch.cuda.synchronize()
    worst = 0.0
    for y, a in zip(ys, ys_alone):
        den = a.abs().amax(dim=0).clamp_min(1e-30)
        worst = max(worst, float(((y - a).abs().amax(dim=0) / den).max()))
    info = b.info()
    b.close()
    for g in graphs:
        g.close()
    return {
        "workload": "64 designs, log-uniform 10k-300k movable cells (medium generator, seeds "
                    "1000+i), 8 columns, sigma 4, orders 1,2,4,8, equal weights",
        "storage": storage, "cells": cells, "rows": rows, "nnz": nnz,
        "per_design_ms": round(ms_alone, 4), "per_design_wall_ms": round(wall_alone, 4),
        "batched_ms": round(ms_batch, 4), "batched_wall_ms": round(wall_batch, 4),
        "speedup": round(ms_alone / ms_batch, 3),
        "batched_nnz_cols_per_s": work / (ms_batch * 1e-3),
        "per_design_nnz_cols_per_s": work / (ms_alone * 1e-3),
        "batched_algorithmic_GBs": round(nbytes / (ms_batch * 1e-3) / 1e9, 1),
        "max_normwise_diff_vs_per_design": worst,
        "schedule": {"tile_class": info["tile_class"], "chunk_cols": info["chunk_cols"],
                     "tuned": info["tuned"], "tune_s": round(create_s, 3),
                     "candidates": [(c["tile_class"], c["chunk_cols"], round(c["ms"], 4))
                                    for c in info["candidates"]]},
    }


def bench_serving(gift, W, torch, n_requests=1000, pool=24, load=0.7):
    """Poisson stream of filter requests (2 columns, sigma 4, orders 1, 2, 4, 8)
    over a pool of designs with log-uniform 5k-2M movable cells: serial
    per-request execution (build on first use, filter, wait) against the
    serving engine, both from an empty graph cache, at an offered load of
    `load` times the measured serial capacity.  Latency is measured from each
    request's arrival time to its completion on the device."""
    import numpy as np
    terms = ([4.0] * 4, [1, 2, 4, 8], [0.25] * 4)
    sizes = W.serving_sizes(pool)
    log(f"[bench] serving: generating {pool} designs")
    nls = [W.sized(n, seed=5000 + i) for i, n in enumerate(sizes)]
    xs = [torch.tensor(W.make_signal(nl, seed=5000 + i), dtype=torch.float32, device="cuda")
          for i, nl in enumerate(nls)]
    design_of = np.random.default_rng(4244).integers(0, pool, size=n_requests)
    torch.cuda.synchronize()

    def wait_until(t):
        while True:
            d = t - time.perf_counter()
            if d <= 0:
                return
            if d > 2e-3:
                time.sleep(d - 1e-3)

    def serial(arrivals):
        cache, outs, lat = {}, [], []
        t0 = time.perf_counter()
        for j, d in enumerate(design_of):
            ta = t0 + arrivals[j] if arrivals is not None else time.perf_counter()
            if arrivals is not None:
                wait_until(ta)
            g = cache.get(d)
            if g is None:
                nl = nls[d]
                g = cache[d] = gift.build_graph(nl.num_cells, nl.net_ptr, nl.pin_cell,
                                                star_threshold=16, sigmas=[4.0])
            outs.append(gift.filter_placement(g, *terms, xs[d]))
            torch.cuda.synchronize()
            lat.append((time.perf_counter() - ta) * 1e3)
        span = time.perf_counter() - t0
        for g in cache.values():
            g.close()
        torch.cuda.synchronize()
        return np.array(lat), span, outs

    log(f"[bench] serving: serial capacity ({n_requests} requests back to back)")
    _, busy, _ = serial(None)
    rate = load * n_requests / busy
    arrivals = W.poisson_arrivals(n_requests, rate)
    log(f"[bench] serving: serial at {rate:.0f} requests/s")
    lat_s, span_s, outs_s = serial(arrivals)

    def served(arrivals):
        srv = gift.Server(*terms, num_cols=2, hbm_budget_bytes=200 << 30, max_inflight=64,
                          num_streams=4, num_builders=2, max_batch=32)
        t0 = time.perf_counter()
        subs = []
        for j, d in enumerate(design_of):
            ta = t0 + arrivals[j] if arrivals is not None else time.perf_counter()
            if arrivals is not None:
                wait_until(ta)
            nl = nls[d]
            lag = (time.perf_counter() - ta) * 1e3
            t, y = srv.submit(int(d), nl.num_cells, nl.net_ptr, nl.pin_cell, xs[d])
            subs.append((t, y, lag))
        lat = np.array([lag + srv.wait(t)["latency_ms"] for t, _, lag in subs])
        span = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        return lat, span, [y for _, y, _ in subs], st

    log("[bench] serving: engine")
    lat_v, span_v, outs_v, st = served(arrivals)
    same = all(torch.equal(a, b) for a, b in zip(outs_s, outs_v))
    log("[bench] serving: engine, all requests at once")
    _, span_sat, outs_sat, st_sat = served(None)
    same = same and all(torch.equal(a, b) for a, b in zip(outs_s, outs_sat))

    def summary(lat, span):
        return {"p50_ms": round(float(np.percentile(lat, 50)), 3),
                "p99_ms": round(float(np.percentile(lat, 99)), 3),
                "mean_ms": round(float(lat.mean()), 3), "makespan_s": round(span, 3),
                "throughput_rps": round(n_requests / span, 1)}
    return {
        "workload": f"{n_requests} requests, Poisson arrivals (seed 4242) at {load} x serial "
                    f"capacity, over {pool} designs with log-uniform 5k-2M movable cells "
                    "(medium generator, seeds 5000+i), 2 columns, sigma 4, orders 1,2,4,8",
        "rate_rps": round(rate, 1), "serial_capacity_rps": round(n_requests / busy, 1),
        "serial": summary(lat_s, span_s), "served": summary(lat_v, span_v),
        "served_batches": st["batches"],
        "served_mean_batch": round(st["batched_requests"] / max(st["batches"], 1), 2),
        "builds": st["builds"], "evictions": st["evictions"],
        "saturated": {"serial_throughput_rps": round(n_requests / busy, 1),
                      "served_throughput_rps": round(n_requests / span_sat, 1),
                      "served_mean_batch": round(st_sat["batched_requests"] /
                                                 max(st_sat["batches"], 1), 2)},
        "results_equal_to_serial": bool(same),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--storage", default="f32", choices=["f32", "bf16", "f16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the extra measurements")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path "
              f"(--gpus {args.gpus} requested)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2502_17632_amd as gift
    from paper_2502_17632_amd import workload as W

    torch.cuda.set_device(0)
    orders = [1, 2, 4, 8, 16]
    terms = ([4.0] * len(orders), orders, [1.0 / len(orders)] * len(orders))
    thr = 16
    log("[bench] generating the large workload")
    nl = W.large()
    x_host = W.make_signal(nl)
    net_ptr = torch.tensor(nl.net_ptr, device="cuda")
    pin_cell = torch.tensor(nl.pin_cell, device="cuda")
    x = torch.tensor(x_host, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()

    def step():
        g = gift.build_graph(nl.num_cells, net_ptr, pin_cell, star_threshold=thr,
                             storage=args.storage, sigmas=[4.0])
        gift.filter_placement(g, *terms, x, out=y)
        info = g.info()
        g.close()
        return info

    log("[bench] warmup")
    info = None
    for _ in range(args.warmup):
        info = step()
    torch.cuda.synchronize()
    if info is None:
        info = step()
        torch.cuda.synchronize()
    info["nnz_cells"] = None
    # nnz of the cell rows: from the exported row pointer of one graph
    g = gift.build_graph(nl.num_cells, net_ptr, pin_cell, star_threshold=thr,
                         storage=args.storage, sigmas=[4.0])
    row_ptr, _, _, _ = g.export()
    info["nnz_cells"] = int(row_ptr[nl.num_cells])

    log(f"[bench] timing {args.steps} steps")
    gift.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    spmm = gift.profile_collect("spmm")
    fin = gift.profile_collect("spmm_final")
    bld = gift.profile_collect("build")
    gift.profile_enable(False)
    ms_step = (t1 - t0) * 1e3 / args.steps
    work = filter_work(info, max(orders), 2)
    value = work / (ms_step * 1e-3)
    avg_ms = spmm["total_ms"] / max(spmm["launches"], 1)
    bytes_launch = spmm["bytes"] / max(spmm["launches"], 1)
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
    traffic = counter_traffic()
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "kernel": "k_spmm (non-final pass)",
                "bytes_per_launch": bytes_launch, "avg_launch_us": round(avg_ms * 1e3, 2),
                "launches": spmm["launches"]}

    out = {
        "metric": METRIC, "value": value, "unit": "nnz·cols/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.storage, "data": "synthetic",
        "config": {"workload": "large: 2M+20k cells, 2.1M nets, Zipf(2.2) pins <= 1000, "
                               "90% local; star above 16 cells; sigma 4, orders 1,2,4,8,16, "
                               "equal weights; 2 columns",
                   "cells": nl.num_cells, "nets": nl.num_nets, "rows": info["num_rows"],
                   "nnz": info["nnz"], "cols": 2, "storage": args.storage,
                   "passes": max(orders)},
        "roofline": roofline,
        "breakdown": {
            "build_ms": round(bld["total_ms"] / max(bld["launches"], 1), 4),
            "filter_final_pass_us": round(fin["total_ms"] / max(fin["launches"], 1) * 1e3, 2),
            "spmm_pass_us": round(avg_ms * 1e3, 2),
        },
    }

    if not args.no_extra:
        # the filter alone on a resident graph
        for _ in range(3):
            gift.filter_placement(g, *terms, x, out=y)
        torch.cuda.synchronize()
        reps = 20
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(reps):
            gift.filter_placement(g, *terms, x, out=y)
        ev1.record()
        torch.cuda.synchronize()
        f_ms = ev0.elapsed_time(ev1) / reps
        out["filter_only"] = {"ms": round(f_ms, 4), "nnz_cols_per_s": work / (f_ms * 1e-3)}
        # what the filter does to the placement: smoothness / quadratic
        # wirelength, Rayleigh quotient and HPWL before and after
        t0 = time.perf_counter()
        m0 = gift.evaluate_placement(g, x, net_ptr, pin_cell)
        ev_ms = (time.perf_counter() - t0) * 1e3
        m1 = gift.evaluate_placement(g, y, net_ptr, pin_cell)
        # the exact filter (I + L~_4)^-1 g that the paper's filter approximates
        for _ in range(2):
            gift.filter_exact(g, 4.0, x, tol=1e-6)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ye, its = gift.filter_exact(g, 4.0, x, tol=1e-6)
        ex_ms = (time.perf_counter() - t0) * 1e3
        out["exact_filter"] = {"sigma": 4.0, "tol": 1e-6, "iterations": its,
                               "ms": round(ex_ms, 3)}
        box = (0.0, 0.0, W.DIE, W.DIE)
        dens = {}
        for name, sig in (("initial", x), ("filtered", y)):
            d = gift.bin_density(sig, box, 512, 512, w0=1.0, h0=1.0)
            dens[name] = {"max_over_bin_area": round(float(d.max()) / (W.DIE / 512) ** 2, 3),
                          "overflow_at_1": round(gift.density_overflow(
                              d, box, 1.0, float(nl.num_cells)), 5)}
        for _ in range(2):
            gift.bin_density(y, box, 512, 512, w0=1.0, h0=1.0)
        ev0.record()
        for _ in range(5):
            gift.bin_density(y, box, 512, 512, w0=1.0, h0=1.0)
        ev1.record()
        torch.cuda.synchronize()
        dens["ms"] = round(ev0.elapsed_time(ev1) / 5, 4)
        out["bin_density_512"] = dens
        # eigenvector placement [u_2, u_3] of the clique-model Laplacian, the
        # paper's comparison baseline
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, einfo = gift.eigen_placement(g, tol=1e-8, max_iter=400)
        e_ms = (time.perf_counter() - t0) * 1e3
        out["eigen_placement"] = {
            "tol": 1e-8, "lambda": [round(v, 9) for v in einfo["lambda"]],
            "residual_over_bound": [v / einfo["spectral_bound"] for v in einfo["residual"]],
            "iterations": einfo["iterations"], "converged": einfo["converged"],
            "component_cells": einfo["component_cells"], "ms": round(e_ms, 2)}
        out["placement_metrics"] = {
            "initial": {k: [round(float(v), 6) for v in m0[k]] for k in m0},
            "filtered": {k: [round(float(v), 6) for v in m1[k]] for k in m1},
            "evaluate_ms": round(ev_ms, 3)}
    g.close()
    if not args.no_extra:
        out["batched"] = [bench_batched(gift, W, torch, st) for st in ("f32", "bf16")]
        out["serving"] = bench_serving(gift, W, torch)

    if not args.no_cpu_baseline:
        from oracle import oracle as O
        log("[bench] timing the CPU oracle (one full step, single thread)")
        model, ncpu = host_cpu()
        xo = x_host.astype(np.float32).astype(np.float64)
        t0 = time.perf_counter()
        og = O.build_netlist(nl, star_threshold=thr)
        t1 = time.perf_counter()
        og.filter(xo, *terms)
        t2 = time.perf_counter()
        og_work = filter_work({"nnz": og.nnz, "num_rows": og.num_rows, "num_cells": og.num_cells,
                               "nnz_cells": int(og.row_ptr[og.num_cells])}, max(orders), 2)
        out["cpu_baseline"] = {
            "value": og_work / (t2 - t0), "unit": "nnz·cols/s", "cores": 1,
            "kind": "oracle",
            "sample": "one whole step of the same large workload (oracle build + 16-pass "
                      "filter, float64), single-threaded C",
            "build_s": round(t1 - t0, 3), "filter_s": round(t2 - t1, 3),
            "host_cpu": model, "host_threads": ncpu}
        og.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
