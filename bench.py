#!/usr/bin/env python3
"""Benchmark of the GiFt hot path on one MI355X.

One step = the whole hot path on the large synthetic workload (2,000,000
movable + 20,000 fixed cells, 2,100,000 nets, pins 2 + Zipf(2.2) capped at
1000, 90% index-local; nets above 16 cells star-expanded): netlist -> graph
build (dedupe, expansion, CSR sort/merge, degrees, normalisation) and the
multi-order filter (sigma 4, orders 1, 2, 4, 8, 16, equal weights, 2 signal
columns, float32 storage, fixed cells kept at their positions).  The netlist
and the signal are resident in HBM before the timed region starts.

Prints one JSON line.  ``value`` is filter work per second of whole step:
sum over the 16 SpMM passes of (stored entries + diagonal) x columns,
divided by the step time (build included).  ``filter_only`` is the same work
over the filter's own time on a resident graph.  The roofline object
describes the dominant kernel, the non-final SpMM pass, timed per launch with
HIP events on its own stream by the library's profiler during the timed
steps.  Further keys: the BF16 leg of the same workload, the tiny (FP64) and
medium (FP32) workloads, the build's algorithmic bytes, the attainable
bandwidth of a plain copy, the placement metrics, the batched and served
workloads, and the CPU oracle (one thread and all host cores) with the
accuracy of the GPU results against it.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "filter nnz·cols/s + achieved HBM GB/s vs peak; p50/p99 request latency"
# rocprofv3 counter summaries of the SpMM pass, one per storage type
COUNTERS = os.path.join(ROOT, "profiles", "spmm_large_{storage}_counters.txt")
STAR = 16
EQ5 = ([4.0] * 5, [1, 2, 4, 8, 16], [0.2] * 5)
EQ4 = ([4.0] * 4, [1, 2, 4, 8], [0.25] * 4)


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
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        usable = os.cpu_count()
    return model, os.cpu_count(), usable


# the timed steps whose launches the library's event profiler brackets
PROF_EVERY = 5


def counter_traffic(storage):
    """HBM bytes per SpMM launch measured with rocprofv3 counters for this
    storage type, if they were taken on the current kernel source."""
    src = os.path.join(ROOT, "paper_2502_17632_amd", "csrc", "filter.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    try:
        kv = {}
        for line in open(COUNTERS.format(storage=storage)):
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
    bo = 8 if storage == "f64" else 4

    def one(r, z, fin):
        b = 4 * (r + 1) + (4 + bt) * z + ba * r + bt * cols * rows
        if not fin:
            return b + bt * cols * r
        return b + (num_terms - 1) * bt * cols * r + bo * cols * r
    return one(rows, nnz, False) * (passes - 1) + one(cells, nnz_cells, True)


def build_bytes(nl, info, storage):
    """Algorithmic bytes of one build: the netlist read (int64 offsets, int32
    pins), the expanded (column, net) keys written once and read once (8 bytes
    each; Z = sum over nets of M(M-1), or 2M for a star), and the resident
    graph written (int32 row_ptr and col, float64 weights and degrees, the
    normalised values in the storage type and the float32 diagonal)."""
    import numpy as np
    m = np.diff(nl.net_ptr)
    z = int(np.where(m > STAR, 2 * m, m * (m - 1)).sum())
    bt = {"f32": 4, "bf16": 2, "f16": 2, "f64": 8}[storage]
    r, nnz = info["num_rows"], info["nnz"]
    netlist = 8 * (nl.num_nets + 1) + 4 * nl.num_pins
    keys = 2 * 8 * z
    graph = 4 * (r + 1) + (4 + 8 + bt) * nnz + 8 * r + 4 * r
    return netlist + keys + graph, z


def timed_events(torch, fn, reps, warm=3):
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def timed_events_each(torch, fn, reps, warm=3):
    """Per-call device times (ms) of `reps` back-to-back calls: events
    between the calls on the current stream, no synchronisation between
    them."""
    import numpy as np
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record()
    for k in range(reps):
        fn()
        ev[k + 1].record()
    torch.cuda.synchronize()
    return np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(reps)])


def host_end_to_end(gift, torch, nl, x_host, terms, reps=5):
    """One step with the netlist and the signal in host memory and the result
    copied back to host memory: the build reads the netlist from pageable
    host arrays (the library uploads it), the signal and the fixed mask go up
    from pinned buffers, the filtered placement comes back into a pinned
    buffer.  Wall time per step, synchronised at both ends."""
    import numpy as np
    xp = torch.from_numpy(np.ascontiguousarray(x_host, dtype=np.float32)).pin_memory()
    fp = torch.from_numpy(np.ascontiguousarray(nl.fixed)).pin_memory()
    out = torch.empty(xp.shape, dtype=torch.float32).pin_memory()

    def once():
        g = gift.build_graph(nl.num_cells, nl.net_ptr, nl.pin_cell, star_threshold=STAR,
                             sigmas=[4.0])
        xd = xp.to("cuda", non_blocking=True)
        fd = fp.to("cuda", non_blocking=True)
        y = gift.filter_placement(g, *terms, xd, fixed=fd)
        out.copy_(y, non_blocking=True)
        g.close()

    once()
    torch.cuda.synchronize()
    t = []
    for _ in range(reps):
        t0 = time.perf_counter()
        once()
        torch.cuda.synchronize()
        t.append((time.perf_counter() - t0) * 1e3)
    return float(np.median(t)), out.numpy().copy()


def attainable_bandwidth(torch):
    """A plain device copy of 1 GiB (read + write): what a streaming kernel
    reaches on this GPU, beside the 8 TB/s peak."""
    n = 1024 * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    ms = timed_events(torch, lambda: b.copy_(a), 10)
    copy = 2 * n * 4 / (ms * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return {"copy_GBs": round(copy, 1),
            "how": "torch copy_ of 1 GiB (bytes read + bytes written), 10 reps"}


def build_roofline(torch, nl, build_ms, b_bytes, copy_gbs):
    """The build's bound.  Turning the net-major netlist into row-major
    entries costs, per pin of a net with at least two cells, one returning
    device-scope atomic add (its slice in the row), one random 8-byte read
    (the row's offset) and one store of its keys into a random row; the rest
    streams b_bytes.  Each rate is what a plain torch kernel reaches for the
    same operation on this netlist's own pin indices (index_add_ on int32
    counters, an int64 gather, an int64 scatter), so the floor is attainable
    work at attainable rates, beside the measured build."""
    import numpy as np
    m = np.diff(nl.net_ptr)
    owner = np.repeat(m, m)
    idx = torch.tensor(nl.pin_cell[owner >= 2].astype(np.int64), device="cuda")
    n = int(idx.numel())
    cnt = torch.zeros(nl.num_cells, dtype=torch.int32, device="cuda")
    ones = torch.ones(n, dtype=torch.int32, device="cuda")
    table = torch.arange(nl.num_cells, dtype=torch.int64, device="cuda")
    dst = torch.empty(nl.num_cells, dtype=torch.int64, device="cuda")
    src = torch.arange(n, dtype=torch.int64, device="cuda")
    ms_atomic = timed_events(torch, lambda: cnt.index_add_(0, idx, ones), 10)
    ms_gather = timed_events(torch, lambda: table[idx], 10)
    ms_scatter = timed_events(torch, lambda: dst.scatter_(0, idx, src), 10)
    del idx, cnt, ones, table, dst, src
    torch.cuda.empty_cache()
    stream_ms = b_bytes / (copy_gbs * 1e9) * 1e3
    floor = ms_atomic + ms_gather + ms_scatter + stream_ms
    return {"bound": "random device-scope operations + HBM streaming",
            "random_ops_per_kind": n,
            "atomic_G_per_s": round(n / (ms_atomic * 1e-3) / 1e9, 1),
            "gather_G_per_s": round(n / (ms_gather * 1e-3) / 1e9, 1),
            "scatter_G_per_s": round(n / (ms_scatter * 1e-3) / 1e9, 1),
            "streamed_bytes": b_bytes, "copy_GBs": copy_gbs,
            "floor_ms": round(floor, 4), "measured_ms": round(build_ms, 4),
            "frac": round(floor / build_ms, 4),
            "how": "rates of torch index_add_ (int32 counters), gather and scatter_ (int64) "
                   "over the pins of nets with >= 2 cells, 10 reps each; streaming at the "
                   "attainable copy bandwidth"}


def filter_leg(gift, W, torch, nl, storage, terms, cols_x, label, reps=20, also_class1=False):
    """Filter-only timing on a resident graph: whole filter (events) and the
    SpMM pass (library profiler), with algorithmic bytes and roofline
    fraction; with also_class1, the same under SpMM tile class 1 (smaller
    tiles, more blocks), which small graphs fill the GPU better with."""
    g = gift.build_graph(nl.num_cells, nl.net_ptr, nl.pin_cell, star_threshold=STAR,
                         storage=storage, sigmas=sorted(set(terms[0])))
    info = g.info()
    row_ptr, _, _, _ = g.export()
    info["nnz_cells"] = int(row_ptr[nl.num_cells])
    dt = torch.float64 if storage == "f64" else torch.float32
    x = torch.tensor(cols_x, dtype=dt, device="cuda")
    fx = torch.tensor(nl.fixed, device="cuda")
    y = torch.empty_like(x)
    passes = max(terms[1])
    ms = timed_events(torch, lambda: gift.filter_placement(g, *terms, x, fixed=fx, out=y,
                                                           out_dtype=dt), reps)
    gift.profile_enable(True)
    timed_events(torch, lambda: gift.filter_placement(g, *terms, x, fixed=fx, out=y,
                                                      out_dtype=dt), 5, warm=0)
    sp = gift.profile_collect("spmm")
    gift.profile_enable(False)
    work = filter_work(info, passes, x.shape[1])
    nbytes = filter_bytes(info["nnz"], info["num_rows"], info["nnz_cells"], info["num_cells"],
                          x.shape[1], passes, len(terms[0]), storage)
    pass_us = sp["total_ms"] / max(sp["launches"], 1) * 1e3
    pass_bytes = sp["bytes"] / max(sp["launches"], 1)
    out = {"workload": label, "storage": storage, "rows": info["num_rows"], "nnz": info["nnz"],
           "cols": int(x.shape[1]), "passes": passes, "filter_ms": round(ms, 4),
           "nnz_cols_per_s": work / (ms * 1e-3),
           "filter_algorithmic_GBs": round(nbytes / (ms * 1e-3) / 1e9, 1),
           "spmm_pass_us": round(pass_us, 2), "spmm_pass_bytes": pass_bytes,
           "spmm_pass_GBs": round(pass_bytes / (pass_us * 1e-6) / 1e9, 1) if pass_us else None,
           "spmm_pass_frac": round(pass_bytes / (pass_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)
           if pass_us else None}
    yh = y.double().cpu().numpy()
    if also_class1:
        g.set_tile_class(1)
        ms1 = timed_events(torch, lambda: gift.filter_placement(g, *terms, x, fixed=fx, out=y,
                                                                out_dtype=dt), reps)
        gift.profile_enable(True)
        timed_events(torch, lambda: gift.filter_placement(g, *terms, x, fixed=fx, out=y,
                                                          out_dtype=dt), 5, warm=0)
        sp1 = gift.profile_collect("spmm")
        gift.profile_enable(False)
        us1 = sp1["total_ms"] / max(sp1["launches"], 1) * 1e3
        b1 = sp1["bytes"] / max(sp1["launches"], 1)
        out["tile_class1"] = {"filter_ms": round(ms1, 4), "nnz_cols_per_s": work / (ms1 * 1e-3),
                              "spmm_pass_us": round(us1, 2),
                              "spmm_pass_frac": round(b1 / (us1 * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)
                              if us1 else None,
                              "note": "gift_graph_set_tile_class(1); the default (class 0) "
                                      "keeps single-graph results bit-identical to the batch "
                                      "default schedule and the server"}
    g.close()
    return out, yh


def bench_tiny_latency(gift, W, torch):
    """The tiny workload in float64 (orders 1, 2, 4, 8: 8 passes): build and
    filter latency, launch-bound."""
    nl = W.tiny()
    x = torch.tensor(W.make_signal(nl), dtype=torch.float64, device="cuda")
    fx = torch.tensor(nl.fixed, device="cuda")
    ms_build = timed_events(torch, lambda: gift.build_graph(
        nl.num_cells, nl.net_ptr, nl.pin_cell, storage="f64", sigmas=[4.0]).close(), 10)
    g = gift.build_graph(nl.num_cells, nl.net_ptr, nl.pin_cell, storage="f64", sigmas=[4.0])
    y = torch.empty_like(x)
    lat = []
    for _ in range(3):
        gift.filter_placement(g, *EQ4, x, fixed=fx, out=y, out_dtype=torch.float64)
    torch.cuda.synchronize()
    for _ in range(50):
        t0 = time.perf_counter()
        gift.filter_placement(g, *EQ4, x, fixed=fx, out=y, out_dtype=torch.float64)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t0) * 1e3)
    dev_ms = timed_events(torch, lambda: gift.filter_placement(g, *EQ4, x, fixed=fx, out=y,
                                                               out_dtype=torch.float64), 50)
    # the same filter captured once into a HIP graph (a batch of this one
    # design, default schedule) and replayed: the launch overhead goes away
    b = gift.Batch([g], *EQ4, num_cols=2, in_dtype=torch.float64, out_dtype=torch.float64,
                   tune=0)
    y2 = torch.empty_like(x)
    for _ in range(3):
        b.run([x], [y2], fixed=[fx])
    torch.cuda.synchronize()
    lat2 = []
    for _ in range(50):
        t0 = time.perf_counter()
        b.run([x], [y2], fixed=[fx])
        torch.cuda.synchronize()
        lat2.append((time.perf_counter() - t0) * 1e3)
    dev2_ms = timed_events(torch, lambda: b.run([x], [y2], fixed=[fx]), 50)
    same = bool(torch.equal(y, y2))
    b.close()
    g.close()
    import numpy as np
    return {"workload": "tiny: 2,000 + 200 cells, 2,500 nets, 2 + Geom(0.5) pins <= 8, uniform; "
                        "sigma 4, orders 1,2,4,8, equal weights; 2 columns, float64",
            "build_wall_ms": round(ms_build, 4),
            "filter_latency_ms_p50": round(float(np.percentile(lat, 50)), 4),
            "filter_latency_ms_p99": round(float(np.percentile(lat, 99)), 4),
            "filter_device_ms": round(dev_ms, 4),
            "captured_latency_ms_p50": round(float(np.percentile(lat2, 50)), 4),
            "captured_latency_ms_p99": round(float(np.percentile(lat2, 99)), 4),
            "captured_device_ms": round(dev2_ms, 4),
            "captured_equal_to_uncaptured": same,
            "note": "latency = call to completion on the host (launch-bound); device = events; "
                    "captured = the filter recorded once into a HIP graph (gift_batch_* with "
                    "this one design) and replayed"}


def bench_batched(gift, W, torch, storage, reps=10):
    """64 designs (log-uniform 10k-300k movable cells, the medium generator,
    per-design seeds), 8 columns each (4 placements), sigma 4, orders
    1, 2, 4, 8, equal weights, fixed cells kept: the per-design path (64
    filter calls) against one tuned batch replaying its captured launch
    sequence."""
    orders = [1, 2, 4, 8]
    terms = ([4.0] * 4, orders, [0.25] * 4)
    sizes = W.batch_sizes(64)
    log(f"[bench] batched {storage}: generating 64 designs")
    nls = [W.sized(n, seed=1000 + i) for i, n in enumerate(sizes)]
    xs = [torch.tensor(W.make_signal(nl, W.BATCH_NOISE, seed=1000 + i), dtype=torch.float32,
                       device="cuda") for i, nl in enumerate(nls)]
    fxs = [torch.tensor(nl.fixed, device="cuda") for nl in nls]
    graphs = [gift.build_graph(nl.num_cells, nl.net_ptr, nl.pin_cell, star_threshold=STAR,
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
        for g, x, f, y in zip(graphs, xs, fxs, ys_alone):
            gift.filter_placement(g, *terms, x, fixed=f, out=y)
    ms_alone, wall_alone = timed(alone)

    t0 = time.perf_counter()
    b = gift.Batch(graphs, *terms, num_cols=8, tune=1)
    create_s = time.perf_counter() - t0
    ys = [torch.empty_like(x) for x in xs]
    ms_batch, wall_batch = timed(lambda: b.run(xs, ys, fixed=fxs))
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
                    "1000+i), 8 columns, sigma 4, orders 1,2,4,8, equal weights, fixed cells kept",
        "storage": storage, "cells": cells, "rows": rows, "nnz": nnz,
        "per_design_ms": round(ms_alone, 4), "per_design_wall_ms": round(wall_alone, 4),
        "batched_ms": round(ms_batch, 4), "batched_wall_ms": round(wall_batch, 4),
        "speedup": round(ms_alone / ms_batch, 3),
        "batched_nnz_cols_per_s": work / (ms_batch * 1e-3),
        "per_design_nnz_cols_per_s": work / (ms_alone * 1e-3),
        "batched_algorithmic_GBs": round(nbytes / (ms_batch * 1e-3) / 1e9, 1),
        "batched_frac": round(nbytes / (ms_batch * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "max_normwise_diff_vs_per_design": worst,
        "schedule": {"tile_class": info["tile_class"], "chunk_cols": info["chunk_cols"],
                     "xcd_affine": info["xcd_affine"],
                     "tuned": info["tuned"], "tune_s": round(create_s, 3),
                     "candidates": [(c["tile_class"], c["chunk_cols"], c["xcd_affine"],
                                     round(c["ms"], 4)) for c in info["candidates"]]},
    }


def bench_serving(gift, W, torch, n_requests=1000, pool=24, loads=(0.7, 2.0), cold_reps=4):
    """Poisson streams of filter requests (2 columns, sigma 4, orders
    1, 2, 4, 8, fixed cells kept) over a pool of designs with log-uniform
    5k-2M movable cells.

    cold: one request per design, every graph built on demand (build +
    filter), `cold_reps` independent streams pooled; warm: every graph
    resident, at offered loads given as multiples of the serial warm
    capacity.  Serial per-request execution (filter, wait)
    is compared with the serving engine.  Latency runs from each request's
    arrival to its completion on the device."""
    import numpy as np
    terms = ([4.0] * 4, [1, 2, 4, 8], [0.25] * 4)
    sizes = W.serving_sizes(pool)
    log(f"[bench] serving: generating {pool} designs")
    nls = [W.sized(n, seed=5000 + i) for i, n in enumerate(sizes)]
    xs = [torch.tensor(W.make_signal(nl, seed=5000 + i), dtype=torch.float32, device="cuda")
          for i, nl in enumerate(nls)]
    fxs = [torch.tensor(nl.fixed, device="cuda") for nl in nls]
    design_of = np.random.default_rng(4244).integers(0, pool, size=n_requests)
    torch.cuda.synchronize()

    def wait_until(t):
        while True:
            d = t - time.perf_counter()
            if d <= 0:
                return
            if d > 2e-3:
                time.sleep(d - 1e-3)

    def summary(lat, span, n):
        return {"p50_ms": round(float(np.percentile(lat, 50)), 3),
                "p99_ms": round(float(np.percentile(lat, 99)), 3),
                "mean_ms": round(float(lat.mean()), 3), "makespan_s": round(span, 3),
                "throughput_rps": round(n / span, 1)}

    def build(d):
        nl = nls[d]
        return gift.build_graph(nl.num_cells, nl.net_ptr, nl.pin_cell, star_threshold=STAR,
                                sigmas=[4.0])

    def serial(order, arrivals, cache):
        outs, lat = [], []
        t0 = time.perf_counter()
        for j, d in enumerate(order):
            ta = t0 + arrivals[j] if arrivals is not None else time.perf_counter()
            if arrivals is not None:
                wait_until(ta)
            g = cache.get(d)
            if g is None:
                g = cache[d] = build(d)
            outs.append(gift.filter_placement(g, *terms, xs[d], fixed=fxs[d]))
            torch.cuda.synchronize()
            lat.append((time.perf_counter() - ta) * 1e3)
        return np.array(lat), time.perf_counter() - t0, outs

    def served(srv, order, arrivals):
        t0 = time.perf_counter()
        subs = []
        for j, d in enumerate(order):
            ta = t0 + arrivals[j] if arrivals is not None else time.perf_counter()
            if arrivals is not None:
                wait_until(ta)
            nl = nls[d]
            lag = (time.perf_counter() - ta) * 1e3
            t, y = srv.submit(int(d), nl.num_cells, nl.net_ptr, nl.pin_cell, xs[d],
                              fixed=fxs[d])
            subs.append((t, y, lag))
        res = [srv.wait(t) for t, _, _ in subs]
        lat = np.array([lag + r["latency_ms"] for (_, _, lag), r in zip(subs, res)])
        return lat, time.perf_counter() - t0, [y for _, y, _ in subs], res

    def new_server():
        return gift.Server(*terms, num_cols=2, hbm_budget_bytes=200 << 30, max_inflight=64,
                           num_streams=4, num_builders=2, max_batch=32)

    out = {"workload": f"{n_requests} requests per warm stream, Poisson arrivals (seed 4242), "
                       f"over {pool} designs with log-uniform 5k-2M movable cells (medium "
                       "generator, seeds 5000+i), 2 columns, sigma 4, orders 1,2,4,8, fixed "
                       f"cells kept; cold: one request per design, {cold_reps} streams"}
    # cold: every design once, each build on demand
    cold_order = np.arange(pool)
    cache = {}
    lat_sc, span_sc, outs_sc = serial(cold_order, None, cache)
    cold_rate = pool / span_sc
    # independent cold streams (fresh graphs and server each), pooled: one
    # stream of 24 requests near the serial capacity is too few for a stable
    # p50 / p99
    lat_sc, lat_vc, span_sc, span_vc, same, srv = [], [], 0.0, 0.0, True, None
    for rep in range(cold_reps):
        for g in cache.values():
            g.close()
        cache = {}
        if srv is not None:
            srv.close()
        arr = W.poisson_arrivals(pool, cold_rate, seed=4245 + rep)
        l_s, sp_s, outs_sc = serial(cold_order, arr, cache)
        srv = new_server()
        l_v, sp_v, outs_vc, _ = served(srv, cold_order, arr)
        same = same and all(torch.equal(a, b) for a, b in zip(outs_sc, outs_vc))
        lat_sc.append(l_s)
        lat_vc.append(l_v)
        span_sc += sp_s
        span_vc += sp_v
    out["cold"] = {"rate_rps": round(cold_rate, 1), "streams": cold_reps,
                   "serial": summary(np.concatenate(lat_sc), span_sc, pool * cold_reps),
                   "served": summary(np.concatenate(lat_vc), span_vc, pool * cold_reps)}
    # warm: every graph resident (the serial cache and the server above)
    _, busy, _ = serial(design_of, None, cache)
    cap = n_requests / busy
    out["serial_warm_capacity_rps"] = round(cap, 1)
    out["warm"] = []
    for load in loads:
        arrivals = W.poisson_arrivals(n_requests, load * cap)
        log(f"[bench] serving: warm, load {load} ({load * cap:.0f} requests/s)")
        lat_s, span_s, outs_s = serial(design_of, arrivals, cache)
        srv.stats(reset=True)
        lat_v, span_v, outs_v, _ = served(srv, design_of, arrivals)
        st = srv.stats()
        same = same and all(torch.equal(a, b) for a, b in zip(outs_s, outs_v))
        out["warm"].append({
            "load": load, "rate_rps": round(load * cap, 1),
            "serial": summary(lat_s, span_s, n_requests),
            "served": summary(lat_v, span_v, n_requests),
            "served_batches": st["batches"],
            "served_mean_batch": round(st["batched_requests"] / max(st["batches"], 1), 2),
            "builds": st["builds"]})
    srv.stats(reset=True)
    _, span_sat, outs_sat, _ = served(srv, design_of, None)
    st = srv.stats()
    same = same and all(torch.equal(a, b) for a, b in zip(outs_s, outs_sat))
    out["warm_saturated"] = {
        "serial_throughput_rps": round(cap, 1),
        "served_throughput_rps": round(n_requests / span_sat, 1),
        "served_mean_batch": round(st["batched_requests"] / max(st["batches"], 1), 2)}
    srv.close()
    for g in cache.values():
        g.close()
    out["results_equal_to_serial"] = bool(same)
    return out


def oracle_worker(argv):
    """One CPU oracle step (build + filter of the large workload) in this
    process; waits for a line on stdin before the timed region so that all
    workers start together, prints one JSON line."""
    import numpy as np
    from paper_2502_17632_amd import workload as W
    from oracle import oracle as O
    nl = W.large()
    x = W.make_signal(nl).astype(np.float32).astype(np.float64)
    O.load()
    print("ready", flush=True)
    sys.stdin.readline()
    t0 = time.perf_counter()
    og = O.build_netlist(nl, star_threshold=STAR, star_order="median")
    t1 = time.perf_counter()
    og.filter(x, *EQ5, fixed=nl.fixed)
    t2 = time.perf_counter()
    work = filter_work({"nnz": og.nnz, "num_rows": og.num_rows, "num_cells": og.num_cells,
                        "nnz_cells": int(og.row_ptr[og.num_cells])}, 16, 2)
    og.close()
    print(json.dumps({"work": work, "build_s": t1 - t0, "filter_s": t2 - t1, "t0": t0, "t2": t2}),
          flush=True)
    return 0


def cpu_all_cores(workers):
    """`workers` oracle processes run one step each, started together; the
    aggregate throughput is their total work over the wall time from the
    common start to the last finish."""
    procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--oracle-worker"],
                              stdin=subprocess.PIPE, stdout=subprocess.PIPE, text=True,
                              cwd=ROOT) for _ in range(workers)]
    for p in procs:
        line = p.stdout.readline()
        if line.strip() != "ready":
            raise RuntimeError(f"oracle worker failed to start: {line!r}")
    t0 = time.perf_counter()
    for p in procs:
        p.stdin.write("go\n")
        p.stdin.flush()
    res = []
    for p in procs:
        res.append(json.loads(p.stdout.readline()))
        p.wait()
    wall = time.perf_counter() - t0
    return {"value": sum(r["work"] for r in res) / wall, "wall_s": round(wall, 3),
            "per_worker_s": [round(r["build_s"] + r["filter_s"], 3) for r in res]}


def accuracy(y, ref):
    """Normwise, spread-relative and RMS error per column against the FP64
    oracle."""
    import numpy as np
    den = np.abs(ref).max(axis=0)
    spread = np.abs(ref - ref.mean(axis=0, keepdims=True)).max(axis=0)
    d = np.abs(y - ref)
    return {"normwise": [float(v) for v in d.max(axis=0) / den],
            "spread_relative": [float(v) for v in d.max(axis=0) / spread],
            "rms": [float(v) for v in np.sqrt(np.mean((y - ref) ** 2, axis=0))]}


def movable_netlist(nl):
    """The netlist with the fixed cells' pins removed (nets keep their
    movable pins), for HPWL over movable cells only."""
    import numpy as np
    keep = nl.fixed[nl.pin_cell] == 0
    counts = np.add.reduceat(keep.astype(np.int64), nl.net_ptr[:-1]) if nl.num_nets else \
        np.zeros(0, np.int64)
    counts = np.where(np.diff(nl.net_ptr) > 0, counts, 0)
    net_ptr = np.zeros(nl.num_nets + 1, dtype=np.int64)
    np.cumsum(counts, out=net_ptr[1:])
    return net_ptr, nl.pin_cell[keep].astype(np.int32)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--storage", default="f32", choices=["f32", "bf16", "f16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the extra measurements")
    ap.add_argument("--oracle-worker", action="store_true", help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.oracle_worker:
        return oracle_worker(sys.argv)
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path "
              f"(--gpus {args.gpus} requested)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2502_17632_amd as gift
    from paper_2502_17632_amd import workload as W

    torch.cuda.set_device(0)
    orders = EQ5[1]
    terms = EQ5
    log("[bench] generating the large workload")
    nl = W.large()
    x_host = W.make_signal(nl)
    net_ptr = torch.tensor(nl.net_ptr, device="cuda")
    pin_cell = torch.tensor(nl.pin_cell, device="cuda")
    fixed = torch.tensor(nl.fixed, device="cuda")
    x = torch.tensor(x_host, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()

    def step():
        g = gift.build_graph(nl.num_cells, net_ptr, pin_cell, star_threshold=STAR,
                             storage=args.storage, sigmas=[4.0])
        gift.filter_placement(g, *terms, x, fixed=fixed, out=y)
        info = g.info()
        g.close()
        return info

    # nnz of the cell rows: from the exported row pointer of one graph, which
    # stays resident for the extra measurements; built before the warm-up so
    # that the warm-up steps already run beside it (memory pools at their
    # steady size when the timed steps start)
    g = gift.build_graph(nl.num_cells, net_ptr, pin_cell, star_threshold=STAR,
                         storage=args.storage, sigmas=[4.0])
    row_ptr, _, _, _ = g.export()
    nnz_cells = int(row_ptr[nl.num_cells])
    log("[bench] warmup")
    info = None
    # the warm-up runs with the event profiler on, so that its event pool is
    # filled before the timed steps (records collected and dropped below)
    gift.profile_enable(True)
    for _ in range(args.warmup):
        info = step()
    torch.cuda.synchronize()
    for kind in ("spmm", "spmm_final", "build"):
        gift.profile_collect(kind)
    if info is None:
        info = step()
        torch.cuda.synchronize()
    info["nnz_cells"] = nnz_cells

    log(f"[bench] timing {args.steps} steps")
    gift.profile_enable(True)
    torch.cuda.synchronize()
    # The library's events bracket every launch of the steps the profiler
    # samples (one step in PROF_EVERY, the first one included): the events
    # cost about 80 us per step, so sampling keeps them off most steps.
    # Events between the steps on the stream the steps run on give per-step
    # times without a synchronisation inside the timed region.
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    sampled = [k for k in range(args.steps) if k % PROF_EVERY == 0]
    t0 = time.perf_counter()
    marks[0].record()
    for k in range(args.steps):
        gift.profile_pause(k % PROF_EVERY != 0)
        step()
        marks[k + 1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    step_ms = [round(marks[k].elapsed_time(marks[k + 1]), 3) for k in range(args.steps)]
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
    traffic = counter_traffic(args.storage)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "kernel": "k_spmm (non-final pass)",
                "bytes_per_launch": bytes_launch, "avg_launch_us": round(avg_ms * 1e3, 2),
                "launches": spmm["launches"]}
    build_ms = bld["total_ms"] / max(bld["launches"], 1)
    b_bytes, z = build_bytes(nl, info, args.storage)

    out = {
        "metric": METRIC, "value": value, "unit": "nnz·cols/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "step_ms": step_ms,
        "profiled_steps": sampled,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.storage, "data": "synthetic",
        "config": {"workload": "large: 2M+20k cells, 2.1M nets, Zipf(2.2) pins <= 1000, "
                               "90% local; star above 16 cells; sigma 4, orders 1,2,4,8,16, "
                               "equal weights; 2 columns; fixed cells kept",
                   "cells": nl.num_cells, "nets": nl.num_nets, "rows": info["num_rows"],
                   "nnz": info["nnz"], "cols": 2, "storage": args.storage,
                   "passes": max(orders)},
        "value_note": "filter work over the whole step (build + filter + release); "
                      "filter_only.nnz_cols_per_s is the filter alone on a resident graph",
        "roofline": roofline,
        "breakdown": {
            "build_ms": round(build_ms, 4),
            "filter_final_pass_us": round(fin["total_ms"] / max(fin["launches"], 1) * 1e3, 2),
            "spmm_pass_us": round(avg_ms * 1e3, 2),
        },
        "build": {"ms": round(build_ms, 4), "algorithmic_bytes": b_bytes, "expanded_keys": z,
                  "algorithmic_GBs": round(b_bytes / (build_ms * 1e-3) / 1e9, 1),
                  "frac": round(b_bytes / (build_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                  "bytes": "netlist read + (column, net) keys written and read (8 B each) + "
                           "resident graph written"},
    }
    y_f32 = None
    y_bf16 = None
    if not args.no_extra:
        out["attainable"] = attainable_bandwidth(torch)
        roofline["frac_of_copy"] = round(achieved / out["attainable"]["copy_GBs"], 4)
        out["build"]["roofline"] = build_roofline(torch, nl, build_ms, b_bytes,
                                                  out["attainable"]["copy_GBs"])
        # the filter alone on a resident graph
        each = timed_events_each(torch, lambda: gift.filter_placement(g, *terms, x, fixed=fixed,
                                                                      out=y), 20)
        ms_f = float(each.mean())
        fbytes = filter_bytes(info["nnz"], info["num_rows"], info["nnz_cells"],
                              info["num_cells"], 2, max(orders), len(orders), args.storage)
        out["filter_only"] = {"ms": round(ms_f, 4), "nnz_cols_per_s": work / (ms_f * 1e-3),
                              "median_ms": round(float(np.median(each)), 4),
                              "p10_ms": round(float(np.percentile(each, 10)), 4),
                              "p90_ms": round(float(np.percentile(each, 90)), 4),
                              "reps": int(each.size),
                              "algorithmic_bytes": fbytes,
                              "algorithmic_GBs": round(fbytes / (ms_f * 1e-3) / 1e9, 1),
                              "frac": round(fbytes / (ms_f * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        # the same step with host-resident inputs and output (PCIe included)
        h_ms, y_host = host_end_to_end(gift, torch, nl, x_host, terms)
        out["host_inputs"] = {
            "ms_per_step": round(h_ms, 3), "nnz_cols_per_s": work / (h_ms * 1e-3),
            "equal_to_device_inputs": bool(np.array_equal(y_host, y.cpu().numpy())),
            "note": "netlist in pageable host arrays (uploaded by the build), signal and "
                    "fixed mask from pinned host buffers, result copied back to pinned host "
                    "memory; median wall time of 5 steps"}
        y_f32 = y.double().cpu().numpy()
        # what the filter does to the placement (fixed cells restored):
        # smoothness / quadratic wirelength, Rayleigh quotient and HPWL
        # before and after; HPWL also over the movable cells' pins only
        t0 = time.perf_counter()
        m0 = gift.evaluate_placement(g, x, net_ptr, pin_cell)
        ev_ms = (time.perf_counter() - t0) * 1e3
        m1 = gift.evaluate_placement(g, y, net_ptr, pin_cell)
        mnp, mpc = movable_netlist(nl)
        h0 = gift.evaluate_placement(g, x, mnp, mpc)["hpwl"]
        h1 = gift.evaluate_placement(g, y, mnp, mpc)["hpwl"]
        # the exact filter (I + L~_4)^-1 g that the paper's filter approximates
        for _ in range(2):
            gift.filter_exact(g, 4.0, x, tol=1e-6, fixed=fixed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ye, its = gift.filter_exact(g, 4.0, x, tol=1e-6, fixed=fixed)
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
        dens["ms"] = round(timed_events(torch, lambda: gift.bin_density(
            y, box, 512, 512, w0=1.0, h0=1.0), 5, warm=2), 4)
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
            "fixed_cells": "kept at their input positions in the filtered placement",
            "initial": {k: [round(float(v), 6) for v in m0[k]] for k in m0},
            "filtered": {k: [round(float(v), 6) for v in m1[k]] for k in m1},
            "hpwl_movable_pins_only": {"initial": [round(float(v), 3) for v in h0],
                                       "filtered": [round(float(v), 3) for v in h1]},
            "evaluate_ms": round(ev_ms, 3)}
    g.close()
    if not args.no_extra:
        log("[bench] large, BF16 storage")
        leg, y_bf16 = filter_leg(gift, W, torch, nl, "bf16", terms, x_host.astype(np.float32),
                                 "large (as above), BF16-stored values and signals, float32 "
                                 "accumulation")
        leg["spmm_pass_traffic"] = counter_traffic("bf16")
        out["large_bf16"] = leg
        log("[bench] tiny (float64) and medium (float32) workloads")
        out["tiny_f64"] = bench_tiny_latency(gift, W, torch)
        nm = W.medium()
        out["medium_f32"], _ = filter_leg(
            gift, W, torch, nm, "f32", EQ4, W.make_signal(nm).astype(np.float32),
            "medium: 200k+2k cells, 220k nets, Zipf(2.2) pins <= 1000, 90% local; star above "
            "16 cells; sigma 4, orders 1,2,4,8, equal weights; 2 columns, float32",
            also_class1=True)
        out["medium_f32"]["note"] = ("fits in the 256 MB MALL, so its GB/s may exceed what "
                                     "HBM alone delivers")
        out["batched"] = [bench_batched(gift, W, torch, st) for st in ("f32", "bf16")]
        out["serving"] = bench_serving(gift, W, torch)

    if not args.no_cpu_baseline:
        from oracle import oracle as O
        log("[bench] timing the CPU oracle (one full step, single thread)")
        model, ncpu, usable = host_cpu()
        xo = x_host.astype(np.float32).astype(np.float64)
        t0 = time.perf_counter()
        og = O.build_netlist(nl, star_threshold=STAR, star_order="median")
        t1 = time.perf_counter()
        ref = og.filter(xo, *terms, fixed=nl.fixed)
        t2 = time.perf_counter()
        og_work = filter_work({"nnz": og.nnz, "num_rows": og.num_rows, "num_cells": og.num_cells,
                               "nnz_cells": int(og.row_ptr[og.num_cells])}, max(orders), 2)
        og.close()
        workers = max(1, min(usable or 1, 16))
        log(f"[bench] timing the CPU oracle on {workers} host cores (one step per process)")
        allc = cpu_all_cores(workers)
        out["cpu_baseline"] = {
            "value": allc["value"], "unit": "nnz·cols/s", "cores": workers, "kind": "oracle",
            "sample": f"{workers} processes, each one whole step of the same large workload "
                      "(oracle build + 16-pass float64 filter), started together; total work "
                      "over the wall time to the last finish",
            "wall_s": allc["wall_s"], "per_process_s": allc["per_worker_s"],
            "single_thread": {"value": og_work / (t2 - t0), "cores": 1,
                              "build_s": round(t1 - t0, 3), "filter_s": round(t2 - t1, 3)},
            "host_cpu": model, "host_threads": ncpu, "usable_threads": usable}
        acc = {}
        if y_f32 is not None:
            acc["f32"] = accuracy(y_f32, ref)
        if y_bf16 is not None:
            acc["bf16"] = accuracy(y_bf16, ref)
        if acc:
            out["accuracy_vs_fp64_oracle"] = acc
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
