"""Helpers shared by the GPU parity tests: run the device path and the CPU
oracle on the same seeded inputs and compare them."""
from __future__ import annotations

import sys
from typing import Optional, Sequence

import numpy as np

from oracle import oracle as O

# Normwise per-column tolerance of the filtered coordinates, by storage type:
# ||y - y*||_inf / ||y*||_inf.  FP32 and BF16 are the stated targets; FP16 has
# three more significand bits than BF16, so 8x tighter; FP64 keeps only the
# rounding of a few dozen float64 operations per entry.
TOL = {"f32": 1e-5, "bf16": 2e-2, "f16": 2.5e-3, "f64": 1e-12}

WEIGHT_MODEL = {"inv_m1": O.W_INV_M1, "two_over_m": O.W_TWO_OVER_M}


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def colwise_error(y: np.ndarray, ref: np.ndarray) -> np.ndarray:
    den = np.abs(ref).max(axis=0)
    den = np.where(den > 0, den, 1.0)
    return np.abs(y - ref).max(axis=0) / den


def bf16_round(x: np.ndarray) -> np.ndarray:
    """float64 -> nearest bfloat16 (ties to even), returned as float64.
    Rounds through float32 and repairs the only case double rounding gets
    wrong: a float32 result exactly halfway between two bfloat16 values."""
    x = np.asarray(x, dtype=np.float64)
    f = x.astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    low = u & 0xFFFF
    f64 = f.astype(np.float64)
    mid = (low == 0x8000) & (f64 != x)
    away = mid & (np.abs(x) > np.abs(f64))
    toward = mid & ~away
    rne = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    res = np.where(away, (u + 0x8000) >> 16, np.where(toward, u >> 16, rne))
    return (res << 16).astype(np.uint32).view(np.float32).astype(np.float64)


def round_storage(x: np.ndarray, storage: str) -> np.ndarray:
    if storage == "f64":
        return np.asarray(x, dtype=np.float64)
    if storage == "f32":
        return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)
    if storage == "f16":
        return np.asarray(x, dtype=np.float64).astype(np.float16).astype(np.float64)
    if storage == "bf16":
        return bf16_round(x)
    raise ValueError(storage)


def check_structure(g, og: O.OracleGraph):
    """CSR, weights and degrees must equal the oracle's bit for bit."""
    row_ptr, col, w, deg = g.export()
    inf = g.info()
    assert inf["num_virtual"] == og.num_virtual
    assert inf["nnz"] == og.nnz
    assert np.array_equal(row_ptr, og.row_ptr)
    assert np.array_equal(col, og.col)
    assert np.array_equal(w.view(np.uint64), og.w.view(np.uint64))
    assert np.array_equal(deg.view(np.uint64), og.deg.view(np.uint64))


def check_normalised(g, og: O.OracleGraph, sigma: float, storage: str):
    """Stored normalised values equal the oracle's float64 values rounded once
    to the storage type; the diagonal to the accumulation type."""
    val, diag = g.export_normalised(sigma)
    a, d = og.normalise(sigma)
    exp_v = round_storage(a, storage)
    exp_d = d if storage == "f64" else d.astype(np.float32).astype(np.float64)
    bad_v = int(np.count_nonzero(val != exp_v))
    bad_d = int(np.count_nonzero(diag != exp_d))
    assert bad_v == 0 and bad_d == 0, (bad_v, bad_d)


def run_pair(netlist, x: np.ndarray, terms, *, storage: str = "f32", star_threshold: int = 0,
             weight_model: str = "inv_m1", fixed: Optional[np.ndarray] = None,
             structure: bool = True, out_dtype=None, og: Optional[O.OracleGraph] = None,
             label: str = ""):
    """Build + filter on the GPU and with the oracle; returns (y_gpu, y_ref, g, og)."""
    import torch
    import paper_2502_17632_amd as gift
    sig, order, alpha = terms
    log(f"[parity] {label} N={netlist.num_cells} E={netlist.num_nets} storage={storage} "
        f"T={star_threshold} terms={list(zip(sig, order, alpha))}")
    g = gift.build_graph(netlist.num_cells, netlist.net_ptr, netlist.pin_cell,
                         weight_model=weight_model, star_threshold=star_threshold,
                         storage=storage, sigmas=sorted(set(sig)))
    if og is None:
        og = O.build_graph(netlist.num_cells, netlist.net_ptr, netlist.pin_cell,
                           weight_model=WEIGHT_MODEL[weight_model],
                           star_threshold=star_threshold, star_order="median")
    if structure:
        check_structure(g, og)
    in_dt = torch.float64 if storage == "f64" else torch.float32
    xin = np.asarray(x, dtype=np.float64)
    if in_dt == torch.float32:
        xin = xin.astype(np.float32).astype(np.float64)
    xt = torch.tensor(xin, dtype=in_dt, device="cuda")
    ft = None if fixed is None else torch.tensor(fixed, dtype=torch.uint8, device="cuda")
    od = out_dtype or (torch.float64 if storage == "f64" else torch.float32)
    y = gift.filter_placement(g, sig, order, alpha, xt, fixed=ft, out_dtype=od)
    torch.cuda.synchronize()
    y = y.double().cpu().numpy()
    ref = og.filter(xin, sig, order, alpha, fixed=fixed)
    return y, ref, g, og


def spread_error(y: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """||y - y*||_inf / ||y* - mean(y*)||_inf per column: the error against
    the spread of the placement rather than its distance from the origin."""
    den = np.abs(ref - ref.mean(axis=0, keepdims=True)).max(axis=0)
    den = np.where(den > 0, den, 1.0)
    return np.abs(y - ref).max(axis=0) / den


def rms_error(y: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """Root mean square of y - y* per column (absolute)."""
    return np.sqrt(np.mean((y - ref) ** 2, axis=0))


def assert_close(y, ref, storage: str, label: str = ""):
    err = colwise_error(y, ref)
    log(f"[parity] {label} normwise error per column: "
        f"{' '.join(f'{e:.3e}' for e in err)} (tol {TOL[storage]:.1e}); spread-relative "
        f"{' '.join(f'{e:.3e}' for e in spread_error(y, ref))}; rms "
        f"{' '.join(f'{e:.3e}' for e in rms_error(y, ref))}")
    assert np.all(np.isfinite(y))
    assert np.all(err <= TOL[storage]), (label, err)
    return err
