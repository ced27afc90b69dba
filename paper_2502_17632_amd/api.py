"""Python binding of the GiFt library: argument marshalling only.

Every computation happens in the HIP library (``libgift.so``); torch is used
for device memory and streams.
"""
from __future__ import annotations

import ctypes as C
from typing import Iterable, Optional, Sequence, Tuple

import numpy as np
import torch

from . import _lib as L

DTYPES = {"f32": L.GIFT_F32, "f64": L.GIFT_F64, "bf16": L.GIFT_BF16, "f16": L.GIFT_F16}
TORCH_DTYPES = {torch.float32: L.GIFT_F32, torch.float64: L.GIFT_F64}
WEIGHT_MODELS = {"inv_m1": L.GIFT_W_INV_M1, "two_over_m": L.GIFT_W_TWO_OVER_M}


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        return t.data_ptr()
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    raise TypeError(f"unsupported buffer type {type(t)}")


def make_terms(sigma: Sequence[float], order: Sequence[int], alpha: Sequence[float]):
    if not (len(sigma) == len(order) == len(alpha)):
        raise ValueError("sigma, order and alpha differ in length")
    arr = (L.Term * len(sigma))()
    for i, (s, k, a) in enumerate(zip(sigma, order, alpha)):
        arr[i].sigma = float(s)
        arr[i].order = int(k)
        arr[i].reserved = 0
        arr[i].alpha = float(a)
    return arr


class Graph:
    """A resident normalised cell graph (owns the library handle)."""

    def __init__(self, handle: C.c_void_p, stream):
        self._h = handle
        self._stream = stream

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        inf = L.GraphInfo()
        L.check(L.lib().gift_graph_get_info(self._h, C.byref(inf)), "gift_graph_get_info")
        return {k: getattr(inf, k) for k, _ in L.GraphInfo._fields_}

    def add_sigma(self, sigma: float, stream=None):
        L.check(L.lib().gift_graph_add_sigma(self._h, float(sigma), _stream_handle(stream)),
                "gift_graph_add_sigma")

    def export(self, stream=None) -> Tuple[np.ndarray, np.ndarray, np.ndarray, np.ndarray]:
        inf = self.info()
        r, nnz = inf["num_rows"], inf["nnz"]
        row_ptr = np.empty(r + 1, dtype=np.int64)
        col = np.empty(nnz, dtype=np.int32)
        w = np.empty(nnz, dtype=np.float64)
        deg = np.empty(r, dtype=np.float64)
        L.check(L.lib().gift_graph_export(self._h, _ptr(row_ptr), _ptr(col), _ptr(w), _ptr(deg),
                                          _stream_handle(stream)), "gift_graph_export")
        return row_ptr, col, w, deg

    def export_normalised(self, sigma: float, stream=None) -> Tuple[np.ndarray, np.ndarray]:
        inf = self.info()
        val = np.empty(inf["nnz"], dtype=np.float64)
        diag = np.empty(inf["num_rows"], dtype=np.float64)
        L.check(L.lib().gift_graph_export_normalised(self._h, float(sigma), _ptr(val), _ptr(diag),
                                                     _stream_handle(stream)),
                "gift_graph_export_normalised")
        return val, diag

    def close(self, stream=None):
        if self._h is not None:
            L.check(L.lib().gift_destroy_graph(self._h, _stream_handle(stream or self._stream)),
                    "gift_destroy_graph")
            self._h = None

    def __del__(self):  # pragma: no cover - best effort
        try:
            if self._h is not None and torch.cuda.is_initialized():
                self.close()
        except Exception:
            pass


def build_graph(num_cells: int, net_ptr, pin_cell, *, weight_model: str = "inv_m1",
                star_threshold: int = 0, storage: str = "f32",
                sigmas: Iterable[float] = (4.0,), stream=None) -> Graph:
    """Netlist -> resident graph.  ``net_ptr``/``pin_cell`` may be numpy
    arrays (host) or CUDA tensors (device)."""
    if isinstance(net_ptr, torch.Tensor) != isinstance(pin_cell, torch.Tensor):
        raise TypeError("net_ptr and pin_cell must both be numpy arrays or both tensors")
    if isinstance(net_ptr, torch.Tensor):
        if not (net_ptr.is_cuda and pin_cell.is_cuda):
            raise TypeError("tensors must live on the GPU")
        if net_ptr.dtype != torch.int64 or pin_cell.dtype != torch.int32:
            raise TypeError("net_ptr must be int64 and pin_cell int32")
        net_ptr, pin_cell = net_ptr.contiguous(), pin_cell.contiguous()
        mem = L.GIFT_MEM_DEVICE
    else:
        net_ptr = np.ascontiguousarray(net_ptr, dtype=np.int64)
        pin_cell = np.ascontiguousarray(pin_cell, dtype=np.int32)
        mem = L.GIFT_MEM_HOST
    if net_ptr.dim() != 1 if isinstance(net_ptr, torch.Tensor) else net_ptr.ndim != 1:
        raise ValueError("net_ptr must be one-dimensional")
    if net_ptr.shape[0] < 1:
        raise ValueError("net_ptr needs num_nets + 1 >= 1 entries")
    if int(net_ptr[-1]) != int(pin_cell.shape[0]):
        raise ValueError(f"pin_cell has {int(pin_cell.shape[0])} entries but net_ptr[-1] = "
                         f"{int(net_ptr[-1])}")
    sig = np.ascontiguousarray(list(sigmas), dtype=np.float64)
    d = L.GraphDesc()
    d.num_cells = int(num_cells)
    d.num_nets = int(net_ptr.shape[0]) - 1
    d.net_ptr = _ptr(net_ptr)
    d.pin_cell = _ptr(pin_cell)
    d.mem_space = mem
    d.weight_model = WEIGHT_MODELS[weight_model]
    d.star_threshold = int(star_threshold)
    d.storage = DTYPES[storage]
    d.num_sigmas = int(sig.shape[0])
    d.sigmas = _ptr(sig)
    h = C.c_void_p()
    st = _stream_handle(stream)
    L.check(L.lib().gift_build_graph(C.byref(d), st, C.byref(h)), "gift_build_graph")
    return Graph(h, stream)


def filter_placement(graph: Graph, sigma: Sequence[float], order: Sequence[int],
                     alpha: Sequence[float], x: torch.Tensor, *,
                     fixed: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None,
                     out_dtype: torch.dtype = torch.float32, stream=None) -> torch.Tensor:
    """g' = sum_t alpha_t A~_{sigma_t}^{order_t} x  (x: N x c CUDA tensor, f32/f64)."""
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dim() == 2):
        raise TypeError("x must be a 2-D CUDA tensor")
    if x.stride(1) != 1:
        x = x.contiguous()
    if x.dtype not in TORCH_DTYPES:
        raise TypeError("x must be float32 or float64")
    n, c = x.shape
    if n != graph.info()["num_cells"]:
        raise ValueError(f"x has {n} rows but the graph has {graph.info()['num_cells']} cells")
    if out is None:
        out = torch.empty((n, c), dtype=out_dtype, device=x.device)
    if out.dtype not in TORCH_DTYPES or out.stride(1) != 1 or tuple(out.shape) != (n, c):
        raise TypeError("out must be an N x c float32/float64 tensor with unit column stride")
    if fixed is not None:
        if not (fixed.is_cuda and fixed.dtype == torch.uint8 and fixed.numel() == n):
            raise TypeError("fixed must be a uint8 CUDA tensor with one entry per cell")
        fixed = fixed.contiguous()
    terms = make_terms(sigma, order, alpha)
    L.check(L.lib().gift_filter_placement(graph.handle, terms, len(terms), _ptr(x), c,
                                          x.stride(0), TORCH_DTYPES[x.dtype], _ptr(out),
                                          out.stride(0), TORCH_DTYPES[out.dtype], _ptr(fixed),
                                          _stream_handle(stream)),
            "gift_filter_placement")
    return out


def profile_enable(on: bool = True):
    """Turn the library's per-launch event profiler on or off."""
    L.check(L.lib().gift_profile_enable(1 if on else 0), "gift_profile_enable")


def profile_collect(kind: str) -> dict:
    """Launch count, device time and algorithmic bytes recorded for one kernel
    class ("spmm", "spmm_final" or "build") since the last collect."""
    cls = {"spmm": L.GIFT_PROF_SPMM, "spmm_final": L.GIFT_PROF_SPMM_FINAL,
           "build": L.GIFT_PROF_BUILD}[kind]
    n = C.c_int64()
    tot = C.c_double()
    mx = C.c_double()
    by = C.c_double()
    L.check(L.lib().gift_profile_collect(cls, C.byref(n), C.byref(tot), C.byref(mx), C.byref(by)),
            "gift_profile_collect")
    return {"launches": n.value, "total_ms": tot.value, "max_ms": mx.value, "bytes": by.value}
