"""Python binding of the GiFt library: argument marshalling only.

Every computation happens in the HIP library (``libgift.so``); torch is used
for device memory and streams.
"""
from __future__ import annotations

import ctypes as C
import threading
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
        # the device the graph was built on (its memory lives there)
        self.device = torch.device("cuda", torch.cuda.current_device())

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        inf = L.GraphInfo()
        L.check(L.lib().gift_graph_get_info(self._h, C.byref(inf)), "gift_graph_get_info")
        return {k: getattr(inf, k) for k, _ in L.GraphInfo._fields_}

    def set_tile_class(self, tile_class: int):
        L.check(L.lib().gift_graph_set_tile_class(self._h, int(tile_class)),
                "gift_graph_set_tile_class")

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
    # a host netlist's pin count is checked here; a device netlist's by the
    # library, which reads net_ptr[-1] back anyway (reading it here would
    # wait for the stream)
    if mem == L.GIFT_MEM_HOST and int(net_ptr[-1]) != int(pin_cell.shape[0]):
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
    d.num_pins = int(pin_cell.shape[0])
    h = C.c_void_p()
    st = _stream_handle(stream)
    L.check(L.lib().gift_build_graph(C.byref(d), st, C.byref(h)), "gift_build_graph")
    return Graph(h, stream)


def import_csr(row_ptr, col, w, *, storage: str = "f32", sigmas: Iterable[float] = (4.0,),
               stream=None) -> Graph:
    """A caller-supplied weighted graph (canonical CSR of A: int64 row_ptr,
    int32 col strictly ascending per row, float64 weights) -> resident graph.
    The arrays may be numpy arrays (host) or CUDA tensors (device)."""
    arrs = (row_ptr, col, w)
    on_dev = [isinstance(a, torch.Tensor) for a in arrs]
    if any(on_dev) and not all(on_dev):
        raise TypeError("row_ptr, col and w must all be numpy arrays or all tensors")
    if all(on_dev):
        if not all(a.is_cuda for a in arrs):
            raise TypeError("tensors must live on the GPU")
        if (row_ptr.dtype, col.dtype, w.dtype) != (torch.int64, torch.int32, torch.float64):
            raise TypeError("row_ptr must be int64, col int32 and w float64")
        row_ptr, col, w = row_ptr.contiguous(), col.contiguous(), w.contiguous()
        mem = L.GIFT_MEM_DEVICE
    else:
        row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int32)
        w = np.ascontiguousarray(w, dtype=np.float64)
        mem = L.GIFT_MEM_HOST
    if row_ptr.shape[0] < 1 or col.shape[0] != w.shape[0]:
        raise ValueError("row_ptr needs R + 1 >= 1 entries and col / w the same length")
    sig = np.ascontiguousarray(list(sigmas), dtype=np.float64)
    d = L.CsrDesc()
    d.num_rows = int(row_ptr.shape[0]) - 1
    d.nnz = int(col.shape[0])
    d.row_ptr, d.col, d.w = _ptr(row_ptr), _ptr(col), _ptr(w)
    d.mem_space = mem
    d.storage = DTYPES[storage]
    d.num_sigmas = int(sig.shape[0])
    d.reserved = 0
    d.sigmas = _ptr(sig)
    h = C.c_void_p()
    L.check(L.lib().gift_graph_import_csr(C.byref(d), _stream_handle(stream), C.byref(h)),
            "gift_graph_import_csr")
    return Graph(h, stream)


def filter_placement(graph: Graph, sigma: Sequence[float], order: Sequence[int],
                     alpha: Sequence[float], x: torch.Tensor, *,
                     fixed: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None,
                     out_dtype: torch.dtype = torch.float32, stream=None,
                     no_alloc: bool = False) -> torch.Tensor:
    """g' = sum_t alpha_t A~_{sigma_t}^{order_t} x  (x: N x c CUDA tensor, f32/f64).
    ``no_alloc`` calls the variant whose signal buffers live in the library's
    static scratch (no device allocation; calls on one GPU must not overlap)."""
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
    name = "gift_filter_placement_noalloc" if no_alloc else "gift_filter_placement"
    L.check(getattr(L.lib(), name)(graph.handle, terms, len(terms), _ptr(x), c, x.stride(0),
                                   TORCH_DTYPES[x.dtype], _ptr(out), out.stride(0),
                                   TORCH_DTYPES[out.dtype], _ptr(fixed), _stream_handle(stream)),
            name)
    return out


def filter_exact(graph: Graph, sigma: float, x: torch.Tensor, *, tol: float = 1e-6,
                 max_iter: int = 500, fixed: Optional[torch.Tensor] = None,
                 out: Optional[torch.Tensor] = None, out_dtype: torch.dtype = torch.float32,
                 stream=None) -> Tuple[torch.Tensor, int]:
    """g' = (I + L~_sigma)^-1 x by conjugate gradients; returns (g', iterations)."""
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dim() == 2):
        raise TypeError("x must be a 2-D CUDA tensor")
    if x.stride(1) != 1:
        x = x.contiguous()
    if x.dtype not in TORCH_DTYPES:
        raise TypeError("x must be float32 or float64")
    n, c = x.shape
    if n != graph.info()["num_cells"]:
        raise ValueError("x rows != graph cells")
    if out is None:
        out = torch.empty((n, c), dtype=out_dtype, device=x.device)
    if fixed is not None:
        if not (fixed.is_cuda and fixed.dtype == torch.uint8 and fixed.numel() == n):
            raise TypeError("fixed must be a uint8 CUDA tensor with one entry per cell")
        fixed = fixed.contiguous()
    it = C.c_int64()
    L.check(L.lib().gift_filter_exact(graph.handle, float(sigma), _ptr(x), c, x.stride(0),
                                      TORCH_DTYPES[x.dtype], _ptr(out), out.stride(0),
                                      TORCH_DTYPES[out.dtype], _ptr(fixed), float(tol),
                                      int(max_iter), C.byref(it), _stream_handle(stream)),
            "gift_filter_exact")
    return out, it.value


def eigen_placement(graph: Graph, *, tol: float = 1e-10, max_iter: int = 1000,
                    seed: int = 1, labels: bool = False, stream=None):
    """Eigenvector placement [u_2, u_3] of the clique-model Laplacian on the
    largest connected component (Section 3.3.1).  Returns (N x 2 float64 CUDA
    tensor, info dict[, int32 labels of every graph row])."""
    inf = graph.info()
    n, r = inf["num_cells"], inf["num_rows"]
    dev = graph.device
    out = torch.empty((n, 2), dtype=torch.float64, device=dev)
    lab = torch.empty(r, dtype=torch.int32, device=dev) if labels else None
    res = L.EigenResult()
    with torch.cuda.device(dev):
        L.check(L.lib().gift_eigen_placement(graph.handle, float(tol), int(max_iter),
                                             int(seed) & 0xFFFFFFFFFFFFFFFF, _ptr(out), 2,
                                             _ptr(lab), C.byref(res), _stream_handle(stream)),
                "gift_eigen_placement")
    lam = getattr(res, "lambda")
    info = {"lambda": [lam[0], lam[1]],
            "residual": [res.residual[0], res.residual[1]],
            "spectral_bound": res.spectral_bound, "component_label": res.component_label,
            "component_cells": res.component_cells, "iterations": res.iterations,
            "sweeps": res.sweeps, "converged": bool(res.converged)}
    return (out, info, lab) if labels else (out, info)


def bin_density(x: torch.Tensor, box: Sequence[float], nbx: int, nby: int, *,
                widths: Optional[torch.Tensor] = None, heights: Optional[torch.Tensor] = None,
                w0: float = 1.0, h0: float = 1.0, stream=None) -> torch.Tensor:
    """Bin density map (eq. density_eq) of the centres x[:, 0:2] as an
    nby x nbx float64 CUDA tensor; box = (xl, yl, xh, yh)."""
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dim() == 2 and x.shape[1] >= 2):
        raise TypeError("x must be an N x (>= 2) CUDA tensor")
    if x.dtype not in TORCH_DTYPES:
        raise TypeError("x must be float32 or float64")
    if x.stride(1) != 1:
        x = x.contiguous()
    n = x.shape[0]
    for t in (widths, heights):
        if t is not None and not (t.is_cuda and t.dtype == torch.float64 and t.numel() == n):
            raise TypeError("widths/heights must be float64 CUDA tensors with one entry per object")
    widths = None if widths is None else widths.contiguous()
    heights = None if heights is None else heights.contiguous()
    out = torch.empty((int(nby), int(nbx)), dtype=torch.float64, device=x.device)
    xl, yl, xh, yh = (float(v) for v in box)
    L.check(L.lib().gift_bin_density(_ptr(x), n, x.stride(0) if n else 2, TORCH_DTYPES[x.dtype],
                                     _ptr(widths), _ptr(heights), float(w0), float(h0), xl, yl,
                                     xh, yh, int(nbx), int(nby), _ptr(out),
                                     _stream_handle(stream)), "gift_bin_density")
    return out


def density_overflow(density: torch.Tensor, box: Sequence[float], target: float,
                     total_area: float, stream=None) -> float:
    """sum_b max(0, rho_b - target * bin area) / total object area of a
    density map from ``bin_density`` (computed by the library)."""
    if not (isinstance(density, torch.Tensor) and density.is_cuda and density.dim() == 2
            and density.dtype == torch.float64):
        raise TypeError("density must be a 2-D float64 CUDA tensor")
    density = density.contiguous()
    nby, nbx = density.shape
    out = C.c_double()
    L.check(L.lib().gift_density_overflow(_ptr(density), nbx, nby, float(box[0]), float(box[1]),
                                          float(box[2]), float(box[3]), float(target),
                                          float(total_area), C.byref(out),
                                          _stream_handle(stream)),
            "gift_density_overflow")
    return out.value


def evaluate_placement(graph: Graph, x: torch.Tensor, net_ptr=None, pin_cell=None,
                       stream=None) -> dict:
    """Per-column smoothness S (eq. smoothness / wire_eq), squared norm,
    Rayleigh quotient S / norm2 (eq. smoothness_ray) and, when the netlist is
    given (numpy or CUDA tensors), half-perimeter wirelength, in float64."""
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dim() == 2):
        raise TypeError("x must be a 2-D CUDA tensor")
    if x.dtype not in TORCH_DTYPES:
        raise TypeError("x must be float32 or float64")
    if x.stride(1) != 1:
        x = x.contiguous()
    n, c = x.shape
    if n != graph.info()["num_cells"]:
        raise ValueError("x rows != graph cells")
    S = np.zeros(c)
    n2 = np.zeros(c)
    rq = np.zeros(c)
    h = np.zeros(c) if net_ptr is not None else None
    np_d = pc_d = None
    E = P = 0
    if net_ptr is not None:
        np_d = torch.as_tensor(np.asarray(net_ptr, dtype=np.int64) if not isinstance(
            net_ptr, torch.Tensor) else net_ptr, device=x.device).to(torch.int64).contiguous()
        pc_d = torch.as_tensor(np.asarray(pin_cell, dtype=np.int32) if not isinstance(
            pin_cell, torch.Tensor) else pin_cell, device=x.device).to(torch.int32).contiguous()
        E = np_d.shape[0] - 1
        P = pc_d.shape[0]
    L.check(L.lib().gift_evaluate_placement(graph.handle, _ptr(x), c, x.stride(0),
                                            TORCH_DTYPES[x.dtype], _ptr(np_d), _ptr(pc_d), E, P,
                                            _ptr(S), _ptr(n2), _ptr(rq), _ptr(h),
                                            _stream_handle(stream)),
            "gift_evaluate_placement")
    out = {"smoothness": S, "norm2": n2, "rayleigh": rq}
    if h is not None:
        out["hpwl"] = h
    return out


class Batch:
    """Many resident graphs filtered with the same terms and column count by
    one captured launch sequence (``gift_batch_create``).  The graphs must
    outlive the batch."""

    def __init__(self, graphs: Sequence[Graph], sigma: Sequence[float], order: Sequence[int],
                 alpha: Sequence[float], num_cols: int, *, in_dtype=torch.float32,
                 out_dtype=torch.float32, tune: int = 1, stream=None):
        if len(graphs) < 1:
            raise ValueError("a batch needs at least one graph")
        self._graphs = list(graphs)  # keeps the graphs alive
        self._cells = [g.info()["num_cells"] for g in self._graphs]
        self.num_cols = int(num_cols)
        self.in_dtype, self.out_dtype = in_dtype, out_dtype
        handles = (C.c_void_p * len(graphs))(*[g.handle for g in graphs])
        terms = make_terms(sigma, order, alpha)
        h = C.c_void_p()
        L.check(L.lib().gift_batch_create(handles, len(graphs), terms, len(terms), self.num_cols,
                                          TORCH_DTYPES[in_dtype], TORCH_DTYPES[out_dtype],
                                          int(tune), _stream_handle(stream), C.byref(h)),
                "gift_batch_create")
        self._h = h

    def info(self) -> dict:
        inf = L.BatchInfo()
        L.check(L.lib().gift_batch_get_info(self._h, C.byref(inf)), "gift_batch_get_info")
        out = {k: getattr(inf, k) for k, _ in L.BatchInfo._fields_
               if not k.startswith("cand_") and k != "reserved"}
        n = inf.num_candidates
        out["candidates"] = [{"tile_class": inf.cand_tile_class[i],
                              "chunk_cols": inf.cand_chunk_cols[i],
                              "xcd_affine": inf.cand_xcd_affine[i], "ms": inf.cand_ms[i]}
                             for i in range(n)]
        return out

    def run(self, xs: Sequence[torch.Tensor], outs: Optional[Sequence[torch.Tensor]] = None,
            fixed: Optional[Sequence[Optional[torch.Tensor]]] = None, stream=None):
        """Filters every graph's signal xs[g] (N_g x num_cols) into outs[g]."""
        ng = len(self._graphs)
        if len(xs) != ng:
            raise ValueError(f"{len(xs)} signals for {ng} graphs")
        if outs is None:
            outs = [torch.empty((n, self.num_cols), dtype=self.out_dtype, device=x.device)
                    for n, x in zip(self._cells, xs)]
        io = (L.BatchIO * ng)()
        keep = []
        for g in range(ng):
            x, y = xs[g], outs[g]
            n = self._cells[g]
            if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == self.in_dtype
                    and x.dim() == 2 and tuple(x.shape) == (n, self.num_cols)
                    and (n == 0 or x.stride(1) == 1)):
                raise TypeError(f"xs[{g}] must be a {n} x {self.num_cols} {self.in_dtype} CUDA "
                                "tensor with unit column stride")
            if not (isinstance(y, torch.Tensor) and y.is_cuda and y.dtype == self.out_dtype
                    and tuple(y.shape) == (n, self.num_cols) and (n == 0 or y.stride(1) == 1)):
                raise TypeError(f"outs[{g}] must be a {n} x {self.num_cols} {self.out_dtype} "
                                "CUDA tensor with unit column stride")
            f = None if fixed is None else fixed[g]
            if f is not None:
                if not (f.is_cuda and f.dtype == torch.uint8 and f.numel() == n):
                    raise TypeError(f"fixed[{g}] must be a uint8 CUDA tensor with {n} entries")
                f = f.contiguous()
                keep.append(f)
            io[g].x_in = _ptr(x)
            io[g].ld_in = x.stride(0) if n > 0 else self.num_cols
            io[g].y_out = _ptr(y)
            io[g].ld_out = y.stride(0) if n > 0 else self.num_cols
            io[g].fixed_mask = _ptr(f)
        L.check(L.lib().gift_batch_run(self._h, io, _stream_handle(stream)), "gift_batch_run")
        return outs

    def close(self):
        if self._h is not None:
            L.check(L.lib().gift_batch_destroy(self._h), "gift_batch_destroy")
            self._h = None

    def __del__(self):  # pragma: no cover - best effort
        try:
            if self._h is not None and torch.cuda.is_initialized():
                self.close()
        except Exception:
            pass


class Server:
    """The library's request-serving engine (``gift_server_create``): designs'
    graphs stay resident, requests are admitted by a device-memory budget and
    batched continuously.  ``submit`` returns a ticket; ``wait`` returns the
    request's timing."""

    def __init__(self, sigma: Sequence[float], order: Sequence[int], alpha: Sequence[float],
                 num_cols: int, *, hbm_budget_bytes: int = 200 << 30, max_inflight: int = 64,
                 num_streams: int = 4, num_builders: int = 2, max_batch: int = 32,
                 max_batch_rows: int = 4_000_000, storage: str = "f32",
                 weight_model: str = "inv_m1", star_threshold: int = 16,
                 in_dtype=torch.float32, out_dtype=torch.float32):
        self._terms = make_terms(sigma, order, alpha)
        cfg = L.ServerConfig()
        cfg.hbm_budget_bytes = int(hbm_budget_bytes)
        cfg.max_inflight = int(max_inflight)
        cfg.num_streams = int(num_streams)
        cfg.num_builders = int(num_builders)
        cfg.max_batch = int(max_batch)
        cfg.max_batch_rows = int(max_batch_rows)
        cfg.storage = DTYPES[storage]
        cfg.weight_model = WEIGHT_MODELS[weight_model]
        cfg.star_threshold = int(star_threshold)
        cfg.num_cols = int(num_cols)
        cfg.in_dtype = TORCH_DTYPES[in_dtype]
        cfg.out_dtype = TORCH_DTYPES[out_dtype]
        cfg.num_terms = len(self._terms)
        cfg.terms = C.addressof(self._terms)
        self.num_cols, self.in_dtype, self.out_dtype = int(num_cols), in_dtype, out_dtype
        h = C.c_void_p()
        L.check(L.lib().gift_server_create(C.byref(cfg), C.byref(h)), "gift_server_create")
        self._h = h
        self._keep = {}  # ticket -> buffers that must outlive the request

    def submit(self, design_id: int, num_cells: int, net_ptr: np.ndarray, pin_cell: np.ndarray,
               x: torch.Tensor, out: Optional[torch.Tensor] = None,
               fixed: Optional[torch.Tensor] = None):
        """Queue one request; returns (ticket, output tensor)."""
        net_ptr = np.ascontiguousarray(net_ptr, dtype=np.int64)
        pin_cell = np.ascontiguousarray(pin_cell, dtype=np.int32)
        if net_ptr.ndim != 1 or net_ptr.shape[0] < 1 or int(net_ptr[-1]) != pin_cell.shape[0]:
            raise ValueError("net_ptr must hold num_nets + 1 offsets ending at len(pin_cell)")
        n = int(num_cells)
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == self.in_dtype
                and tuple(x.shape) == (n, self.num_cols) and (n == 0 or x.stride(1) == 1)):
            raise TypeError(f"x must be a {n} x {self.num_cols} {self.in_dtype} CUDA tensor "
                            "with unit column stride")
        if out is None:
            out = torch.empty((n, self.num_cols), dtype=self.out_dtype, device=x.device)
        if not (out.is_cuda and out.dtype == self.out_dtype and tuple(out.shape) ==
                (n, self.num_cols) and (n == 0 or out.stride(1) == 1)):
            raise TypeError("out does not match the request")
        if fixed is not None:
            if not (fixed.is_cuda and fixed.dtype == torch.uint8 and fixed.numel() == n):
                raise TypeError("fixed must be a uint8 CUDA tensor with one entry per cell")
            fixed = fixed.contiguous()
        r = L.Request()
        r.design_id = int(design_id)
        r.num_cells = n
        r.num_nets = int(net_ptr.shape[0]) - 1
        r.net_ptr = _ptr(net_ptr)
        r.pin_cell = _ptr(pin_cell) if pin_cell.shape[0] else _ptr(np.zeros(1, np.int32))
        r.x_in = _ptr(x)
        r.ld_in = x.stride(0) if n else self.num_cols
        r.y_out = _ptr(out)
        r.ld_out = out.stride(0) if n else self.num_cols
        r.fixed_mask = _ptr(fixed)
        t = C.c_uint64()
        L.check(L.lib().gift_server_submit(self._h, C.byref(r), C.byref(t)), "gift_server_submit")
        self._keep[t.value] = (net_ptr, pin_cell, x, out, fixed)
        return t.value, out

    def wait(self, ticket: int, timeout_s: float = -1.0) -> dict:
        res = L.RequestResult()
        st = L.lib().gift_server_wait(self._h, int(ticket), float(timeout_s), C.byref(res))
        if st == L.GIFT_EBUSY:
            raise TimeoutError(f"request {ticket} not finished")
        self._keep.pop(int(ticket), None)
        L.check(st, "gift_server_wait")
        return {k: getattr(res, k) for k, _ in L.RequestResult._fields_}

    def stats(self, reset: bool = False) -> dict:
        st = L.ServerStats()
        L.check(L.lib().gift_server_get_stats(self._h, 1 if reset else 0, C.byref(st)),
                "gift_server_get_stats")
        return {k: getattr(st, k) for k, _ in L.ServerStats._fields_}

    def close(self):
        if self._h is not None:
            L.check(L.lib().gift_server_destroy(self._h), "gift_server_destroy")
            self._h = None
            self._keep.clear()

    def __del__(self):  # pragma: no cover - best effort
        try:
            if self._h is not None and torch.cuda.is_initialized():
                self.close()
        except Exception:
            pass


class TorchAllocator:
    """The library's device allocator hook (gift_set_allocator) served by
    torch's caching allocator, so library memory counts against torch's pool
    and budget.  A block freed on a stream other than the one it was
    allocated for is released only after that stream's queued work is done
    (torch may reuse a freed block at once on its allocation stream)."""

    def __init__(self):
        self._lock = threading.Lock()
        self._stream_of = {}
        self.allocs = 0
        self.frees = 0
        self.live_bytes = 0

        def _alloc(nbytes, device, stream, ctx):
            try:
                with torch.cuda.device(int(device)):
                    p = torch.cuda.caching_allocator_alloc(int(nbytes), device=int(device),
                                                           stream=int(stream or 0))
            except Exception:  # pragma: no cover - reported as GIFT_ENOMEM
                return None
            with self._lock:
                self._stream_of[p] = (int(stream or 0), int(device), int(nbytes))
                self.allocs += 1
                self.live_bytes += int(nbytes)
            return p

        def _free(ptr, nbytes, device, stream, ctx):
            with self._lock:
                a_stream, dev, size = self._stream_of.pop(ptr)
                self.frees += 1
                self.live_bytes -= size
            s = int(stream or 0)
            if s != a_stream:
                with torch.cuda.device(dev):
                    if s:
                        torch.cuda.ExternalStream(s).synchronize()
                    else:
                        torch.cuda.synchronize(dev)
            torch.cuda.caching_allocator_delete(ptr)

        self._fns = (L.ALLOC_FN(_alloc), L.FREE_FN(_free))
        self.struct = L.Allocator(self._fns[0], self._fns[1], None)


_ALLOCATOR = None


def set_allocator(allocator) -> None:
    """Route the library's device allocations to ``allocator`` (an object with
    a ``struct`` field of type ``_lib.Allocator`` whose callbacks it keeps
    alive, e.g. ``TorchAllocator()``); None switches back to the library's
    own cache.  Blocks always go back to the allocator that provided them."""
    global _ALLOCATOR
    if allocator is None:
        L.check(L.lib().gift_set_allocator(None), "gift_set_allocator")
    else:
        L.check(L.lib().gift_set_allocator(C.byref(allocator.struct)), "gift_set_allocator")
    # keep the callbacks alive while the library may call them; the previous
    # allocator stays referenced too (its blocks are returned to it later)
    _ALLOCATOR = (allocator, _ALLOCATOR)


def use_torch_allocator(on: bool = True) -> Optional[TorchAllocator]:
    """Serve the library's device memory from torch's caching allocator (on)
    or from the library's own cache (off)."""
    a = TorchAllocator() if on else None
    set_allocator(a)
    return a


def profile_enable(on: bool = True):
    """Turn the library's per-launch event profiler on or off."""
    L.check(L.lib().gift_profile_enable(1 if on else 0), "gift_profile_enable")


def profile_pause(paused: bool = True):
    """Pause or resume the enabled profiler, keeping its records."""
    L.check(L.lib().gift_profile_pause(1 if paused else 0), "gift_profile_pause")


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
