"""ctypes wrapper over the C oracle (test infrastructure only).

Only the tests, the package smoke check and the benchmark's CPU-baseline leg
may use this module.  Every array it returns is float64 / int64 / int32 numpy.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
from typing import Optional, Sequence

import numpy as np

from . import build as _build

_lib = None


def load(path: Optional[str] = None):
    """Load the oracle library, compiling it first if nothing is built."""
    global _lib
    if path is None and _lib is not None:
        return _lib
    p = path or _build.LIB
    if not os.path.exists(p):
        _build.build(p)
    lib = C.CDLL(p)
    i64, i32 = C.c_int64, C.c_int32
    vp = C.c_void_p
    lib.oracle_build.argtypes = [i64, i64, i64, vp, vp, C.c_int, i64, C.POINTER(vp)]
    lib.oracle_build.restype = C.c_int
    lib.oracle_build_ordered.argtypes = [i64, i64, i64, vp, vp, C.c_int, i64, C.c_int,
                                         C.POINTER(vp)]
    lib.oracle_build_ordered.restype = C.c_int
    lib.oracle_free.argtypes = [vp]
    lib.oracle_free.restype = None
    lib.oracle_sizes.argtypes = [vp, vp]
    lib.oracle_sizes.restype = None
    lib.oracle_export.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.oracle_export.restype = None
    lib.oracle_normalise.argtypes = [vp, C.c_double, vp, vp]
    lib.oracle_normalise.restype = C.c_int
    lib.oracle_filter.argtypes = [vp, i64, vp, vp, vp, vp, i64, vp, vp]
    lib.oracle_filter.restype = C.c_int
    lib.oracle_evaluate.argtypes = [vp, vp, i64, vp, vp, vp]
    lib.oracle_evaluate.restype = C.c_int
    lib.oracle_filter_exact.argtypes = [vp, C.c_double, vp, i64, C.c_double, i64, vp, vp, vp]
    lib.oracle_filter_exact.restype = C.c_int
    lib.oracle_bin_density.argtypes = [i64, vp, vp, vp, C.c_double, C.c_double, C.c_double,
                                       C.c_double, i64, i64, vp]
    lib.oracle_bin_density.restype = C.c_int
    lib.oracle_density_overflow.argtypes = [vp, i64, i64, C.c_double, C.c_double, C.c_double,
                                            C.c_double, C.c_double, C.c_double, vp]
    lib.oracle_density_overflow.restype = C.c_int
    lib.oracle_import_csr.argtypes = [i64, i64, vp, vp, vp, C.POINTER(vp)]
    lib.oracle_import_csr.restype = C.c_int
    if path is None:
        _lib = lib
    return lib


class OracleError(RuntimeError):
    pass


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


W_INV_M1 = 0
W_TWO_OVER_M = 1


@dataclasses.dataclass
class OracleGraph:
    num_cells: int
    num_virtual: int
    row_ptr: np.ndarray  # int64[R+1]
    col: np.ndarray  # int32[nnz]
    w: np.ndarray  # float64[nnz]
    deg: np.ndarray  # float64[R]
    virt_net: np.ndarray  # int32[V]
    handle: "C.c_void_p" = None
    lib: object = None

    @property
    def num_rows(self) -> int:
        return self.num_cells + self.num_virtual

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def close(self):
        if self.handle is not None:
            self.lib.oracle_free(self.handle)
            self.handle = None

    def __del__(self):  # pragma: no cover - best effort
        try:
            self.close()
        except Exception:
            pass

    def normalise(self, sigma: float):
        a = np.empty(self.nnz, dtype=np.float64)
        d = np.empty(self.num_rows, dtype=np.float64)
        rc = self.lib.oracle_normalise(self.handle, float(sigma), _ptr(a), _ptr(d))
        if rc:
            raise OracleError(f"oracle_normalise failed ({rc})")
        return a, d

    def filter(self, x: np.ndarray, sigma: Sequence[float], order: Sequence[int],
               alpha: Sequence[float], fixed: Optional[np.ndarray] = None) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64)
        if x.ndim == 1:
            x = x[:, None]
        if x.shape[0] != self.num_cells:
            raise OracleError("signal rows != cells")
        c = x.shape[1]
        s = np.ascontiguousarray(sigma, dtype=np.float64)
        k = np.ascontiguousarray(order, dtype=np.int32)
        al = np.ascontiguousarray(alpha, dtype=np.float64)
        if not (s.shape == k.shape == al.shape):
            raise OracleError("term arrays differ in length")
        fx = None if fixed is None else np.ascontiguousarray(fixed, dtype=np.uint8)
        y = np.empty_like(x)
        rc = self.lib.oracle_filter(self.handle, s.shape[0], _ptr(s), _ptr(k), _ptr(al),
                                    _ptr(x), c, _ptr(fx), _ptr(y))
        if rc:
            raise OracleError(f"oracle_filter failed ({rc})")
        return y


    def filter_exact(self, x: np.ndarray, sigma: float, tol: float = 1e-14,
                     max_iter: int = 1000, fixed: Optional[np.ndarray] = None):
        """(I + L~_sigma)^-1 x by conjugate gradients (see oracle_filter_exact);
        returns (y, iterations)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        if x.ndim == 1:
            x = x[:, None]
        if x.shape[0] != self.num_cells:
            raise OracleError("signal rows != cells")
        fx = None if fixed is None else np.ascontiguousarray(fixed, dtype=np.uint8)
        y = np.empty_like(x)
        it = np.zeros(1, dtype=np.int64)
        rc = self.lib.oracle_filter_exact(self.handle, float(sigma), _ptr(x), x.shape[1],
                                          float(tol), int(max_iter), _ptr(fx), _ptr(y), _ptr(it))
        if rc:
            raise OracleError(f"oracle_filter_exact failed ({rc})")
        return y, int(it[0])

    def evaluate(self, x: np.ndarray):
        """Per-column (S, norm2, hpwl) of the placement x (see oracle_evaluate)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        if x.ndim == 1:
            x = x[:, None]
        if x.shape[0] != self.num_cells:
            raise OracleError("signal rows != cells")
        c = x.shape[1]
        S, n2, h = (np.empty(c, dtype=np.float64) for _ in range(3))
        rc = self.lib.oracle_evaluate(self.handle, _ptr(x), c, _ptr(S), _ptr(n2), _ptr(h))
        if rc:
            raise OracleError(f"oracle_evaluate failed ({rc})")
        return S, n2, h


STAR_ORDERS = {"net": 0, "median": 1}


def build_graph(num_cells: int, net_ptr: np.ndarray, pin_cell: np.ndarray, *,
                weight_model: int = W_INV_M1, star_threshold: int = 0,
                star_order: str = "net", lib=None) -> OracleGraph:
    """Steps O1-O4 (see oracle_build_ordered).  star_order labels the
    virtual rows N..N+V-1: "net" in ascending net id, "median" in ascending
    median cell of the net (index M/2 of its ascending distinct cells), ties
    by net id."""
    lib = lib or load()
    net_ptr = np.ascontiguousarray(net_ptr, dtype=np.int64)
    pin_cell = np.ascontiguousarray(pin_cell, dtype=np.int32)
    h = C.c_void_p()
    if star_order not in STAR_ORDERS:
        raise OracleError(f"star_order must be one of {sorted(STAR_ORDERS)}")
    rc = lib.oracle_build_ordered(int(num_cells), net_ptr.shape[0] - 1, pin_cell.shape[0],
                                  _ptr(net_ptr), _ptr(pin_cell), int(weight_model),
                                  int(star_threshold), STAR_ORDERS[star_order], C.byref(h))
    if rc:
        raise OracleError(f"oracle_build failed ({rc})")
    sizes = np.zeros(4, dtype=np.int64)
    lib.oracle_sizes(h, _ptr(sizes))
    n, v, r, nnz = (int(t) for t in sizes)
    row_ptr = np.empty(r + 1, dtype=np.int64)
    col = np.empty(nnz, dtype=np.int32)
    w = np.empty(nnz, dtype=np.float64)
    deg = np.empty(r, dtype=np.float64)
    vn = np.empty(v, dtype=np.int32)
    lib.oracle_export(h, _ptr(row_ptr), _ptr(col), _ptr(w), _ptr(deg), _ptr(vn))
    return OracleGraph(n, v, row_ptr, col, w, deg, vn, h, lib)


def import_csr(row_ptr: np.ndarray, col: np.ndarray, w: np.ndarray, lib=None) -> OracleGraph:
    """A caller-supplied weighted graph in canonical CSR (see
    oracle_import_csr): every row is a cell, degrees are summed in ascending
    column."""
    lib = lib or load()
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.float64)
    r = row_ptr.shape[0] - 1
    nnz = col.shape[0]
    if w.shape[0] != nnz or r < 0:
        raise OracleError("row_ptr / col / w sizes disagree")
    h = C.c_void_p()
    rc = lib.oracle_import_csr(r, nnz, _ptr(row_ptr), _ptr(col), _ptr(w), C.byref(h))
    if rc:
        raise OracleError(f"oracle_import_csr failed ({rc})")
    deg = np.empty(r, dtype=np.float64)
    lib.oracle_export(h, None, None, None, _ptr(deg), None)
    return OracleGraph(r, 0, row_ptr.copy(), col.copy(), w.copy(), deg,
                       np.empty(0, dtype=np.int32), h, lib)


def build_netlist(netlist, **kw) -> OracleGraph:
    return build_graph(netlist.num_cells, netlist.net_ptr, netlist.pin_cell, **kw)


def bin_density(x: np.ndarray, w, h, box, nbx: int, nby: int, lib=None) -> np.ndarray:
    """Bin density (see oracle_bin_density): x is N x 2 cell centres, w/h the
    cell widths/heights (arrays or scalars), box = (xl, yl, xh, yh)."""
    lib = lib or load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    n = x.shape[0]
    w = np.ascontiguousarray(np.broadcast_to(np.asarray(w, dtype=np.float64), (n,)))
    h = np.ascontiguousarray(np.broadcast_to(np.asarray(h, dtype=np.float64), (n,)))
    out = np.empty((nby, nbx), dtype=np.float64)
    rc = lib.oracle_bin_density(n, _ptr(x), _ptr(w), _ptr(h), float(box[0]), float(box[1]),
                                float(box[2]), float(box[3]), int(nbx), int(nby), _ptr(out))
    if rc:
        raise OracleError(f"oracle_bin_density failed ({rc})")
    return out


def density_overflow(density: np.ndarray, box, target: float, total_area: float,
                     lib=None) -> float:
    """sum_b max(0, rho_b - target * bin area) / total_area of an nby x nbx
    density map (see oracle_density_overflow)."""
    lib = lib or load()
    d = np.ascontiguousarray(density, dtype=np.float64)
    nby, nbx = d.shape
    out = np.zeros(1, dtype=np.float64)
    rc = lib.oracle_density_overflow(_ptr(d), nbx, nby, float(box[0]), float(box[1]),
                                     float(box[2]), float(box[3]), float(target),
                                     float(total_area), _ptr(out))
    if rc:
        raise OracleError(f"oracle_density_overflow failed ({rc})")
    return float(out[0])
