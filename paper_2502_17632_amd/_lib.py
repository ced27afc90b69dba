"""ctypes declarations of the C ABI in ``include/gift.h``.

Loading fails loudly when ``libgift.so`` has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("GIFT_LIBRARY", os.path.join(HERE, "libgift.so"))

GIFT_OK, GIFT_EINVAL, GIFT_ENOMEM, GIFT_EDEVICE, GIFT_EUNSUPPORTED, GIFT_EBUSY = range(6)
GIFT_F32, GIFT_F64, GIFT_BF16, GIFT_F16 = range(4)
GIFT_W_INV_M1, GIFT_W_TWO_OVER_M = range(2)
GIFT_MEM_HOST, GIFT_MEM_DEVICE = range(2)
GIFT_PROF_SPMM, GIFT_PROF_SPMM_FINAL, GIFT_PROF_BUILD = range(3)


class GraphDesc(C.Structure):
    _fields_ = [
        ("num_cells", C.c_int64),
        ("num_nets", C.c_int64),
        ("net_ptr", C.c_void_p),
        ("pin_cell", C.c_void_p),
        ("mem_space", C.c_int32),
        ("weight_model", C.c_int32),
        ("star_threshold", C.c_int64),
        ("storage", C.c_int32),
        ("num_sigmas", C.c_int32),
        ("sigmas", C.c_void_p),
        ("num_pins", C.c_int64),
    ]


class CsrDesc(C.Structure):
    _fields_ = [
        ("num_rows", C.c_int64),
        ("nnz", C.c_int64),
        ("row_ptr", C.c_void_p),
        ("col", C.c_void_p),
        ("w", C.c_void_p),
        ("mem_space", C.c_int32),
        ("storage", C.c_int32),
        ("num_sigmas", C.c_int32),
        ("reserved", C.c_int32),
        ("sigmas", C.c_void_p),
    ]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_int32, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_int32, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


class Term(C.Structure):
    _fields_ = [("sigma", C.c_double), ("order", C.c_int32), ("reserved", C.c_int32),
                ("alpha", C.c_double)]


class GraphInfo(C.Structure):
    _fields_ = [
        ("num_cells", C.c_int64),
        ("num_virtual", C.c_int64),
        ("num_rows", C.c_int64),
        ("nnz", C.c_int64),
        ("bytes_resident", C.c_int64),
        ("storage", C.c_int32),
        ("num_sigmas", C.c_int32),
    ]


class BatchIO(C.Structure):
    _fields_ = [("x_in", C.c_void_p), ("ld_in", C.c_int64), ("y_out", C.c_void_p),
                ("ld_out", C.c_int64), ("fixed_mask", C.c_void_p)]


BATCH_MAX_CANDIDATES = 8


class BatchInfo(C.Structure):
    _fields_ = [
        ("num_graphs", C.c_int32),
        ("tile_class", C.c_int32),
        ("chunk_cols", C.c_int32),
        ("tuned", C.c_int32),
        ("num_rows", C.c_int64),
        ("nnz", C.c_int64),
        ("num_tiles", C.c_int64),
        ("device_bytes", C.c_int64),
        ("tuned_ms", C.c_double),
        ("num_candidates", C.c_int32),
        ("xcd_affine", C.c_int32),
        ("cand_tile_class", C.c_int32 * BATCH_MAX_CANDIDATES),
        ("cand_chunk_cols", C.c_int32 * BATCH_MAX_CANDIDATES),
        ("cand_ms", C.c_double * BATCH_MAX_CANDIDATES),
        ("cand_xcd_affine", C.c_int32 * BATCH_MAX_CANDIDATES),
    ]


class ServerConfig(C.Structure):
    _fields_ = [
        ("hbm_budget_bytes", C.c_int64),
        ("max_inflight", C.c_int32),
        ("num_streams", C.c_int32),
        ("num_builders", C.c_int32),
        ("max_batch", C.c_int32),
        ("max_batch_rows", C.c_int64),
        ("storage", C.c_int32),
        ("weight_model", C.c_int32),
        ("star_threshold", C.c_int64),
        ("num_cols", C.c_int32),
        ("in_dtype", C.c_int32),
        ("out_dtype", C.c_int32),
        ("num_terms", C.c_int32),
        ("terms", C.c_void_p),
    ]


class Request(C.Structure):
    _fields_ = [
        ("design_id", C.c_uint64),
        ("num_cells", C.c_int64),
        ("num_nets", C.c_int64),
        ("net_ptr", C.c_void_p),
        ("pin_cell", C.c_void_p),
        ("x_in", C.c_void_p),
        ("ld_in", C.c_int64),
        ("y_out", C.c_void_p),
        ("ld_out", C.c_int64),
        ("fixed_mask", C.c_void_p),
    ]


class RequestResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("built", C.c_int32), ("latency_ms", C.c_double),
                ("queue_ms", C.c_double), ("service_ms", C.c_double)]


class ServerStats(C.Structure):
    _fields_ = [
        ("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64),
        ("builds", C.c_int64), ("evictions", C.c_int64),
        ("batches", C.c_int64), ("batched_requests", C.c_int64),
        ("resident_graphs", C.c_int64), ("resident_bytes", C.c_int64),
        ("reserved_bytes", C.c_int64), ("peak_reserved_bytes", C.c_int64),
        ("p50_ms", C.c_double), ("p99_ms", C.c_double), ("mean_ms", C.c_double),
        ("max_ms", C.c_double), ("elapsed_s", C.c_double),
    ]


class EigenResult(C.Structure):
    _fields_ = [
        ("lambda", C.c_double * 2), ("residual", C.c_double * 2),
        ("spectral_bound", C.c_double), ("component_label", C.c_int64),
        ("component_cells", C.c_int64), ("iterations", C.c_int32), ("sweeps", C.c_int32),
        ("converged", C.c_int32), ("reserved", C.c_int32),
    ]


class GiftError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        self.status = status
        super().__init__(f"{where}: status {status}: {message}")


_lib = None

# name -> (restype, argtypes)
SIGNATURES = {
    "gift_build_graph": (C.c_int, [C.POINTER(GraphDesc), C.c_void_p, C.POINTER(C.c_void_p)]),
    "gift_graph_import_csr": (C.c_int, [C.POINTER(CsrDesc), C.c_void_p, C.POINTER(C.c_void_p)]),
    "gift_filter_placement": (C.c_int, [C.c_void_p, C.POINTER(Term), C.c_int32, C.c_void_p,
                                        C.c_int32, C.c_int64, C.c_int32, C.c_void_p, C.c_int64,
                                        C.c_int32, C.c_void_p, C.c_void_p]),
    "gift_filter_placement_noalloc": (C.c_int, [C.c_void_p, C.POINTER(Term), C.c_int32,
                                                C.c_void_p, C.c_int32, C.c_int64, C.c_int32,
                                                C.c_void_p, C.c_int64, C.c_int32, C.c_void_p,
                                                C.c_void_p]),
    "gift_graph_add_sigma": (C.c_int, [C.c_void_p, C.c_double, C.c_void_p]),
    "gift_filter_exact": (C.c_int, [C.c_void_p, C.c_double, C.c_void_p, C.c_int32, C.c_int64,
                                    C.c_int32, C.c_void_p, C.c_int64, C.c_int32, C.c_void_p,
                                    C.c_double, C.c_int64, C.POINTER(C.c_int64), C.c_void_p]),
    "gift_graph_get_info": (C.c_int, [C.c_void_p, C.POINTER(GraphInfo)]),
    "gift_graph_set_tile_class": (C.c_int, [C.c_void_p, C.c_int32]),
    "gift_bin_density": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64, C.c_int32, C.c_void_p,
                                   C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_double,
                                   C.c_double, C.c_double, C.c_int32, C.c_int32, C.c_void_p,
                                   C.c_void_p]),
    "gift_eigen_placement": (C.c_int, [C.c_void_p, C.c_double, C.c_int32, C.c_uint64,
                                       C.c_void_p, C.c_int64, C.c_void_p,
                                       C.POINTER(EigenResult), C.c_void_p]),
    "gift_evaluate_placement": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int64,
                                          C.c_int32, C.c_void_p, C.c_void_p, C.c_int64,
                                          C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                          C.c_void_p, C.c_void_p]),
    "gift_density_overflow": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_double,
                                        C.c_double, C.c_double, C.c_double, C.c_double,
                                        C.c_double, C.POINTER(C.c_double), C.c_void_p]),
    "gift_graph_export": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p]),
    "gift_graph_export_normalised": (C.c_int, [C.c_void_p, C.c_double, C.c_void_p, C.c_void_p,
                                               C.c_void_p]),
    "gift_destroy_graph": (C.c_int, [C.c_void_p, C.c_void_p]),
    "gift_batch_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(Term), C.c_int32,
                                    C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                    C.POINTER(C.c_void_p)]),
    "gift_batch_run": (C.c_int, [C.c_void_p, C.POINTER(BatchIO), C.c_void_p]),
    "gift_batch_get_info": (C.c_int, [C.c_void_p, C.POINTER(BatchInfo)]),
    "gift_batch_destroy": (C.c_int, [C.c_void_p]),
    "gift_server_create": (C.c_int, [C.POINTER(ServerConfig), C.POINTER(C.c_void_p)]),
    "gift_server_submit": (C.c_int, [C.c_void_p, C.POINTER(Request), C.POINTER(C.c_uint64)]),
    "gift_server_wait": (C.c_int, [C.c_void_p, C.c_uint64, C.c_double,
                                   C.POINTER(RequestResult)]),
    "gift_server_get_stats": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(ServerStats)]),
    "gift_server_destroy": (C.c_int, [C.c_void_p]),
    "gift_profile_enable": (C.c_int, [C.c_int32]),
    "gift_profile_pause": (C.c_int, [C.c_int32]),
    "gift_profile_collect": (C.c_int, [C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                       C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "gift_memory_stats": (C.c_int, [C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "gift_release_cached_memory": (C.c_int, []),
    "gift_set_allocator": (C.c_int, [C.POINTER(Allocator)]),
    "gift_status_string": (C.c_char_p, [C.c_int]),
    "gift_last_error": (C.c_char_p, []),
    "gift_abi_version": (C.c_int32, []),
}


def lib():
    """The loaded library (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'` "
            "or `python paper_2502_17632_amd/build_lib.py` first")
    L = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(L, name, None)
        if fn is None:
            continue
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def check(status: int, where: str):
    if status != GIFT_OK:
        msg = lib().gift_last_error().decode(errors="replace")
        raise GiftError(status, where, msg)
