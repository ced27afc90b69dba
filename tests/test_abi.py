"""The C-ABI library loads and exports every symbol ``include/gift.h``
declares; argument checks that return before any device work (no GPU)."""
import ctypes as C
import os
import re

import pytest

from paper_2502_17632_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gift.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gift_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_core_entry_points():
    names = declared_functions()
    for n in ("gift_build_graph", "gift_filter_placement", "gift_destroy_graph"):
        assert n in names


def test_every_declared_symbol_is_exported():
    lib = L.lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_every_declared_symbol_has_a_binding_signature():
    missing = [n for n in declared_functions() if n not in L.SIGNATURES]
    assert not missing, missing


def test_abi_version_and_status_strings():
    lib = L.lib()
    assert lib.gift_abi_version() == 3
    for s in range(6):
        assert lib.gift_status_string(s).startswith(b"GIFT_")
    assert b"unknown" in lib.gift_status_string(99)


STRUCTS = {"gift_graph_desc": L.GraphDesc, "gift_csr_desc": L.CsrDesc, "gift_term": L.Term, "gift_graph_info": L.GraphInfo,
           "gift_batch_io": L.BatchIO, "gift_batch_info": L.BatchInfo,
           "gift_server_config": L.ServerConfig, "gift_request": L.Request,
           "gift_request_result": L.RequestResult, "gift_server_stats": L.ServerStats,
           "gift_eigen_result": L.EigenResult, "gift_allocator": L.Allocator}


def c_layouts(tmp_path):
    """sizeof and every field offset of the header's structs, as the host C
    compiler lays them out."""
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "gift.h"', "int main(void) {"]
    for cname, py in STRUCTS.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "probe"
    import subprocess
    subprocess.run(["gcc", "-std=c99", "-Wall", "-I", os.path.join(ROOT, "include"), str(src),
                    "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return {tuple(line.split()[:2]): int(line.split()[2]) for line in out.splitlines()}


def test_struct_layouts_match_header(tmp_path):
    lay = c_layouts(tmp_path)
    for cname, py in STRUCTS.items():
        assert lay[(cname, "size")] == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert lay[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_null_arguments_are_rejected_without_device_work():
    lib = L.lib()
    out = C.c_void_p()
    assert lib.gift_build_graph(None, None, C.byref(out)) == L.GIFT_EINVAL
    assert b"NULL" in lib.gift_last_error()
    assert lib.gift_build_graph(None, None, None) == L.GIFT_EINVAL
    terms = (L.Term * 1)()
    assert lib.gift_filter_placement(None, terms, 1, None, 2, 2, 0, None, 2, 0, None,
                                     None) == L.GIFT_EINVAL
    info = L.GraphInfo()
    assert lib.gift_graph_get_info(None, C.byref(info)) == L.GIFT_EINVAL
    assert lib.gift_destroy_graph(None, None) == L.GIFT_OK


@pytest.mark.parametrize("field,value", [("num_cells", -1), ("weight_model", 7),
                                         ("storage", 9), ("star_threshold", -2),
                                         ("num_sigmas", 0), ("mem_space", 5)])
def test_bad_descriptor_fields(field, value):
    import numpy as np
    lib = L.lib()
    net_ptr = np.array([0, 2], dtype=np.int64)
    pins = np.array([0, 1], dtype=np.int32)
    sig = np.array([4.0])
    d = L.GraphDesc(num_cells=2, num_nets=1, net_ptr=net_ptr.ctypes.data,
                    pin_cell=pins.ctypes.data, mem_space=L.GIFT_MEM_HOST, weight_model=0,
                    star_threshold=0, storage=0, num_sigmas=1, sigmas=sig.ctypes.data,
                    num_pins=2)
    setattr(d, field, value)
    out = C.c_void_p()
    assert lib.gift_build_graph(C.byref(d), None, C.byref(out)) == L.GIFT_EINVAL
    assert out.value is None


def test_negative_sigma_rejected_before_device_work():
    import numpy as np
    lib = L.lib()
    net_ptr = np.array([0, 2], dtype=np.int64)
    pins = np.array([0, 1], dtype=np.int32)
    for bad in (-1.0, float("nan"), float("inf")):
        sig = np.array([bad])
        d = L.GraphDesc(num_cells=2, num_nets=1, net_ptr=net_ptr.ctypes.data,
                        pin_cell=pins.ctypes.data, mem_space=L.GIFT_MEM_HOST, weight_model=0,
                        star_threshold=0, storage=0, num_sigmas=1, sigmas=sig.ctypes.data,
                    num_pins=2)
        out = C.c_void_p()
        assert lib.gift_build_graph(C.byref(d), None, C.byref(out)) == L.GIFT_EINVAL


def test_host_net_ptr_must_start_at_zero():
    import numpy as np
    lib = L.lib()
    net_ptr = np.array([1, 2], dtype=np.int64)
    pins = np.array([0, 1], dtype=np.int32)
    sig = np.array([4.0])
    d = L.GraphDesc(num_cells=2, num_nets=1, net_ptr=net_ptr.ctypes.data,
                    pin_cell=pins.ctypes.data, mem_space=L.GIFT_MEM_HOST, weight_model=0,
                    star_threshold=0, storage=0, num_sigmas=1, sigmas=sig.ctypes.data,
                    num_pins=2)
    out = C.c_void_p()
    assert lib.gift_build_graph(C.byref(d), None, C.byref(out)) == L.GIFT_EINVAL


def test_pin_count_checked_before_device_work():
    """num_pins: a host netlist whose pin count (net_ptr[num_nets]) differs
    from the stated length of pin_cell, or a num_pins below -1, is rejected
    before any device work."""
    import numpy as np
    lib = L.lib()
    net_ptr = np.array([0, 2, 5], dtype=np.int64)
    pins = np.array([0, 1, 1], dtype=np.int32)
    sig = np.array([4.0])
    for num_pins in (3, 4, -2):
        d = L.GraphDesc(num_cells=3, num_nets=2, net_ptr=net_ptr.ctypes.data,
                        pin_cell=pins.ctypes.data, mem_space=L.GIFT_MEM_HOST, weight_model=0,
                        star_threshold=0, storage=0, num_sigmas=1, sigmas=sig.ctypes.data,
                        num_pins=num_pins)
        out = C.c_void_p()
        assert lib.gift_build_graph(C.byref(d), None, C.byref(out)) == L.GIFT_EINVAL
        assert out.value is None
        assert b"num_pins" in lib.gift_last_error() or b"entries" in lib.gift_last_error()


def test_batch_arguments_rejected_without_device_work():
    lib = L.lib()
    out = C.c_void_p()
    terms = (L.Term * 1)()
    assert lib.gift_batch_create(None, 1, terms, 1, 2, 0, 0, 1, None, C.byref(out)) == L.GIFT_EINVAL
    graphs = (C.c_void_p * 1)()
    assert lib.gift_batch_create(graphs, 0, terms, 1, 2, 0, 0, 1, None, C.byref(out)) == L.GIFT_EINVAL
    assert lib.gift_batch_create(graphs, 1, terms, 0, 2, 0, 0, 1, None, C.byref(out)) == L.GIFT_EINVAL
    assert lib.gift_batch_create(graphs, 1, terms, 1, 0, 0, 0, 1, None, C.byref(out)) == L.GIFT_EINVAL
    assert lib.gift_batch_create(graphs, 1, terms, 1, 2, 2, 0, 1, None,
                                 C.byref(out)) == L.GIFT_EUNSUPPORTED
    assert lib.gift_batch_create(graphs, 1, terms, 1, 2, 0, 0, 4, None, C.byref(out)) == L.GIFT_EINVAL
    assert lib.gift_batch_create(graphs, 1, terms, 1, 2, 0, 0, 1, None, None) == L.GIFT_EINVAL
    assert out.value is None
    io = (L.BatchIO * 1)()
    assert lib.gift_batch_run(None, io, None) == L.GIFT_EINVAL
    info = L.BatchInfo()
    assert lib.gift_batch_get_info(None, C.byref(info)) == L.GIFT_EINVAL
    assert lib.gift_batch_destroy(None) == L.GIFT_OK


def test_server_arguments_rejected_without_device_work():
    lib = L.lib()
    out = C.c_void_p()
    assert lib.gift_server_create(None, C.byref(out)) == L.GIFT_EINVAL
    terms = (L.Term * 1)()
    terms[0].sigma, terms[0].order, terms[0].alpha = 4.0, 2, 1.0
    good = dict(hbm_budget_bytes=1 << 30, max_inflight=4, num_streams=2, num_builders=1,
                max_batch=8, max_batch_rows=1 << 20, storage=0, weight_model=0,
                star_threshold=16, num_cols=2, in_dtype=0, out_dtype=0, num_terms=1,
                terms=C.addressof(terms))
    for field, bad in [("hbm_budget_bytes", 1000), ("max_inflight", 0), ("num_streams", 17),
                       ("num_builders", 0), ("max_batch", 0), ("max_batch_rows", 0),
                       ("storage", 9), ("weight_model", 3), ("star_threshold", -1),
                       ("num_cols", 0), ("num_terms", 0), ("terms", None)]:
        cfg = L.ServerConfig(**good)
        setattr(cfg, field, bad)
        assert lib.gift_server_create(C.byref(cfg), C.byref(out)) == L.GIFT_EINVAL, field
        assert out.value is None
    cfg = L.ServerConfig(**good)
    cfg.in_dtype = 2
    assert lib.gift_server_create(C.byref(cfg), C.byref(out)) == L.GIFT_EUNSUPPORTED
    terms[0].order = 0
    cfg = L.ServerConfig(**good)
    assert lib.gift_server_create(C.byref(cfg), C.byref(out)) == L.GIFT_EINVAL
    r = L.Request()
    t = C.c_uint64()
    assert lib.gift_server_submit(None, C.byref(r), C.byref(t)) == L.GIFT_EINVAL
    assert lib.gift_server_wait(None, 1, 0.0, None) == L.GIFT_EINVAL
    st = L.ServerStats()
    assert lib.gift_server_get_stats(None, 0, C.byref(st)) == L.GIFT_EINVAL
    assert lib.gift_server_destroy(None) == L.GIFT_OK


def test_evaluate_arguments_rejected_without_device_work():
    lib = L.lib()
    out = (C.c_double * 2)()
    assert lib.gift_evaluate_placement(None, None, 2, 2, 0, None, None, 0, 0, out, None, None,
                                       None, None) == L.GIFT_EINVAL


def test_eigen_arguments_rejected_without_device_work():
    lib = L.lib()
    res = L.EigenResult()
    y = (C.c_double * 16)()
    assert lib.gift_eigen_placement(None, 1e-8, 10, 1, y, 2, None, C.byref(res),
                                    None) == L.GIFT_EINVAL
    assert lib.gift_eigen_placement(None, 1e-8, 10, 1, y, 2, None, None, None) == L.GIFT_EINVAL


@pytest.mark.parametrize("field,value", [("num_rows", -1), ("nnz", -3), ("storage", 9),
                                         ("num_sigmas", 0), ("mem_space", 5), ("reserved", 1),
                                         ("num_rows", 1 << 31)])
def test_bad_csr_descriptor_fields(field, value):
    import numpy as np
    lib = L.lib()
    rp = np.array([0, 1, 2], dtype=np.int64)
    col = np.array([1, 0], dtype=np.int32)
    w = np.array([1.0, 1.0])
    sig = np.array([4.0])
    d = L.CsrDesc(num_rows=2, nnz=2, row_ptr=rp.ctypes.data, col=col.ctypes.data,
                  w=w.ctypes.data, mem_space=L.GIFT_MEM_HOST, storage=0, num_sigmas=1,
                  reserved=0, sigmas=sig.ctypes.data)
    setattr(d, field, value)
    out = C.c_void_p()
    st = lib.gift_graph_import_csr(C.byref(d), None, C.byref(out))
    assert st in (L.GIFT_EINVAL, L.GIFT_EUNSUPPORTED) and out.value is None


def test_host_csr_row_ptr_checked_before_device_work():
    import numpy as np
    lib = L.lib()
    col = np.array([1, 0], dtype=np.int32)
    w = np.array([1.0, 1.0])
    sig = np.array([4.0])
    for rp in ([1, 1, 2], [0, 1, 3]):
        rp = np.array(rp, dtype=np.int64)
        d = L.CsrDesc(num_rows=2, nnz=2, row_ptr=rp.ctypes.data, col=col.ctypes.data,
                      w=w.ctypes.data, mem_space=L.GIFT_MEM_HOST, storage=0, num_sigmas=1,
                      reserved=0, sigmas=sig.ctypes.data)
        out = C.c_void_p()
        assert lib.gift_graph_import_csr(C.byref(d), None, C.byref(out)) == L.GIFT_EINVAL
    assert lib.gift_graph_import_csr(None, None, C.byref(out)) == L.GIFT_EINVAL


def test_allocator_needs_both_callbacks():
    lib = L.lib()
    a = L.Allocator()
    assert lib.gift_set_allocator(C.byref(a)) == L.GIFT_EINVAL
    assert lib.gift_set_allocator(None) == L.GIFT_OK


def test_density_overflow_arguments_rejected_without_device_work():
    lib = L.lib()
    out = C.c_double()
    buf = (C.c_double * 4)()
    assert lib.gift_density_overflow(None, 2, 2, 0, 0, 1, 1, 1.0, 1.0, C.byref(out),
                                     None) == L.GIFT_EINVAL
    assert lib.gift_density_overflow(buf, 0, 2, 0, 0, 1, 1, 1.0, 1.0, C.byref(out),
                                     None) == L.GIFT_EINVAL
    assert lib.gift_density_overflow(buf, 2, 2, 0, 0, 1, 1, 1.0, 0.0, C.byref(out),
                                     None) == L.GIFT_EINVAL
    assert lib.gift_density_overflow(buf, 2, 2, 1, 0, 1, 1, 1.0, 1.0, C.byref(out),
                                     None) == L.GIFT_EINVAL
