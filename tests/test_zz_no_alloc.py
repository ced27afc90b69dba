"""The allocation-free filter entry point against gift_filter_placement,
called through the C ABI (needs a GPU): bit-identical results on two calls in
a row (the second on a smaller design), no device allocation by the call, and
a clear refusal past the scratch size."""
import ctypes as C

import numpy as np
import pytest

from paper_2502_17632_amd import _lib as L
from paper_2502_17632_amd import workload as W

pytestmark = pytest.mark.gpu

TERMS = ([4.0] * 5, [1, 2, 4, 8, 16], [0.2] * 5)


def call(name, g, terms, x, y, fixed=None):
    import torch
    fn = getattr(L.lib(), name)
    st = fn(g.handle, terms, len(terms), C.c_void_p(x.data_ptr()), x.shape[1], x.stride(0),
            L.GIFT_F32, C.c_void_p(y.data_ptr()), y.stride(0), L.GIFT_F32,
            None if fixed is None else C.c_void_p(fixed.data_ptr()),
            C.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st


def test_no_alloc_matches_and_allocates_nothing():
    import torch
    import paper_2502_17632_amd as gift
    from paper_2502_17632_amd.api import make_terms
    terms = make_terms(*TERMS)
    cases = []
    for nl, storage, fixed in ((W.medium(), "f32", True), (W.tiny(seed=3), "bf16", False)):
        g = gift.build_graph(nl.num_cells, nl.net_ptr, nl.pin_cell, star_threshold=16,
                             storage=storage, sigmas=[4.0])
        x = torch.tensor(W.make_signal(nl), dtype=torch.float32, device="cuda")
        fx = torch.tensor(nl.fixed, device="cuda") if fixed else None
        ref = torch.empty_like(x)
        assert call("gift_filter_placement", g, terms, x, ref, fx) == L.GIFT_OK
        cases.append((g, x, fx, ref))
    torch.cuda.synchronize()
    outs = [torch.full_like(ref, float("nan")) for _, _, _, ref in cases]
    held0 = (C.c_int64(), C.c_int64())
    L.lib().gift_memory_stats(C.byref(held0[0]), C.byref(held0[1]))
    torch_before = torch.cuda.memory_allocated()
    for (g, x, fx, ref), y in zip(cases, outs):  # the second call is the smaller design
        print(f"[no-alloc] rows={g.info()['num_rows']} storage={g.info()['storage']}", flush=True)
        st = call("gift_filter_placement_noalloc", g, terms, x, y, fx)
        assert st == L.GIFT_OK, L.lib().gift_last_error()
    torch.cuda.synchronize()
    held1 = (C.c_int64(), C.c_int64())
    L.lib().gift_memory_stats(C.byref(held1[0]), C.byref(held1[1]))
    assert held1[0].value == held0[0].value and held1[1].value == held0[1].value
    assert torch.cuda.memory_allocated() == torch_before
    for (g, _, _, ref), y in zip(cases, outs):
        assert torch.equal(y, ref)
    # once more, large then small again: the array keeps the last call's
    # contents, which must not leak into the next result
    for (g, x, fx, ref), y in zip(cases, outs):
        y.fill_(float("nan"))
        assert call("gift_filter_placement_noalloc", g, terms, x, y, fx) == L.GIFT_OK
    torch.cuda.synchronize()
    for (_, _, _, ref), y in zip(cases, outs):
        assert torch.equal(y, ref)
    for g, *_ in cases:
        g.close()


def test_no_alloc_refuses_inputs_past_its_scratch():
    import torch
    import paper_2502_17632_amd as gift
    from paper_2502_17632_amd.api import make_terms
    rows = 3_000_000  # 16 columns: x0, ping, pong of 64 bytes per row exceed 128 MiB
    g = gift.import_csr(np.zeros(rows + 1, dtype=np.int64), np.zeros(0, dtype=np.int32),
                        np.zeros(0), sigmas=[4.0])
    x = torch.zeros(rows, 16, device="cuda")
    y = torch.zeros_like(x)
    terms = make_terms([4.0], [2], [1.0])
    st = call("gift_filter_placement_noalloc", g, terms, x, y)
    assert st == L.GIFT_EUNSUPPORTED
    msg = L.lib().gift_last_error().decode()
    assert "scratch holds" in msg, msg
    print(f"[no-alloc] refused: {msg}", flush=True)
    g.close()
