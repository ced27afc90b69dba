"""gift_set_allocator (needs a GPU): with a counting allocator installed
through the C ABI, every device allocation of build, import, filter, exact
filter, evaluators, eigen placement, density, batch and server goes through
it (the library's own pool does not grow) and every block comes back; results
are bit-identical to the library's own cache; torch's caching allocator can
serve the library."""
import ctypes as C

import numpy as np
import pytest

from paper_2502_17632_amd import _lib as L
from paper_2502_17632_amd import workload as W

pytestmark = pytest.mark.gpu

EQ4 = ([4.0] * 4, [1, 2, 4, 8], [0.25] * 4)


class Counting:
    """A C-ABI allocator (ctypes callbacks) that takes its blocks from torch and
    counts them."""

    def __init__(self):
        import torch
        self.live = {}
        self.allocs = 0
        self.frees = 0
        self.bad_frees = 0

        def alloc(nbytes, device, stream, ctx):
            t = torch.empty(int(nbytes), dtype=torch.uint8, device=f"cuda:{int(device)}")
            self.live[t.data_ptr()] = (t, int(nbytes), int(stream or 0))
            self.allocs += 1
            return t.data_ptr()

        def free(ptr, nbytes, device, stream, ctx):
            ent = self.live.pop(ptr, None)
            if ent is None or ent[1] != int(nbytes):
                self.bad_frees += 1
                return
            self.frees += 1
            # the tensor's memory may be reused by torch on its allocation
            # stream: wait for the stream the library freed the block on
            torch.cuda.synchronize()

        self.fns = (L.ALLOC_FN(alloc), L.FREE_FN(free))
        self.struct = L.Allocator(self.fns[0], self.fns[1], None)


def pool_stats():
    held, used = C.c_int64(), C.c_int64()
    L.lib().gift_memory_stats(C.byref(held), C.byref(used))
    return held.value, used.value


def workload_once(gift, torch):
    nl = W.sized(30_000, seed=77)
    x = torch.tensor(W.make_signal(nl), dtype=torch.float32, device="cuda")
    fx = torch.tensor(nl.fixed, device="cuda")
    outs = {}
    g = gift.build_graph(nl.num_cells, nl.net_ptr, nl.pin_cell, star_threshold=16,
                         storage="f32", sigmas=[2.0, 4.0])
    outs["filter"] = gift.filter_placement(g, *EQ4, x, fixed=fx)
    outs["exact"], _ = gift.filter_exact(g, 4.0, x, tol=1e-6)
    m = gift.evaluate_placement(g, outs["filter"], torch.tensor(nl.net_ptr, device="cuda"),
                                torch.tensor(nl.pin_cell, device="cuda"))
    outs["smooth"] = torch.tensor(m["smoothness"])
    outs["eigen"], _ = gift.eigen_placement(g, tol=1e-6, max_iter=60)
    outs["density"] = gift.bin_density(outs["filter"], (0.0, 0.0, W.DIE, W.DIE), 64, 64)
    # a graph without edges through the import path
    gi = gift.import_csr(np.zeros(nl.num_cells + 1, np.int64), np.zeros(0, np.int32),
                         np.zeros(0), sigmas=[4.0])
    outs["import"] = gift.filter_placement(gi, [4.0], [2], [1.0], x)
    gi.close()
    nl2 = W.sized(12_000, seed=78)
    g2 = gift.build_graph(nl2.num_cells, nl2.net_ptr, nl2.pin_cell, star_threshold=16,
                          storage="f32", sigmas=[4.0])
    x2 = torch.tensor(W.make_signal(nl2), dtype=torch.float32, device="cuda")
    b = gift.Batch([g, g2], *EQ4, num_cols=2, tune=0)
    ys = b.run([x, x2])
    outs["batch0"], outs["batch1"] = ys
    torch.cuda.synchronize()
    b.close()
    srv = gift.Server(*EQ4, num_cols=2, hbm_budget_bytes=4 << 30, num_builders=1, num_streams=2)
    tickets = [srv.submit(i, n.num_cells, n.net_ptr, n.pin_cell, xx)
               for i, (n, xx) in enumerate([(nl, x), (nl2, x2), (nl, x)])]
    for t, y in tickets:
        srv.wait(t)
    outs["served"] = tickets[2][1]
    srv.close()
    torch.cuda.synchronize()
    g.close()
    g2.close()
    torch.cuda.synchronize()
    return outs


def test_counting_allocator_sees_every_block():
    import torch
    import paper_2502_17632_amd as gift
    ref = workload_once(gift, torch)  # the library's own cache
    held0, used0 = pool_stats()
    cnt = Counting()
    assert L.lib().gift_set_allocator(C.byref(cnt.struct)) == L.GIFT_OK
    try:
        got = workload_once(gift, torch)
    finally:
        assert L.lib().gift_set_allocator(None) == L.GIFT_OK
    held1, used1 = pool_stats()
    print(f"[allocator] {cnt.allocs} allocations, {cnt.frees} frees, pool held "
          f"{held0} -> {held1} bytes", flush=True)
    assert cnt.allocs > 50 and cnt.frees == cnt.allocs and not cnt.live and cnt.bad_frees == 0
    assert held1 == held0 and used1 == used0  # nothing bypassed the hook
    for k in ref:
        assert torch.equal(ref[k], got[k]), k


def test_torch_caching_allocator_serves_the_library():
    import torch
    import paper_2502_17632_amd as gift
    held0, _ = pool_stats()
    ta = gift.use_torch_allocator(True)
    try:
        nl = W.sized(40_000, seed=79)
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        g = gift.build_graph(nl.num_cells, nl.net_ptr, nl.pin_cell, star_threshold=16,
                             sigmas=[4.0])
        torch.cuda.synchronize()
        resident = torch.cuda.memory_allocated() - before
        assert resident >= g.info()["bytes_resident"] > 0
        x = torch.tensor(W.make_signal(nl), dtype=torch.float32, device="cuda")
        y = gift.filter_placement(g, *EQ4, x)
        g.close()
        torch.cuda.synchronize()
        assert ta.allocs == ta.frees and ta.live_bytes == 0
        assert torch.isfinite(y).all()
    finally:
        gift.use_torch_allocator(False)
    assert pool_stats()[0] == held0
