"""gift_graph_import_csr against the oracle's import of the same CSR (needs a
GPU): a caller-supplied weighted graph (Section 2.1's A = {w_ij}, the input of
Algorithm 1) becomes a resident graph whose degrees are bit-equal to the
oracle's, whose stored normalised values are the oracle's rounded once, and
whose filter matches the oracle's."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2502_17632_amd import workload as W

from parity import TOL, assert_close, check_normalised, log

pytestmark = pytest.mark.gpu

EQ4 = ([4.0] * 4, [1, 2, 4, 8], [0.25] * 4)
PAPER = (W.PAPER_DEFAULT.sigma, W.PAPER_DEFAULT.order, W.PAPER_DEFAULT.alpha)


def check_import(g, og):
    row_ptr, col, w, deg = g.export()
    assert g.info()["num_virtual"] == 0 and g.info()["num_rows"] == og.num_rows
    assert np.array_equal(row_ptr, og.row_ptr) and np.array_equal(col, og.col)
    assert np.array_equal(w.view(np.uint64), og.w.view(np.uint64))
    assert np.array_equal(deg.view(np.uint64), og.deg.view(np.uint64))


def filter_pair(g, og, x, terms, storage):
    import torch
    import paper_2502_17632_amd as gift
    dt = torch.float64 if storage == "f64" else torch.float32
    xin = np.asarray(x, dtype=np.float64)
    if dt == torch.float32:
        xin = xin.astype(np.float32).astype(np.float64)
    y = gift.filter_placement(g, *terms, torch.tensor(xin, dtype=dt, device="cuda"), out_dtype=dt)
    torch.cuda.synchronize()
    return y.double().cpu().numpy(), og.filter(xin, *terms)


def random_weighted(rng, n, density):
    a = np.triu(rng.random((n, n)) * (rng.random((n, n)) < density) * 3.0, 1)
    a = a + a.T
    rows, cols = np.nonzero(a)
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, rows + 1, 1)
    return np.cumsum(rp), cols.astype(np.int32), a[rows, cols]


@pytest.mark.parametrize("storage", ["f32", "bf16", "f64"])
def test_medium_csr_host(storage):
    import paper_2502_17632_amd as gift
    nl = W.medium()
    ob = O.build_netlist(nl, star_threshold=0, star_order="median")
    og = O.import_csr(ob.row_ptr, ob.col, ob.w)
    ob.close()
    log(f"[import] medium clique CSR R={og.num_rows} nnz={og.nnz} storage={storage}")
    g = gift.import_csr(og.row_ptr, og.col, og.w, storage=storage, sigmas=[2.0, 4.0])
    check_import(g, og)
    for s in (2.0, 4.0):
        check_normalised(g, og, s, storage)
    x = W.make_signal(nl)
    y, ref = filter_pair(g, og, x, PAPER if storage != "f64" else EQ4, storage)
    assert_close(y, ref, storage, f"import medium {storage}")
    g.close()
    og.close()


def test_random_weighted_device_arrays():
    import torch
    import paper_2502_17632_amd as gift
    rng = np.random.default_rng(31)
    for n, dens in ((1, 0.0), (7, 0.5), (300, 0.02), (3000, 0.003)):
        rp, col, w = random_weighted(rng, n, dens)
        log(f"[import] random weighted graph n={n} nnz={len(col)} (device arrays)")
        og = O.import_csr(rp, col, w)
        dev = [torch.tensor(a, device="cuda") for a in (rp, col, w)]
        g = gift.import_csr(*dev, storage="f64", sigmas=[0.5, 4.0])
        check_import(g, og)
        check_normalised(g, og, 0.5, "f64")
        x = rng.normal(size=(n, 3)) * 40 + 500
        y, ref = filter_pair(g, og, x, ([0.5, 4.0, 4.0], [3, 1, 6], [0.3, 0.3, 0.4]), "f64")
        assert_close(y, ref, "f64", f"import random n={n}")
        g.close()
        og.close()


def test_isolated_rows_keep_their_signal():
    import torch
    import paper_2502_17632_amd as gift
    rp = np.zeros(4, dtype=np.int64)
    g = gift.import_csr(rp, np.zeros(0, dtype=np.int32), np.zeros(0), storage="f32", sigmas=[4.0])
    x = torch.tensor([[1.0, 2.0], [3.0, 4.0], [5.0, 6.0]], device="cuda")
    y = gift.filter_placement(g, [4.0, 4.0], [1, 3], [0.25, 0.5], x)
    assert torch.equal(y, 0.75 * x)
    g.close()


@pytest.mark.parametrize("case", ["unsorted", "diagonal", "negative", "nan", "range",
                                  "row_ptr"])
def test_malformed_device_csr_is_refused(case):
    import torch
    import paper_2502_17632_amd as gift
    rp, col, w = np.array([0, 2, 3, 4]), np.array([1, 2, 0, 0]), np.array([1.0, 2.0, 1.0, 2.0])
    if case == "unsorted":
        col = np.array([2, 1, 0, 0])
    elif case == "diagonal":
        col = np.array([1, 2, 1, 0])
    elif case == "negative":
        w = np.array([1.0, -2.0, 1.0, 2.0])
    elif case == "nan":
        w = np.array([1.0, np.nan, 1.0, 2.0])
    elif case == "range":
        col = np.array([1, 3, 0, 0])
    elif case == "row_ptr":
        rp = np.array([0, 3, 2, 4])
    dev = [torch.tensor(a, dtype=t, device="cuda")
           for a, t in ((rp, torch.int64), (col, torch.int32), (w, torch.float64))]
    with pytest.raises(gift.GiftError) as ei:
        gift.import_csr(*dev, sigmas=[4.0])
    assert ei.value.status == 1
    log(f"[import] malformed ({case}) refused: {ei.value}")


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_large_built_csr_imported_from_device(storage):
    """The large design's graph (2.06M rows with its star nodes, 23.7M
    entries), built from the netlist, exported and imported back from device
    memory: the same CSR, degrees and stored normalised values bit for bit
    (every row of the imported graph is a cell, so the star rows become
    ordinary rows with the same weights)."""
    import torch
    import paper_2502_17632_amd as gift
    nl = W.large()
    gb = gift.build_graph(nl.num_cells, nl.net_ptr, nl.pin_cell, star_threshold=16,
                          storage=storage, sigmas=[4.0])
    rp, col, w, deg = gb.export()
    log(f"[import] large built CSR R={len(rp) - 1} nnz={len(col)} storage={storage} (device)")
    dev = (torch.tensor(rp.astype(np.int64), device="cuda"), torch.tensor(col, device="cuda"),
           torch.tensor(w, device="cuda"))
    gi = gift.import_csr(*dev, storage=storage, sigmas=[4.0])
    rp2, col2, w2, deg2 = gi.export()
    assert np.array_equal(rp2, rp) and np.array_equal(col2, col)
    assert np.array_equal(w2.view(np.uint64), w.view(np.uint64))
    assert np.array_equal(deg2.view(np.uint64), deg.view(np.uint64))
    for u, v in zip(gb.export_normalised(4.0), gi.export_normalised(4.0)):
        assert np.array_equal(u.view(np.uint64), v.view(np.uint64))
    gb.close()
    gi.close()
