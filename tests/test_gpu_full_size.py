"""The batched and serving workloads at the sizes the benchmark times (needs a
GPU).  Every design's result is compared with the per-design filter (a
property that holds at any size: a batch or a served launch computes each
design's rows with the arithmetic of filtering it alone), and sampled designs
with the float64 oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2502_17632_amd import workload as W

from parity import TOL, assert_close, colwise_error, log

pytestmark = pytest.mark.gpu

EQ4 = ([4.0] * 4, [1, 2, 4, 8], [0.25] * 4)


@pytest.fixture(scope="module")
def batch_designs():
    """64 designs of 10k-300k movable cells (medium generator, seeds 1000+i),
    8 columns each: 4 placements with noise 5, 10, 20, 40."""
    sizes = W.batch_sizes(64)
    nls = [W.sized(n, seed=1000 + i) for i, n in enumerate(sizes)]
    xs = [W.make_signal(nl, W.BATCH_NOISE, seed=1000 + i) for i, nl in enumerate(nls)]
    return nls, xs


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_batched_workload_at_full_size(batch_designs, storage):
    """The tuned batch of all 64 designs, fixed cells kept: each design equals
    its per-design filter (bit for bit when the tuner keeps tile class 0,
    whose tiles are the per-design path's), and every 8th design meets the
    oracle bar."""
    import torch
    import paper_2502_17632_amd as gift
    nls, xs = batch_designs
    log(f"[full] batch of {len(nls)} designs, {sum(nl.num_cells for nl in nls)} cells, "
        f"8 columns, {storage}")
    graphs = [gift.build_graph(nl.num_cells, nl.net_ptr, nl.pin_cell, star_threshold=16,
                               storage=storage, sigmas=[4.0]) for nl in nls]
    xt = [torch.tensor(x, dtype=torch.float32, device="cuda") for x in xs]
    ft = [torch.tensor(nl.fixed, device="cuda") for nl in nls]
    alone = [gift.filter_placement(g, *EQ4, x, fixed=f) for g, x, f in zip(graphs, xt, ft)]
    b = gift.Batch(graphs, *EQ4, num_cols=8, tune=1)
    ys = b.run(xt, fixed=ft)
    torch.cuda.synchronize()
    info = b.info()
    diffs = [float(colwise_error(y.double().cpu().numpy(), a.double().cpu().numpy()).max())
             for y, a in zip(ys, alone)]
    log(f"[full] schedule: tile class {info['tile_class']}, chunk {info['chunk_cols']}, "
        f"xcd_affine {info['xcd_affine']}; largest difference from per-design {max(diffs):.2e}")
    if info["tile_class"] == 0:
        assert max(diffs) == 0.0
    assert max(diffs) <= TOL[storage]
    for i in range(0, len(nls), 8):
        og = O.build_netlist(nls[i], star_threshold=16, star_order="median")
        xin = xs[i].astype(np.float32).astype(np.float64)
        ref = og.filter(xin, *EQ4, fixed=nls[i].fixed)
        og.close()
        assert_close(ys[i].double().cpu().numpy(), ref, storage,
                     f"full batch {storage} design {i} ({nls[i].num_cells} cells)")
    b.close()
    for g in graphs:
        g.close()


def test_serving_pool_at_full_size():
    """The 24-design serving pool (5k-2M movable cells, medium generator,
    seeds 5000+i) through the server as the benchmark configures it: every
    design requested twice (cold: built on demand; then warm), all submitted
    at once, fixed cells kept.  Each result equals the design filtered alone
    bit for bit; the largest design meets the oracle bar."""
    import torch
    import paper_2502_17632_amd as gift
    sizes = W.serving_sizes(24)
    nls = [W.sized(n, seed=5000 + i) for i, n in enumerate(sizes)]
    xs = [W.make_signal(nl, seed=5000 + i) for i, nl in enumerate(nls)]
    log(f"[full] serving pool of {len(nls)} designs, {sum(nl.num_cells for nl in nls)} cells")
    xt = [torch.tensor(x, dtype=torch.float32, device="cuda") for x in xs]
    ft = [torch.tensor(nl.fixed, device="cuda") for nl in nls]
    alone = []
    for nl, x, f in zip(nls, xt, ft):
        g = gift.build_graph(nl.num_cells, nl.net_ptr, nl.pin_cell, star_threshold=16,
                             sigmas=[4.0])
        alone.append(gift.filter_placement(g, *EQ4, x, fixed=f))
        torch.cuda.synchronize()
        g.close()
    srv = gift.Server(*EQ4, num_cols=2, hbm_budget_bytes=200 << 30, max_inflight=64,
                      num_streams=4, num_builders=2, max_batch=32)
    for rnd in ("cold", "warm"):
        subs = []
        for i, nl in enumerate(nls):
            t, y = srv.submit(i, nl.num_cells, nl.net_ptr, nl.pin_cell, xt[i], fixed=ft[i])
            subs.append((t, y, i))
        built = 0
        for t, y, i in subs:
            res = srv.wait(t)
            assert res["status"] == 0, (rnd, i)
            built += res["built"]
            assert torch.equal(y, alone[i]), f"{rnd} request for design {i} differs from alone"
        st = srv.stats()
        log(f"[full] serving {rnd}: {built} builds, {st['batches']} launches so far")
        assert built == (len(nls) if rnd == "cold" else 0)
    srv.close()
    big = int(np.argmax(sizes))
    og = O.build_netlist(nls[big], star_threshold=16, star_order="median")
    ref = og.filter(xs[big].astype(np.float32).astype(np.float64), *EQ4, fixed=nls[big].fixed)
    og.close()
    assert_close(alone[big].double().cpu().numpy(), ref, "f32",
                 f"full serving design {big} ({nls[big].num_cells} cells)")
