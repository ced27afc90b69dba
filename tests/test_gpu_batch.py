"""Batched filtering (one captured launch sequence over many designs) against
the per-design path and the CPU oracle (needs a GPU).

A batch is block-diagonal: every design's rows are computed by the same
arithmetic as when it is filtered alone, so with the default schedule the
results are bit-identical to the per-design path; any tuned schedule stays
within the storage type's tolerance of the oracle.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2502_17632_amd import workload as W

from parity import TOL, assert_close, colwise_error, log

pytestmark = pytest.mark.gpu

EQ4 = ([4.0] * 4, [1, 2, 4, 8], [0.25] * 4)
PAPER = (W.PAPER_DEFAULT.sigma, W.PAPER_DEFAULT.order, W.PAPER_DEFAULT.alpha)
SIZES = [3_000, 11_000, 800, 27_000, 5_500]


@pytest.fixture(scope="module")
def designs():
    nls = [W.sized(n, seed=1000 + i) for i, n in enumerate(SIZES)]
    xs = [W.make_signal(nl, W.BATCH_NOISE, seed=1000 + i) for i, nl in enumerate(nls)]
    return nls, xs


@pytest.fixture(scope="module")
def oracles(designs):
    nls, _ = designs
    return [O.build_netlist(nl, star_threshold=16, star_order="median") for nl in nls]


def build_all(nls, storage, sigmas):
    import paper_2502_17632_amd as gift
    return [gift.build_graph(nl.num_cells, nl.net_ptr, nl.pin_cell, star_threshold=16,
                             storage=storage, sigmas=sigmas) for nl in nls]


def to_dev(x, dtype):
    import torch
    return torch.tensor(np.asarray(x, dtype=np.float64), dtype=dtype, device="cuda")


@pytest.mark.parametrize("storage,tune", [("f32", 0), ("bf16", 0), ("f32", 3), ("bf16", 3)])
def test_batch_default_schedule_is_bit_identical_to_alone(designs, storage, tune):
    """The default schedule, with the round-robin and with the XCD-affine
    tile layout: every design's result equals filtering it alone."""
    import torch
    import paper_2502_17632_amd as gift
    nls, xs = designs
    graphs = build_all(nls, storage, [4.0])
    xt = [to_dev(x, torch.float32) for x in xs]
    b = gift.Batch(graphs, *EQ4, num_cols=8, tune=tune)
    info = b.info()
    log(f"[batch] default schedule {storage}, xcd_affine {info['xcd_affine']}: "
        f"{info['num_graphs']} graphs, rows {info['num_rows']}, tiles {info['num_tiles']}")
    assert info["tuned"] == 0 and info["tile_class"] == 0 and info["chunk_cols"] == 8
    assert info["xcd_affine"] == (1 if tune == 3 else 0)
    ys = b.run(xt)
    alone = [gift.filter_placement(g, *EQ4, x) for g, x in zip(graphs, xt)]
    torch.cuda.synchronize()
    for i, (y, a) in enumerate(zip(ys, alone)):
        assert torch.equal(y, a), f"design {i} differs from the per-design result"
    b.close()


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_batch_tuned_matches_oracle(designs, oracles, storage):
    import torch
    import paper_2502_17632_amd as gift
    nls, xs = designs
    graphs = build_all(nls, storage, [2.0, 4.0])
    xt = [to_dev(np.asarray(x, np.float32), torch.float32) for x in xs]
    b = gift.Batch(graphs, *PAPER, num_cols=8, tune=2)
    info = b.info()
    log(f"[batch] tuned {storage}: class {info['tile_class']} chunk {info['chunk_cols']} "
        f"candidates {[(c['tile_class'], c['chunk_cols'], round(c['ms'], 4)) for c in info['candidates']]}")
    assert info["tuned"] == 1 and info["num_candidates"] >= 2
    ys = b.run(xt)
    torch.cuda.synchronize()
    for i, (y, og) in enumerate(zip(ys, oracles)):
        xin = xt[i].double().cpu().numpy()
        ref = og.filter(xin, *PAPER)
        assert_close(y.double().cpu().numpy(), ref, storage, f"batch {storage} design {i}")
    b.close()


def test_graph_replays_match_eager_with_work_in_between(designs):
    """Replays of the captured sequence with new inputs each time, eager
    per-design filters and synchronisations in between: every replay equals
    the eager per-design result."""
    import torch
    import paper_2502_17632_amd as gift
    nls, xs = designs
    graphs = build_all(nls, "f32", [4.0])
    b = gift.Batch(graphs, *EQ4, num_cols=8, tune=0)
    rng = np.random.default_rng(5)
    for rep in range(4):
        xt = [to_dev(x + rng.normal(0, 3.0, size=x.shape), torch.float32) for x in xs]
        ys = b.run(xt)
        torch.cuda.synchronize()
        alone = [gift.filter_placement(g, *EQ4, x) for g, x in zip(graphs, xt)]
        torch.cuda.synchronize()
        for i, (y, a) in enumerate(zip(ys, alone)):
            assert torch.equal(y, a), f"replay {rep}, design {i}"
        log(f"[batch] replay {rep} equal to eager")
    b.close()


def test_runs_on_two_streams_in_a_row(designs):
    """Two runs of one batch enqueued back to back on two different streams,
    with different inputs and no host synchronisation between them: the
    second waits for the first (they share the batch's buffers), so each
    result equals filtering its own inputs alone, bit for bit."""
    import torch
    import paper_2502_17632_amd as gift
    nls, xs = designs
    graphs = build_all(nls, "f32", [4.0])
    b = gift.Batch(graphs, *EQ4, num_cols=8, tune=0)
    rng = np.random.default_rng(9)
    inputs = [[to_dev(x + rng.normal(0, 5.0, size=x.shape), torch.float32) for x in xs]
              for _ in range(2)]
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    ys1 = b.run(inputs[0], stream=s1)
    ys2 = b.run(inputs[1], stream=s2)
    torch.cuda.synchronize()
    for rep, ys in enumerate((ys1, ys2)):
        alone = [gift.filter_placement(g, *EQ4, x) for g, x in zip(graphs, inputs[rep])]
        torch.cuda.synchronize()
        for i, (y, a) in enumerate(zip(ys, alone)):
            assert torch.equal(y, a), f"run {rep} on its own stream, design {i}"
    log("[batch] runs on two streams in a row equal to eager")
    b.close()


def test_batch_outputs_in_place_and_fixed_rows(designs, oracles):
    """Caller-provided outputs with a leading dimension, fixed masks on some
    designs, float64 input."""
    import torch
    import paper_2502_17632_amd as gift
    nls, xs = designs
    graphs = build_all(nls, "f32", [4.0])
    b = gift.Batch(graphs, *EQ4, num_cols=8, in_dtype=torch.float64, tune=1)
    xt = [to_dev(x, torch.float64) for x in xs]
    big = [torch.full((x.shape[0], 11), -7.0, dtype=torch.float32, device="cuda") for x in xs]
    outs = [t[:, 1:9] for t in big]
    fixed = [torch.tensor(nl.fixed, dtype=torch.uint8, device="cuda") if i % 2 == 0 else None
             for i, nl in enumerate(nls)]
    b.run(xt, outs, fixed)
    torch.cuda.synchronize()
    for i, (nl, og) in enumerate(zip(nls, oracles)):
        t = big[i].cpu().numpy()
        assert np.all(t[:, 0] == -7.0) and np.all(t[:, 9:] == -7.0)
        ref = og.filter(xs[i], *EQ4, fixed=nl.fixed if i % 2 == 0 else None)
        assert_close(t[:, 1:9].astype(np.float64), ref, "f32", f"batch ld/fixed design {i}")
    b.close()


def test_batch_with_empty_and_netless_designs():
    import torch
    import paper_2502_17632_amd as gift
    empty = W.Netlist(0, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.uint8), "e")
    netless = W.Netlist(5, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(5, np.uint8), "n")
    small = W.sized(400, seed=77)
    nls = [empty, netless, small]
    graphs = build_all(nls, "f64", [4.0])
    b = gift.Batch(graphs, *EQ4, num_cols=3, in_dtype=torch.float64, out_dtype=torch.float64,
                   tune=1)
    xs = [W.make_signal(nl, (10.0, 20.0), seed=3)[:, :3] if nl.num_cells else
          np.zeros((0, 3)) for nl in nls]
    xt = [to_dev(x, torch.float64).contiguous() for x in xs]
    ys = b.run(xt)
    torch.cuda.synchronize()
    assert ys[0].shape == (0, 3)
    for i in (1, 2):
        og = O.build_netlist(nls[i], star_threshold=16, star_order="median")
        ref = og.filter(xs[i], *EQ4)
        assert_close(ys[i].cpu().numpy(), ref, "f64", f"batch degenerate design {i}")
    b.close()


def test_tuning_cache_is_reused(designs):
    import torch
    import paper_2502_17632_amd as gift
    nls, xs = designs
    graphs = build_all(nls, "f32", [4.0])
    b1 = gift.Batch(graphs, *EQ4, num_cols=8, tune=2)
    b2 = gift.Batch(graphs, *EQ4, num_cols=8, tune=1)
    i1, i2 = b1.info(), b2.info()
    assert i1["tuned"] == 1 and i2["tuned"] == 2
    assert (i1["tile_class"], i1["chunk_cols"]) == (i2["tile_class"], i2["chunk_cols"])
    xt = [to_dev(x, torch.float32) for x in xs]
    y1, y2 = b1.run(xt), b2.run(xt)
    torch.cuda.synchronize()
    for a, c in zip(y1, y2):
        assert torch.equal(a, c)
    b1.close()
    b2.close()


def test_batch_rejects_bad_arguments(designs):
    import torch
    import paper_2502_17632_amd as gift
    nls, xs = designs
    g32 = build_all(nls[:1], "f32", [4.0])
    g16 = build_all(nls[1:2], "bf16", [4.0])
    with pytest.raises(gift.GiftError):
        gift.Batch(g32 + g16, *EQ4, num_cols=8)          # mixed storage
    with pytest.raises(gift.GiftError):
        gift.Batch(g32, [3.0], [2], [1.0], num_cols=8)     # sigma not prepared
    b = gift.Batch(g32, *EQ4, num_cols=8, tune=0)
    with pytest.raises(TypeError):
        b.run([to_dev(xs[0][:, :4], torch.float32)])      # wrong column count
    b.close()
