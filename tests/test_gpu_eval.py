"""Placement metrics on the GPU (smoothness / quadratic wirelength, Rayleigh
quotient, HPWL) against the CPU oracle (needs a GPU)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2502_17632_amd import workload as W

from parity import log

pytestmark = pytest.mark.gpu

EQ4 = ([4.0] * 4, [1, 2, 4, 8], [0.25] * 4)
TOL = 1e-11  # float64 sums in a different order


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return np.abs(a - b) / np.maximum(np.abs(b), 1e-300)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_metrics_match_the_oracle_before_and_after_filtering(dtype):
    import torch
    import paper_2502_17632_amd as gift
    nl = W.medium(seed=2)
    x = W.make_signal(nl, (10.0, 40.0), seed=2)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    if dtype == "f32":
        x = x.astype(np.float32).astype(np.float64)
    og = O.build_netlist(nl, star_threshold=16, star_order="median")
    g = gift.build_graph(nl.num_cells, nl.net_ptr, nl.pin_cell, star_threshold=16,
                         sigmas=[4.0])
    xt = torch.tensor(x, dtype=tdt, device="cuda")
    yt = gift.filter_placement(g, *EQ4, xt, out_dtype=tdt)
    for name, sig in (("initial", xt), ("filtered", yt)):
        m = gift.evaluate_placement(g, sig, nl.net_ptr, nl.pin_cell)
        S, n2, h = og.evaluate(sig.double().cpu().numpy())
        log(f"[eval] {dtype} {name}: S {m['smoothness']} (oracle {S}), HPWL {m['hpwl']}, "
            f"R {m['rayleigh']}")
        assert np.all(rel(m["smoothness"], S) < TOL), (name, m["smoothness"], S)
        assert np.all(rel(m["norm2"], n2) < TOL)
        assert np.all(rel(m["rayleigh"], S / n2) < TOL)  # eq. smoothness_ray
        assert np.all(rel(m["hpwl"], h) < TOL)
    # the low-pass filter smooths a white-noise signal (Section 3.1): the
    # Rayleigh quotient drops.  (A placement whose fixed cells sit on the die
    # boundary need not lose wirelength: the raw filter also moves them.)
    noise = torch.tensor(np.random.default_rng(3).normal(size=(nl.num_cells, 2)), dtype=tdt,
                         device="cuda")
    m0 = gift.evaluate_placement(g, noise)
    m1 = gift.evaluate_placement(g, gift.filter_placement(g, *EQ4, noise, out_dtype=tdt))
    log(f"[eval] white noise R {m0['rayleigh']} -> {m1['rayleigh']}")
    assert np.all(m1["rayleigh"] < 0.5 * m0["rayleigh"])
    g.close()


def test_smoothness_does_not_depend_on_the_star_threshold():
    """A star with its node at the mean of its cells has its clique's
    quadratic wirelength exactly (the Schur complement), so the graph built
    with stars and the all-clique graph give the same S."""
    import torch
    import paper_2502_17632_amd as gift
    nl = W.sized(20_000, seed=9)
    x = torch.tensor(W.make_signal(nl, seed=9), device="cuda")
    vals = []
    for T in (0, 8, 16):
        g = gift.build_graph(nl.num_cells, nl.net_ptr, nl.pin_cell, star_threshold=T,
                             sigmas=[4.0])
        vals.append(gift.evaluate_placement(g, x, nl.net_ptr, nl.pin_cell))
        g.close()
    for v in vals[1:]:
        assert np.all(rel(v["smoothness"], vals[0]["smoothness"]) < 1e-10)
        assert np.array_equal(v["hpwl"], vals[0]["hpwl"])
    log(f"[eval] S by threshold: {[v['smoothness'].tolist() for v in vals]}")


def test_metrics_are_deterministic_and_check_arguments():
    import torch
    import paper_2502_17632_amd as gift
    nl = W.sized(5_000, seed=4)
    g = gift.build_graph(nl.num_cells, nl.net_ptr, nl.pin_cell, star_threshold=16)
    x = torch.tensor(W.make_signal(nl, seed=4), dtype=torch.float32, device="cuda")
    a = gift.evaluate_placement(g, x, nl.net_ptr, nl.pin_cell)
    b = gift.evaluate_placement(g, x, nl.net_ptr, nl.pin_cell)
    for k in a:
        assert np.array_equal(a[k], b[k])
    # pins outside the cells and offsets beyond the pins are ignored, not read
    bad_pins = nl.pin_cell.copy()
    bad_pins[0] = nl.num_cells + 100
    bad_ptr = nl.net_ptr.copy()
    bad_ptr[-1] += 1000
    gift.evaluate_placement(g, x, bad_ptr, bad_pins)
    with pytest.raises(ValueError):
        gift.evaluate_placement(g, x[:10])
    g.close()


@pytest.mark.parametrize("threshold", [16, 0])
def test_metrics_with_a_ragged_column_count(threshold):
    """Seven columns (a full group of four and a ragged three) on a design
    with nets of up to 1000 pins: star rows and, without stars, clique rows
    longer than one row tile's limit, and nets long enough to be taken by a
    whole wave, all against the oracle."""
    import torch
    import paper_2502_17632_amd as gift
    nl = W.sized(30_000, seed=21)
    x = np.random.default_rng(21).normal(scale=50.0, size=(nl.num_cells, 7))
    og = O.build_netlist(nl, star_threshold=threshold, star_order="median")
    g = gift.build_graph(nl.num_cells, nl.net_ptr, nl.pin_cell, star_threshold=threshold)
    xt = torch.tensor(x, dtype=torch.float64, device="cuda")
    m = gift.evaluate_placement(g, xt, nl.net_ptr, nl.pin_cell)
    S, n2, h = og.evaluate(x)
    og.close()
    g.close()
    sizes = np.diff(nl.net_ptr)
    log(f"[eval] 7 columns, threshold {threshold}: longest net {sizes.max()} pins; "
        f"S {m['smoothness'][:2]}.. (oracle {S[:2]}..)")
    assert np.all(rel(m["smoothness"], S) < TOL)
    assert np.all(rel(m["norm2"], n2) < TOL)
    assert np.all(rel(m["hpwl"], h) < TOL)
