"""Device path vs the CPU oracle on the same seeded inputs (needs a GPU)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2502_17632_amd import workload as W

from parity import TOL, assert_close, check_normalised, check_structure, log, run_pair

pytestmark = pytest.mark.gpu

EQ4 = ([4.0] * 4, [1, 2, 4, 8], [0.25] * 4)
EQ5 = ([4.0] * 5, [1, 2, 4, 8, 16], [0.2] * 5)
PAPER = (W.PAPER_DEFAULT.sigma, W.PAPER_DEFAULT.order, W.PAPER_DEFAULT.alpha)


def handmade(nets, n):
    net_ptr = np.zeros(len(nets) + 1, dtype=np.int64)
    net_ptr[1:] = np.cumsum([len(p) for p in nets])
    pins = np.array([c for p in nets for c in p], dtype=np.int32)
    return W.Netlist(n, net_ptr, pins, np.zeros(n, dtype=np.uint8), "handmade")


@pytest.fixture(scope="module")
def medium():
    return W.medium()


@pytest.fixture(scope="module")
def medium_oracle(medium):
    return O.build_netlist(medium, star_threshold=16, star_order="median")


def test_tiny_f64_equal_weights():
    nl = W.tiny()
    x = W.make_signal(nl)
    y, ref, g, og = run_pair(nl, x, EQ4, storage="f64", label="tiny f64")
    check_normalised(g, og, 4.0, "f64")
    assert_close(y, ref, "f64", "tiny f64")


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16", "f16"])
def test_tiny_paper_filter(storage):
    nl = W.tiny(seed=1)
    x = W.make_signal(nl, seed=1)
    y, ref, g, og = run_pair(nl, x, PAPER, storage=storage, label=f"tiny paper {storage}")
    for s in (2.0, 4.0):
        check_normalised(g, og, s, storage)
    assert_close(y, ref, storage, f"tiny paper {storage}")


@pytest.mark.parametrize("storage", ["f32", "bf16", "f16"])
def test_medium(medium, medium_oracle, storage):
    x = W.make_signal(medium)
    y, ref, g, og = run_pair(medium, x, EQ4, storage=storage, star_threshold=16,
                             og=medium_oracle, label=f"medium {storage}")
    check_normalised(g, og, 4.0, storage)
    assert_close(y, ref, storage, f"medium {storage}")


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_centred_16bit_on_the_fixed_point(storage):
    """Theorem 1 with the self-loop: v = sqrt(d + sigma) satisfies
    A~_sigma v = v, so with one sigma the filter of x = k v is (sum of alpha)
    k v.  The 16-bit path iterates on x - c v with c = sum x / sum v; for
    x = k v that iterate is only the input's rounding residue, so the result
    must match the float64 oracle far inside the 16-bit gate (1e-5 against
    2e-2).  A centring on another vector, with another c, or without c v
    added back in the combine misses by orders of magnitude."""
    # nets of at most 16 cells: no star rows, whose start value (the mean of
    # their cells) is not k v
    nl = W.make_netlist(50_000, 500, 55_000, cap=16, seed=7, name="capped")
    og = O.build_graph(nl.num_cells, nl.net_ptr, nl.pin_cell, star_threshold=16,
                       star_order="median")
    assert og.num_virtual == 0
    v = np.sqrt(og.deg + 4.0)
    x = np.stack([3.5 * v, 120.0 * v], axis=1)
    y, ref, g, og = run_pair(nl, x, EQ4, storage=storage, star_threshold=16, og=og,
                             label=f"fixed point {storage}")
    xin = x.astype(np.float32).astype(np.float64)
    # the premise, on the oracle: the signal is (up to its float32 rounding)
    # the fixed point, and the equal weights sum to 1
    assert np.abs(ref - xin).max() <= 1e-6 * np.abs(xin).max()
    err = assert_close(y, ref, storage, f"fixed point {storage}")
    assert np.all(err <= 1e-5), err


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_centred_16bit_keeps_bad_inputs_local(storage):
    """A NaN or infinite input reaches, in one pass, only its own row and its
    neighbours' rows.  Centring must not spread it through the centring
    multiplier to every row: the non-finite pattern of the 16-bit result
    equals the float32 one."""
    import torch
    import paper_2502_17632_amd as gift
    nl = W.tiny(seed=2)
    x = W.make_signal(nl, seed=2).astype(np.float32)
    x[17, 0] = np.nan
    x[99, 1] = np.inf
    xt = torch.tensor(x, device="cuda")
    finite = {}
    for st in ("f32", storage):
        g = gift.build_graph(nl.num_cells, nl.net_ptr, nl.pin_cell, storage=st, sigmas=[4.0])
        y = gift.filter_placement(g, [4.0], [1], [1.0], xt)
        torch.cuda.synchronize()
        finite[st] = np.isfinite(y.cpu().numpy())
        g.close()
    log(f"[parity] bad inputs {storage}: {int((~finite[storage]).sum())} non-finite outputs "
        f"(f32: {int((~finite['f32']).sum())})")
    assert (~finite["f32"]).sum() < 0.05 * finite["f32"].size
    assert np.array_equal(finite["f32"], finite[storage])


def test_sixty_four_terms_float64():
    """The largest filter the boundary takes: 64 terms, 8 self-loop weights
    with orders 1..8 each and arbitrary weights alpha (not summing to 1),
    against the oracle at the float64 bar; a 65th term is refused."""
    import torch
    import paper_2502_17632_amd as gift
    nl = W.tiny(seed=5)
    x = W.make_signal(nl, seed=5)
    rng = np.random.default_rng(64)
    sig = [s for s in (0.25, 0.5, 1.0, 1.5, 2.0, 3.0, 4.0, 6.0) for _ in range(8)]
    order = [k for _ in range(8) for k in range(1, 9)]
    alpha = list(rng.uniform(-0.5, 1.0, size=64))
    y, ref, g, og = run_pair(nl, x, (sig, order, alpha), storage="f64", label="64 terms f64")
    assert_close(y, ref, "f64", "64 terms f64")
    xt = torch.tensor(x, device="cuda")
    with pytest.raises(gift.GiftError):
        gift.filter_placement(g, sig + [4.0], order + [1], alpha + [0.1], xt,
                              out_dtype=torch.float64)
    g.close()


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_sixty_four_sigma_groups_16bit(storage):
    """64 terms with 64 distinct self-loop weights: the centring of 16-bit
    iterates sums x and sqrt(d + sigma) for every group (four groups per
    round of its reduction kernel, 16 rounds here), and the combine adds each
    term's own c v back."""
    nl = W.tiny(seed=6)
    x = W.make_signal(nl, seed=6)
    sig = [0.1 * (t + 1) for t in range(64)]
    order = [1 + t % 3 for t in range(64)]
    alpha = [1.0 / 64] * 64
    y, ref, g, og = run_pair(nl, x, (sig, order, alpha), storage=storage,
                             label=f"64 groups {storage}")
    assert_close(y, ref, storage, f"64 groups {storage}")
    g.close()


def test_medium_two_over_m_paper_terms(medium):
    x = W.make_signal(medium, seed=3)
    y, ref, g, og = run_pair(medium, x, PAPER, storage="f32", star_threshold=16,
                             weight_model="two_over_m", label="medium 2/M paper")
    assert_close(y, ref, "f32", "medium 2/M paper")


def test_medium_all_cliques(medium):
    # T = 0: nets of up to 1000 pins expand as cliques (long rows, big sorts)
    x = W.make_signal(medium, seed=4)
    y, ref, g, og = run_pair(medium, x, EQ4, storage="f32", star_threshold=0,
                             label="medium cliques")
    assert_close(y, ref, "f32", "medium cliques")


def test_sort_tiers_and_long_rows():
    # nets of 3, 40 (wave tier), 500 (LDS tier) and 9000 (global merge tier)
    # pins, with repeated pins; cell 0 on 5000 two-pin nets (row sorted by the
    # global merge tier), cell 1 on 300 (LDS tier), cell 2 on 40 (wave tier)
    rng = np.random.default_rng(11)
    n = 20_000
    nets = [[5, 6, 7]]
    for m in (40, 500, 9000):
        cells = list(rng.choice(np.arange(10, n), size=m, replace=False))
        cells += cells[:3]  # repeated pins
        rng.shuffle(cells)
        nets.append(cells)
    for hub, count in ((0, 5000), (1, 300), (2, 40)):
        for c in rng.choice(np.arange(10, n), size=count, replace=False):
            nets.append([hub, int(c)] if rng.random() < 0.5 else [int(c), hub])
    nl = handmade(nets, n)
    x = rng.normal(500, 50, size=(n, 2))
    for thr in (16, 600):
        y, ref, g, og = run_pair(nl, x, PAPER, storage="f32", star_threshold=thr,
                                 label=f"tiers T={thr}")
        assert_close(y, ref, "f32", f"tiers T={thr}")


def test_virtual_rows_labelled_by_median():
    """Virtual rows in ascending (median cell, net id) order, against the
    oracle's median labelling bit for bit: 3000 star nets whose middle cell is
    cell 100 (one median bucket of 3000 keys, sorted through global memory
    since it exceeds one LDS chunk), 300 with medians spread over the design
    in descending net order, and 200 tied pairs of identical nets."""
    rng = np.random.default_rng(23)
    n = 3000 * 8 + 20_000
    nets = []
    for e in range(3000):  # 8 cells below 100, cell 100, 8 above: median 100
        low = [int(c) for c in rng.choice(100, size=8, replace=False)]
        nets.append(low + [100] + list(range(200 + 8 * e, 208 + 8 * e)))
    for k in range(300):  # 20-cell nets around a descending anchor
        a = n - 100 - 60 * k
        nets.append([a + int(d) for d in rng.choice(np.arange(-40, 40), size=20, replace=False)])
    for k in range(200):  # identical pairs: equal medians, ordered by net id
        cells = [int(c) for c in rng.choice(n, size=18, replace=False)]
        nets += [cells, cells[::-1]]
    for _ in range(2000):
        nets.append([int(c) for c in rng.choice(n, size=3, replace=False)])
    order = rng.permutation(len(nets))
    nl = handmade([nets[i] for i in order], n)
    x = rng.normal(500, 50, size=(n, 2))
    y, ref, g, og = run_pair(nl, x, PAPER, storage="f32", star_threshold=16,
                             label="median labelling")
    v = og.num_virtual
    assert v == 3000 + 300 + 400
    lens = np.diff(og.row_ptr[n:])
    med = og.col[og.row_ptr[n:-1] + lens // 2].astype(np.int64)
    assert np.all(np.diff(med * (1 << 32) + og.virt_net) > 0)
    assert_close(y, ref, "f32", "median labelling")


def test_degenerate_netlists():
    rng = np.random.default_rng(12)
    x = rng.normal(0, 3, size=(6, 2))
    cases = {
        "no nets": handmade([], 6),
        "only 0/1-pin and repeated-pin nets": handmade([[], [3], [2, 2, 2]], 6),
        "one 2-pin net": handmade([[4, 1]], 6),
        "parallel nets": handmade([[0, 1], [1, 0], [0, 1, 2], [5, 4, 4]], 6),
    }
    for name, nl in cases.items():
        for terms in (PAPER, ([0.5], [3], [1.0])):
            y, ref, g, og = run_pair(nl, x, terms, storage="f64", label=name)
            assert_close(y, ref, "f64", name)


def test_sigma_zero_isolated_rows():
    nl = handmade([[0, 1], [1, 2, 3]], 6)  # cells 4, 5 isolated
    x = np.arange(12, dtype=np.float64).reshape(6, 2) + 1
    y, ref, g, og = run_pair(nl, x, ([0.0, 2.0], [2, 1], [0.5, 0.5]), storage="f64",
                             label="sigma 0")
    assert_close(y, ref, "f64", "sigma 0")
    # (sigma s) s with s = 1/sqrt(sigma) is 1 only up to rounding
    assert np.allclose(y[4:], 0.5 * x[4:], rtol=1e-15, atol=0)


@pytest.mark.parametrize("cols", [1, 3, 8, 16, 19])
def test_column_counts_and_leading_dimension(cols):
    import torch
    import paper_2502_17632_amd as gift
    nl = W.sized(30_000, seed=77)
    rng = np.random.default_rng(cols)
    x = rng.normal(500, 20, size=(nl.num_cells, cols)).astype(np.float32)
    og = O.build_netlist(nl, star_threshold=16, star_order="median")
    g = gift.build_graph(nl.num_cells, nl.net_ptr, nl.pin_cell, star_threshold=16,
                         sigmas=[2.0, 4.0])
    wide = torch.zeros((nl.num_cells, cols + 5), dtype=torch.float32, device="cuda")
    wide[:, 2:2 + cols] = torch.tensor(x, device="cuda")
    xv = wide[:, 2:2 + cols]  # leading dimension cols + 5
    out = torch.full((nl.num_cells, cols + 3), float("nan"), dtype=torch.float64, device="cuda")
    ov = out[:, 1:1 + cols]
    gift.filter_placement(g, *PAPER, xv, out=ov)
    torch.cuda.synchronize()
    y = ov.cpu().numpy()
    ref = og.filter(x.astype(np.float64), *PAPER)
    assert_close(y, ref, "f32", f"{cols} columns")
    assert torch.isnan(out[:, 0]).all() and torch.isnan(out[:, 1 + cols:]).all()


@pytest.mark.parametrize("storage,cols", [("f64", 2), ("f64", 8), ("f32", 8)])
def test_float64_input_with_star_nets(storage, cols):
    """A float64 signal on a design with star nets: the star rows' start
    values are gathered from float64 input (two cells per lane at a time),
    at two and eight columns, stored as float64 or float32."""
    import torch
    import paper_2502_17632_amd as gift
    nl = W.sized(20_000, seed=31)
    x = np.random.default_rng(31 + cols).normal(500, 20, size=(nl.num_cells, cols))
    og = O.build_netlist(nl, star_threshold=16, star_order="median")
    g = gift.build_graph(nl.num_cells, nl.net_ptr, nl.pin_cell, star_threshold=16,
                         storage=storage, sigmas=[2.0, 4.0])
    y = gift.filter_placement(g, *PAPER, torch.tensor(x, device="cuda"),
                              out_dtype=torch.float64)
    torch.cuda.synchronize()
    ref = og.filter(x, *PAPER)
    og.close()
    g.close()
    assert_close(y.cpu().numpy(), ref, storage, f"float64 input, {storage}, {cols} columns")


def test_fixed_rows_restored():
    nl = W.tiny(seed=2)
    x = W.make_signal(nl, seed=2)
    y, ref, g, og = run_pair(nl, x, PAPER, storage="f32", fixed=nl.fixed, label="fixed")
    assert_close(y, ref, "f32", "fixed")
    fx = nl.fixed.astype(bool)
    assert np.array_equal(y[fx], x[fx].astype(np.float32).astype(np.float64))


def test_device_resident_netlist_and_determinism():
    import torch
    import paper_2502_17632_amd as gift
    nl = W.sized(50_000, seed=5)
    npd = torch.tensor(nl.net_ptr, device="cuda")
    pcd = torch.tensor(nl.pin_cell, device="cuda")
    g1 = gift.build_graph(nl.num_cells, npd, pcd, star_threshold=16, sigmas=[4.0])
    g2 = gift.build_graph(nl.num_cells, nl.net_ptr, nl.pin_cell, star_threshold=16,
                          sigmas=[4.0])
    og = O.build_netlist(nl, star_threshold=16, star_order="median")
    check_structure(g1, og)
    for a, b in zip(g1.export(), g2.export()):
        assert np.array_equal(a, b)
    x = torch.tensor(W.make_signal(nl), dtype=torch.float32, device="cuda")
    y1 = gift.filter_placement(g1, *EQ4, x)
    y2 = gift.filter_placement(g1, *EQ4, x)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)


def test_invalid_netlists_are_rejected():
    import torch
    import paper_2502_17632_amd as gift
    bad = [
        (np.array([0, 2, 3]), np.array([0, 1, 9])),  # pin out of range
        (np.array([0, 2, 3]), np.array([0, -1, 1])),  # negative pin
        (np.array([0, 3, 2]), np.array([0, 1])),  # decreasing net_ptr
        (np.array([1, 2, 3]), np.array([0, 1, 1])),  # does not start at 0
    ]
    for net_ptr, pins in bad:
        for dev in (False, True):
            a, b = net_ptr.astype(np.int64), pins.astype(np.int32)
            if dev:
                a, b = torch.tensor(a, device="cuda"), torch.tensor(b, device="cuda")
            with pytest.raises(gift.GiftError) as ei:
                gift.build_graph(3, a, b)
            assert ei.value.status == 1
    with pytest.raises(ValueError):  # pin array shorter than net_ptr[-1]
        gift.build_graph(3, np.array([0, 2, 5]), np.array([0, 1, 1]))
    with pytest.raises(gift.GiftError) as ei:  # the same on the device: the library checks
        gift.build_graph(3, torch.tensor([0, 2, 5], device="cuda"),
                         torch.tensor([0, 1, 1], dtype=torch.int32, device="cuda"))
    assert ei.value.status == 1
    g = gift.build_graph(3, np.array([0, 2]), np.array([0, 1]), sigmas=[4.0])
    x = torch.zeros((3, 2), device="cuda")
    with pytest.raises(gift.GiftError):
        gift.filter_placement(g, [2.0], [1], [1.0], x)  # sigma not prepared
    with pytest.raises(gift.GiftError):
        gift.filter_placement(g, [4.0], [0], [1.0], x)  # order 0
    g.add_sigma(2.0)
    gift.filter_placement(g, [2.0], [1], [1.0], x)
    torch.cuda.synchronize()


@pytest.mark.parametrize("storage", ["f32", "bf16", "f16"])
def test_large_full_size(storage):
    """The large workload (2M + 20k cells, 2.1M nets), as the benchmark runs it
    (fixed cells kept at their input positions)."""
    nl = W.large()
    x = W.make_signal(nl)
    og = getattr(test_large_full_size, "_og", None)
    if og is None:
        log("[parity] building the large oracle graph")
        og = O.build_netlist(nl, star_threshold=16, star_order="median")
        test_large_full_size._og = og
    y, ref, g, og = run_pair(nl, x, EQ5, storage=storage, star_threshold=16, og=og,
                             fixed=nl.fixed, label=f"large {storage}")
    check_normalised(g, og, 4.0, storage)
    assert_close(y, ref, storage, f"large {storage}")
    assert np.array_equal(y[nl.fixed != 0], x.astype(np.float32).astype(np.float64)[nl.fixed != 0])
