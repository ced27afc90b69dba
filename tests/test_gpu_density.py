"""Bin density (eq. density_eq) on the GPU against the CPU oracle (needs a
GPU).  The device sums each overlap rounded to 2^-40 of a bin's area, so a
bin with k contributions may differ from the float64 sum by k 2^-41 bin
areas; the tolerance allows one such unit per object."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2502_17632_amd import workload as W

from parity import log

pytestmark = pytest.mark.gpu


def test_density_matches_the_oracle_random_objects():
    import torch
    import paper_2502_17632_amd as gift
    rng = np.random.default_rng(8)
    n = 5000
    x = np.column_stack([rng.uniform(-5, 105, n), rng.uniform(-5, 105, n), rng.normal(size=n)])
    w = rng.uniform(0.2, 6.0, n)
    h = rng.uniform(0.2, 6.0, n)
    box = (0.0, 0.0, 100.0, 100.0)
    ref = O.bin_density(x[:, :2], w, h, box, 37, 23)
    for dt in (torch.float64, torch.float32):
        xt = torch.tensor(x, dtype=dt, device="cuda")  # ld 3: a third column is ignored
        xin = xt.double().cpu().numpy()[:, :2]
        ref = O.bin_density(xin, w, h, box, 37, 23)
        d = gift.bin_density(xt, box, 37, 23, widths=torch.tensor(w, device="cuda"),
                             heights=torch.tensor(h, device="cuda")).cpu().numpy()
        bin_area = (100 / 37) * (100 / 23)
        assert np.allclose(d, ref, rtol=1e-12, atol=n * 2.0 ** -40 * bin_area), \
            np.abs(d - ref).max()
        d2 = gift.bin_density(xt, box, 37, 23, widths=torch.tensor(w, device="cuda"),
                              heights=torch.tensor(h, device="cuda")).cpu().numpy()
        assert np.array_equal(d, d2)


def test_density_of_the_filtered_medium_placement():
    import torch
    import paper_2502_17632_amd as gift
    nl = W.medium(seed=3)
    x = W.make_signal(nl, seed=3)
    g = gift.build_graph(nl.num_cells, nl.net_ptr, nl.pin_cell, star_threshold=16)
    xt = torch.tensor(x, device="cuda")
    y = gift.filter_placement(g, [4.0] * 4, [1, 2, 4, 8], [0.25] * 4, xt,
                              out_dtype=torch.float64)
    box = (0.0, 0.0, 1000.0, 1000.0)
    for name, sig in (("initial", xt), ("filtered", y)):
        d = gift.bin_density(sig, box, 64, 64, w0=1.0, h0=1.0)
        ref = O.bin_density(sig.cpu().numpy(), 1.0, 1.0, box, 64, 64)
        tol = nl.num_cells * 2.0 ** -40 * (1000 / 64) ** 2
        assert np.allclose(d.cpu().numpy(), ref, rtol=1e-12, atol=tol), \
            np.abs(d.cpu().numpy() - ref).max()
        over = gift.density_overflow(d, box, 1.0, float(nl.num_cells))
        ref_over = O.density_overflow(ref, box, 1.0, float(nl.num_cells))
        # each bin of the map may differ by tol; the overflow by at most
        # (bins) * tol / total area
        assert abs(over - ref_over) <= 64 * 64 * tol / nl.num_cells + 1e-12, (over, ref_over)
        log(f"[density] {name}: max {d.max().item():.1f} of bin area "
            f"{(1000 / 64) ** 2:.1f}, overflow at target 1: {over:.4f}")
    g.close()


def test_density_arguments():
    import torch
    import paper_2502_17632_amd as gift
    x = torch.zeros((3, 2), device="cuda")
    with pytest.raises(gift.GiftError):
        gift.bin_density(x, (0, 0, 0, 1), 4, 4)
    with pytest.raises(gift.GiftError):
        gift.bin_density(x, (0, 0, 1, 1), 0, 4)
    with pytest.raises(gift.GiftError):
        gift.bin_density(x, (0, 0, 1, 1), 4, 4, w0=0.0)
    e = gift.bin_density(torch.zeros((0, 2), device="cuda"), (0, 0, 1, 1), 2, 2)
    assert float(e.abs().sum()) == 0.0
