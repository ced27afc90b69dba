"""The exact filter (I + L~_sigma)^-1 g by conjugate gradients on the GPU
against the CPU oracle's converged solution (needs a GPU)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2502_17632_amd import workload as W

from parity import colwise_error, log

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("storage,tol,bar", [("f32", 1e-6, 1e-5), ("f64", 1e-12, 1e-10)])
def test_exact_filter_matches_the_oracle(storage, tol, bar):
    import torch
    import paper_2502_17632_amd as gift
    nl = W.medium(seed=5)
    x = W.make_signal(nl, (10.0,), seed=5)
    og = O.build_netlist(nl, star_threshold=16, star_order="median")
    g = gift.build_graph(nl.num_cells, nl.net_ptr, nl.pin_cell, star_threshold=16,
                         storage=storage, sigmas=[2.0])
    dt = torch.float32 if storage == "f32" else torch.float64
    xin = x.astype(np.float32).astype(np.float64) if storage == "f32" else x
    xt = torch.tensor(xin, dtype=dt, device="cuda")
    fixed = torch.tensor(nl.fixed, dtype=torch.uint8, device="cuda")
    y, it = gift.filter_exact(g, 2.0, xt, tol=tol, out_dtype=torch.float64, fixed=fixed)
    ref, oit = og.filter_exact(xin, 2.0, fixed=nl.fixed)
    err = colwise_error(y.cpu().numpy(), ref)
    log(f"[exact] {storage}: {it} iterations (oracle {oit} to 1e-14), normwise error {err}")
    assert np.all(err <= bar), err
    assert it <= 80
    # the paper's filter is the first-order approximation of this one: the
    # two agree to first order, not exactly (checked loosely on a smooth input)
    g.close()


def test_exact_filter_small_cases_and_errors():
    import torch
    import paper_2502_17632_amd as gift
    # two cells, one net: g' = mean + (g - mean)(1 + s)/(s + 3)
    g = gift.build_graph(2, np.array([0, 2]), np.array([0, 1]), storage="f64", sigmas=[4.0])
    y, _ = gift.filter_exact(g, 4.0, torch.tensor([[0.0], [1.0]], dtype=torch.float64,
                                                  device="cuda"), tol=1e-14,
                             out_dtype=torch.float64)
    k = 5.0 / 7.0
    assert np.allclose(y.cpu().numpy()[:, 0], [0.5 - 0.5 * k, 0.5 + 0.5 * k], rtol=1e-13)
    with pytest.raises(gift.GiftError):  # sigma not prepared
        gift.filter_exact(g, 2.0, torch.zeros((2, 1), device="cuda"))
    g.close()
    nl = W.tiny()
    gb = gift.build_graph(nl.num_cells, nl.net_ptr, nl.pin_cell, storage="bf16", sigmas=[2.0])
    with pytest.raises(gift.GiftError) as e:
        gift.filter_exact(gb, 2.0, torch.zeros((nl.num_cells, 2), device="cuda"))
    assert e.value.status == 4
    gb.close()
