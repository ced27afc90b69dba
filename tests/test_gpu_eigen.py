"""Eigenvector placement [u_2, u_3] (Section 3.3.1, eq. ideal_filter) on the
GPU against the dense oracle (needs a GPU).  Component labels are integers
and must be identical; eigenvalues and eigenvectors agree to what the
residual tolerance allows (the oracle is a dense float64 solve)."""
import numpy as np
import pytest

from oracle import eigen as EG
from oracle import oracle as O
from paper_2502_17632_amd import workload as W

from parity import log

pytestmark = pytest.mark.gpu


def _netlist(num_cells, nets):
    net_ptr = np.zeros(len(nets) + 1, dtype=np.int64)
    net_ptr[1:] = np.cumsum([len(n) for n in nets])
    pins = np.array([c for n in nets for c in n], dtype=np.int32)
    return num_cells, net_ptr, pins


def _check(gift, torch, n, net_ptr, pins, threshold, tol=1e-11, what="", model="inv_m1"):
    g = gift.build_graph(n, net_ptr, pins, star_threshold=threshold, sigmas=[1.0],
                         weight_model=model)
    y, info, lab = gift.eigen_placement(g, tol=tol, max_iter=2000, labels=True)
    torch.cuda.synchronize()
    lam, vec, labels, gl, full = EG.eigen_placement(n, net_ptr, pins,
                                                    1 if model == "two_over_m" else 0)
    yh = y.cpu().numpy()
    log(f"[eigen] {what}: lambda {info['lambda']} (oracle {lam}), residual {info['residual']}, "
        f"{info['iterations']} iterations, {info['sweeps']} sweeps, component {gl} "
        f"({info['component_cells']} cells)")
    assert info["converged"]
    # the oracle lists the virtual rows in net order; the library labels them
    # by median cell (the oracle graph in that labelling gives the net of
    # each virtual row)
    exp = EG.row_labels(n, net_ptr, pins, threshold)
    if threshold > 0:
        star_nets = [e for e in range(len(net_ptr) - 1)
                     if threshold < len(set(pins[net_ptr[e]:net_ptr[e + 1]].tolist()))]
        og = O.build_graph(n, net_ptr, pins, star_threshold=threshold, star_order="median")
        rank = {e: i for i, e in enumerate(star_nets)}
        exp = np.concatenate([exp[:n], exp[n + np.array([rank[int(e)] for e in og.virt_net],
                                                        dtype=np.int64)]])
        og.close()
    assert np.array_equal(lab.cpu().numpy(), exp)
    assert info["component_label"] == gl and info["component_cells"] == np.count_nonzero(labels == gl)
    b = info["spectral_bound"]
    assert np.allclose(info["lambda"], lam, rtol=1e-9, atol=tol * b)
    # eigenvector error <= residual / gap to the rest of the spectrum
    for q in range(2):
        gap = min(abs(full[1 + q] - full[q]), abs(full[2 + q] - full[1 + q]))
        bound = 10 * tol * b / gap + 1e-12
        err = min(np.linalg.norm(yh[:, q] - vec[:, q]), np.linalg.norm(yh[:, q] + vec[:, q]))
        assert err <= bound, (q, err, bound)
        assert yh[int(np.argmax(np.abs(yh[:, q]))), q] > 0
    assert np.all(yh[labels != gl] == 0.0)
    g.close()
    return yh, info


def test_tiny_design_matches_the_oracle():
    import torch
    import paper_2502_17632_amd as gift
    nl = W.tiny()
    _check(gift, torch, nl.num_cells, nl.net_ptr, nl.pin_cell, 16, what="tiny")


@pytest.mark.parametrize("threshold", [0, 8, 16])
def test_star_nets_are_eliminated_exactly(threshold):
    """Star rows at the mean of their cells give exactly the clique model's
    Laplacian, so the result does not depend on the star threshold."""
    import torch
    import paper_2502_17632_amd as gift
    nl = W.sized(1500, seed=7)
    _check(gift, torch, nl.num_cells, nl.net_ptr, nl.pin_cell, threshold,
           what=f"1.5k cells, star threshold {threshold}")


def test_two_over_m_weights():
    """The 2/M weight model (Section 2.2, eq. wire_eq): stars of weight
    M w(M) = 2 still eliminate exactly."""
    import torch
    import paper_2502_17632_amd as gift
    nl = W.sized(1200, seed=9)
    _check(gift, torch, nl.num_cells, nl.net_ptr, nl.pin_cell, 16, what="2/M weights",
           model="two_over_m")


def test_giant_component_is_not_the_first():
    """A small path first (cells 0..9), then isolated cells, then a larger
    design: the labels name each component's smallest cell and the vectors
    vanish outside the largest one."""
    import torch
    import paper_2502_17632_amd as gift
    big = W.sized(600, seed=3)
    off = 40
    nets = [[i, i + 1] for i in range(9)]
    for e in range(len(big.net_ptr) - 1):
        nets.append([int(c) + off for c in big.pin_cell[big.net_ptr[e]:big.net_ptr[e + 1]]])
    n, net_ptr, pins = _netlist(big.num_cells + off, nets)
    y, info = _check(gift, torch, n, net_ptr, pins, 16, what="two designs")
    assert info["component_label"] >= off


def test_too_small_components_are_rejected():
    import torch
    import paper_2502_17632_amd as gift
    n, net_ptr, pins = _netlist(40, [[2 * i, 2 * i + 1] for i in range(20)])
    g = gift.build_graph(n, net_ptr, pins, star_threshold=16, sigmas=[1.0])
    with pytest.raises(gift.GiftError) as e:
        gift.eigen_placement(g)
    assert e.value.status == 1
    g.close()


def test_medium_design_properties():
    """On the 202k-cell design the dense oracle is out of reach: the labels
    are checked against the oracle's union-find, and the vectors by their
    residual, orthonormality, zero mean on the component and Rayleigh
    quotient S(u) / |u|^2 (the smoothness evaluator, another kernel)."""
    import torch
    import paper_2502_17632_amd as gift
    nl = W.medium()
    g = gift.build_graph(nl.num_cells, nl.net_ptr, nl.pin_cell, star_threshold=16, sigmas=[1.0])
    y, info, lab = gift.eigen_placement(g, tol=1e-9, max_iter=3000, labels=True)
    torch.cuda.synchronize()
    log(f"[eigen] medium: lambda {info['lambda']}, residual {info['residual']}, "
        f"{info['iterations']} iterations, {info['sweeps']} sweeps, "
        f"{info['component_cells']} cells in the component")
    labels = EG.components(nl.num_cells, nl.net_ptr, nl.pin_cell)
    assert np.array_equal(lab.cpu().numpy()[:nl.num_cells], labels)
    gl = EG.giant_component(labels)
    assert info["component_label"] == gl
    assert info["converged"]
    yh = y.cpu().numpy()
    assert np.allclose(yh.T @ yh, np.eye(2), atol=1e-9)
    assert np.allclose(yh[labels == gl].sum(axis=0), 0.0, atol=1e-8)
    assert np.all(yh[labels != gl] == 0.0)
    m = gift.evaluate_placement(g, y)
    for q in range(2):
        rq = m["smoothness"][q] / m["norm2"][q]
        assert abs(rq - info["lambda"][q]) <= 1e-8 * max(1.0, info["lambda"][q]), (rq, info)
    assert 0.0 < info["lambda"][0] <= info["lambda"][1]
    g.close()
