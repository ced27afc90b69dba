"""Pins that tie the CPU oracle to the paper and to mathematics.

Each ``pin_*`` function takes an oracle library handle and raises
``AssertionError`` when the oracle disagrees with what the paper or the
mathematics fixes.  ``test_oracle_pins.py`` runs them on the real oracle and
``test_oracle_mutants.py`` runs them on deliberately broken copies of the
oracle source, each of which must fail at least one pin.
"""
from __future__ import annotations

import os
from fractions import Fraction

import numpy as np
import scipy.sparse as sp

from oracle import dense as D
from oracle import oracle as O
from paper_2502_17632_amd import workload as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = (t.strip() for t in line.split("=", 1))
            out[k] = [Fraction(t) for t in v.split()]
    return out


def _random_netlist(rng, n_cells, n_nets, max_pins, dup_prob=0.2):
    """Tiny netlists with the awkward cases: repeated pins on one net, 0- and
    1-pin nets, parallel nets and isolated cells."""
    sizes = rng.integers(0, max_pins + 1, size=n_nets)
    pins = []
    for m in sizes:
        cells = list(rng.integers(0, n_cells, size=m))
        if m >= 2 and rng.random() < dup_prob:
            cells.append(cells[0])  # a repeated pin
        pins.append(cells)
    if n_nets >= 2 and len(pins[0]) >= 2:
        pins[1] = list(pins[0][:2])  # a parallel net on one pair
    net_ptr = np.zeros(n_nets + 1, dtype=np.int64)
    net_ptr[1:] = np.cumsum([len(p) for p in pins])
    pin_cell = np.array([c for p in pins for c in p], dtype=np.int32)
    return net_ptr, pin_cell


def _dense_from(g: O.OracleGraph) -> np.ndarray:
    r = g.num_rows
    a = np.zeros((r, r))
    for i in range(r):
        for p in range(g.row_ptr[i], g.row_ptr[i + 1]):
            a[i, g.col[p]] = g.w[p]
    return a


def _csr(g: O.OracleGraph, vals):
    return sp.csr_matrix((vals, g.col, g.row_ptr), shape=(g.num_rows, g.num_rows))


# -------------------------------------------------------------------------


def pin_golden_two_cell(lib):
    """The hand-derived two-cell example of the paper's filter."""
    gd = _read_golden("two_cell_paper_filter.txt")
    g = O.build_graph(int(gd["num_cells"][0]), np.array(gd["net_ptr"], dtype=np.int64),
                      np.array(gd["pin_cell"], dtype=np.int32), lib=lib)
    x = np.array([float(v) for v in gd["x"]])[:, None]
    y = g.filter(x, [float(v) for v in gd["sigma"]], [int(v) for v in gd["order"]],
                 [float(v) for v in gd["alpha"]])
    exp = np.array([float(v) for v in gd["expected"]])
    assert np.allclose(y[:, 0], exp, rtol=0, atol=1e-15), (y[:, 0], exp)
    for s, k, key in ((2.0, 2, "offdiag_A2_pow2"), (4.0, 2, "offdiag_A4_pow2"),
                      (4.0, 4, "offdiag_A4_pow4")):
        yk = g.filter(x, [s], [k], [1.0])
        assert abs(yk[0, 0] - float(gd[key][0])) <= 1e-15, (s, k, yk[0, 0])
    g.close()


def pin_clique_closed_form(lib):
    """One net of M cells: every cell has degree (M-1) w, and
    A~^k x = mean(x) 1 + mu^k (x - mean(x) 1), mu = (sigma - w)/(d + sigma)."""
    rng = np.random.default_rng(1)
    for model in (O.W_INV_M1, O.W_TWO_OVER_M):
        for m in (2, 3, 5, 9):
            w = 2.0 / m if model == O.W_TWO_OVER_M else 1.0 / (m - 1)
            d = (m - 1) * w
            perm = rng.permutation(m).astype(np.int32)
            g = O.build_graph(m, np.array([0, m], dtype=np.int64), perm,
                              weight_model=model, lib=lib)
            assert g.nnz == m * (m - 1)
            x = rng.normal(size=(m, 2)) * 10 + 3
            for s in (0.5, 2.0, 4.0):
                mu = (s - w) / (d + s)
                for k in (1, 2, 3, 7):
                    y = g.filter(x, [s], [k], [1.0])
                    xb = x.mean(axis=0, keepdims=True)
                    exp = xb + mu ** k * (x - xb)
                    assert np.allclose(y, exp, rtol=1e-13, atol=1e-13), (model, m, s, k)
            g.close()


def pin_hand_built(lib):
    """Hand-built weights and degrees (clique model, w = 1/(M-1))."""
    g = O.build_graph(4, np.array([0, 4]), np.array([3, 1, 0, 2]), lib=lib)
    assert g.nnz == 12 and np.all(g.w == 1.0 / 3.0) and np.all(g.deg == 1.0)
    g = O.build_graph(2, np.array([0, 2, 4]), np.array([0, 1, 1, 0]), lib=lib)
    assert list(g.col) == [1, 0] and list(g.w) == [2.0, 2.0]
    g = O.build_graph(3, np.array([0, 3, 5]), np.array([0, 1, 2, 1, 0]), lib=lib)
    a = _dense_from(g)
    assert a[0, 1] == 1.5 and a[1, 0] == 1.5 and a[0, 2] == 0.5 and a[1, 2] == 0.5
    assert list(g.deg) == [2.0, 2.0, 1.0]
    # repeated pins and a single-cell net add nothing
    g = O.build_graph(3, np.array([0, 3, 5]), np.array([0, 0, 1, 2, 2]), lib=lib)
    assert g.nnz == 2 and list(g.w) == [1.0, 1.0] and g.deg[2] == 0.0


def pin_brute_force_structure(lib):
    """CSR, weights and degrees equal (bitwise) a dense matrix accumulated
    straight from the net model, for both weight models, with and without
    star expansion."""
    rng = np.random.default_rng(2)
    for trial in range(40):
        n = int(rng.integers(1, 25))
        e = int(rng.integers(0, 30))
        net_ptr, pin_cell = _random_netlist(rng, n, e, 9)
        for model in (O.W_INV_M1, O.W_TWO_OVER_M):
            for thr in (0, 3, 5):
                g = O.build_graph(n, net_ptr, pin_cell, weight_model=model,
                                  star_threshold=thr, lib=lib)
                a, star = D.dense_adjacency(n, net_ptr, pin_cell, weight_model=model,
                                            star_threshold=thr)
                assert g.num_rows == a.shape[0], (trial, model, thr)
                assert list(g.virt_net) == star
                rows, cols = np.nonzero(a)
                ptr = np.zeros(a.shape[0] + 1, dtype=np.int64)
                np.add.at(ptr, rows + 1, 1)
                ptr = np.cumsum(ptr)
                assert np.array_equal(g.row_ptr, ptr)
                assert np.array_equal(g.col, cols.astype(np.int32))
                assert np.array_equal(g.w.view(np.uint64), a[rows, cols].view(np.uint64))
                dd = D.dense_degree(a)
                assert np.array_equal(g.deg.view(np.uint64), dd.view(np.uint64))
                g.close()


def pin_spectral(lib):
    """The filter equals U h(Lambda) U^T x from a dense eigendecomposition of
    the augmented normalised Laplacian, h(l) = sum alpha (1 - l)^k."""
    rng = np.random.default_rng(3)
    cases = [([4.0] * 4, [1, 2, 4, 8], [0.25] * 4),
             ([2.0, 4.0, 4.0], [2, 2, 4], [0.1, 0.7, 0.2]),
             ([0.0, 1.0, 3.5], [3, 1, 5], [0.5, -0.25, 0.75])]
    for trial in range(24):
        n = int(rng.integers(2, 30))
        e = int(rng.integers(1, 40))
        net_ptr, pin_cell = _random_netlist(rng, n, e, 8)
        thr = int(rng.choice([0, 3, 4]))
        model = int(rng.integers(0, 2))
        g = O.build_graph(n, net_ptr, pin_cell, weight_model=model, star_threshold=thr,
                          lib=lib)
        a, star = D.dense_adjacency(n, net_ptr, pin_cell, weight_model=model,
                                    star_threshold=thr)
        x = rng.normal(size=(n, 2)) * 30 + 500
        xe = D.extend_signal(x, net_ptr, pin_cell, star)
        for sig, k, al in cases:
            y = g.filter(x, sig, k, al)
            ref = D.spectral_filter(a, xe, sig, k, al)[:n]
            err = np.abs(y - ref).max() / max(np.abs(ref).max(), 1e-300)
            assert err <= 1e-12, (trial, sig, k, err)
        g.close()


def pin_theorem1_fixed_point(lib):
    """Theorem 1 with self-loops: sqrt(d + sigma) is an eigenvector of A~_sigma
    with eigenvalue 1; so with one sigma and weights summing to one it is a
    fixed point of the whole filter."""
    nl = W.make_netlist(600, 20, 700, dist="zipf", param=2.2, cap=40, seed=5)
    g = O.build_netlist(nl, lib=lib)
    for s in (0.5, 2.0, 4.0):
        a, dl = g.normalise(s)
        m = _csr(g, a) + sp.diags(dl)
        v = np.sqrt(g.deg + s)
        assert np.allclose(m @ v, v, rtol=1e-13, atol=0)
        y = g.filter(np.stack([v, 2 * v], axis=1), [s] * 3, [1, 3, 6], [0.2, 0.5, 0.3])
        assert np.allclose(y, np.stack([v, 2 * v], axis=1), rtol=1e-12, atol=0)
    g.close()


def pin_spectrum(lib):
    """Eigenvalues of A~_sigma lie in [1 - 2 max d/(d + sigma), 1] (since the
    Laplacian is at most 2D) and a larger self-loop lowers the largest
    eigenvalue of the normalised Laplacian (Section 3.2.1, Fig. 2a)."""
    rng = np.random.default_rng(6)
    net_ptr, pin_cell = _random_netlist(rng, 40, 60, 6, dup_prob=0.0)
    g = O.build_graph(40, net_ptr, pin_cell, lib=lib)
    tops = []
    for s in (0.0, 1.0, 2.0, 3.0):
        a, dl = g.normalise(s)
        m = (_csr(g, a) + sp.diags(dl)).toarray()
        assert np.allclose(m, m.T, rtol=4e-16, atol=0)
        lam = np.linalg.eigvalsh(m)
        conn = g.deg > 0
        lo = 1.0 - 2.0 * np.max(g.deg[conn] / (g.deg[conn] + s))
        assert lam.max() <= 1.0 + 1e-12 and lam.min() >= lo - 1e-12, (s, lam.min(), lo)
        assert abs(lam.max() - 1.0) < 1e-12
        tops.append(1.0 - lam.min())
    assert all(tops[i + 1] < tops[i] for i in range(len(tops) - 1)), tops
    g.close()


def pin_isolated_and_fixed(lib):
    """An isolated cell keeps (sum alpha) x with a self-loop and vanishes
    without one; fixed rows are restored from the input on request."""
    g = O.build_graph(4, np.array([0, 2, 4]), np.array([0, 1, 1, 2]), lib=lib)
    x = np.array([[1.0, 2.0], [3.0, 4.0], [5.0, 6.0], [7.0, 8.0]])
    y = g.filter(x, [2.0, 4.0], [3, 1], [0.3, 0.5])
    assert np.allclose(y[3], 0.8 * x[3], rtol=1e-15)
    y0 = g.filter(x, [0.0], [2], [1.0])
    assert np.all(y0[3] == 0.0)
    fixed = np.array([0, 1, 0, 1], dtype=np.uint8)
    yf = g.filter(x, [2.0], [2], [1.0], fixed=fixed)
    yn = g.filter(x, [2.0], [2], [1.0])
    assert np.array_equal(yf[[1, 3]], x[[1, 3]]) and np.array_equal(yf[[0, 2]], yn[[0, 2]])
    g.close()


def pin_star_schur(lib):
    """A star of weight M w(M) around a virtual node is the clique exactly:
    eliminating the virtual nodes from the star graph's Laplacian (Schur
    complement) gives the clique graph's Laplacian."""
    rng = np.random.default_rng(7)
    for model in (O.W_INV_M1, O.W_TWO_OVER_M):
        net_ptr, pin_cell = _random_netlist(rng, 30, 25, 9)
        gc = O.build_graph(30, net_ptr, pin_cell, weight_model=model, lib=lib)
        gs = O.build_graph(30, net_ptr, pin_cell, weight_model=model, star_threshold=3,
                           lib=lib)
        assert gs.num_virtual > 0
        lc = np.diag(gc.deg) - _dense_from(gc)
        ls = np.diag(gs.deg) - _dense_from(gs)
        n = 30
        schur = ls[:n, :n] - ls[:n, n:] @ np.linalg.solve(ls[n:, n:], ls[n:, :n])
        assert np.allclose(schur, lc, rtol=0, atol=1e-12)
        gc.close(); gs.close()


def pin_star_start_value(lib):
    """The start value of a star's virtual row (reading D4: the mean of its
    cells), by a closed form of eq. A_formulation.  One star net of M cells
    and weight g = M w(M): every cell has degree g and the virtual node M g,
    so one pass gives, for cell c,
        y_c = g / sqrt((g + s)(M g + s)) * x_v + s / (g + s) * x_c,
    with x_v the virtual row's start value; a start other than the mean of
    the cells (another divisor, a missing cell) changes every y_c."""
    for m, model, s, x in ((5, O.W_INV_M1, 2.0, [3.0, -1.0, 7.5, 0.25, 10.0]),
                           (7, O.W_TWO_OVER_M, 0.5, [1.0, 2.0, 4.0, 8.0, 16.0, 32.0, 64.0])):
        net_ptr = np.array([0, m], dtype=np.int64)
        pins = np.arange(m, dtype=np.int32)[::-1].copy()
        g = O.build_graph(m, net_ptr, pins, weight_model=model, star_threshold=m - 1, lib=lib)
        assert g.num_virtual == 1
        w = 1.0 / (m - 1) if model == O.W_INV_M1 else 2.0 / m
        gam = m * w
        xv = sum(x) / m
        a_cv = gam / np.sqrt((gam + s) * (m * gam + s))
        exp = np.array([a_cv * xv + s / (gam + s) * xc for xc in x])
        y = g.filter(np.array(x)[:, None], [s], [1], [1.0])[:, 0]
        assert np.allclose(y, exp, rtol=1e-14, atol=1e-14), (y, exp)
        g.close()


def pin_star_order_golden(lib):
    """Labelling of the virtual rows by the median cell of their net (the
    paper leaves the labelling free).  Ten cells, T = 2: the star nets and
    the medians of their ascending distinct cells (index M/2) are
    e0 {7,8,9} -> 8, e1 {0,1,2} -> 1, e2 {4,5,6} -> 5, e3 {1,2,3} -> 2 (its
    pins repeat a cell) and e5 {3,4,5,6} -> 5 (M even: the upper of the two
    middle cells); e4 {0,9} is a clique.  By median, ties by net id: e1, e3,
    e2, e5, e0.  In net order: e0, e1, e2, e3, e5."""
    nets = [[9, 7, 8], [2, 0, 1], [6, 4, 5], [3, 2, 1, 2], [0, 9], [6, 5, 4, 3]]
    net_ptr = np.cumsum([0] + [len(n) for n in nets]).astype(np.int64)
    pins = np.array([c for n in nets for c in n], dtype=np.int32)
    for order, exp in (("median", [1, 3, 2, 5, 0]), ("net", [0, 1, 2, 3, 5])):
        g = O.build_graph(10, net_ptr, pins, star_threshold=2, star_order=order, lib=lib)
        assert g.num_virtual == 5 and g.virt_net.tolist() == exp, (order, g.virt_net)
        for v, e in enumerate(exp):  # each virtual row holds its net's cells
            cells = sorted(set(nets[e]))
            assert g.col[g.row_ptr[10 + v]:g.row_ptr[11 + v]].tolist() == cells, (order, v)
        g.close()


def pin_star_order_relabels(lib):
    """Both labellings give one graph: on generated netlists with star nets,
    the median-labelled CSR equals the net-labelled one with the virtual rows
    and columns relabelled, weights bit for bit; degrees of virtual rows are
    bit-equal, those of cells (a sum over the row in ascending column, whose
    order the relabelling changes) equal to 1e-15; the medians of the virtual
    rows never decrease, and equal medians come in ascending net id."""
    rng = np.random.default_rng(11)
    for seed, thr in ((5, 4), (6, 8)):
        nl = W.make_netlist(400, 4, 420, cap=60, window=64, seed=seed)
        a = O.build_netlist(nl, star_threshold=thr, lib=lib)
        b = O.build_netlist(nl, star_threshold=thr, star_order="median", lib=lib)
        n, v = a.num_cells, a.num_virtual
        assert v > 10 and b.num_virtual == v
        pos = {int(e): i for i, e in enumerate(a.virt_net)}
        new_of_old = np.arange(n + v)
        for i, e in enumerate(b.virt_net):
            new_of_old[n + pos[int(e)]] = n + i
        for r in rng.permutation(n + v)[:200].tolist() + list(range(n, n + v)):
            ra = slice(a.row_ptr[r], a.row_ptr[r + 1])
            rb = slice(b.row_ptr[new_of_old[r]], b.row_ptr[new_of_old[r] + 1])
            ca, wa = new_of_old[a.col[ra]], a.w[ra]
            o = np.argsort(ca, kind="stable")
            assert np.array_equal(ca[o], b.col[rb]), r
            assert np.array_equal(wa[o].view(np.uint64), b.w[rb].view(np.uint64)), r
            if r >= n:
                assert a.deg[r] == b.deg[new_of_old[r]], r
            else:
                assert abs(a.deg[r] - b.deg[r]) <= 1e-15 * a.deg[r], r
        lens = np.diff(b.row_ptr[n:])
        med = b.col[b.row_ptr[n:-1] + lens // 2].astype(np.int64)
        key = med * (1 << 32) + b.virt_net.astype(np.int64)
        assert np.all(np.diff(key) > 0)
        a.close()
        b.close()


def pin_generated_invariants(lib):
    """On a generated clique-model netlist: weights are symmetric bit for bit,
    with w = 1/(M-1) every cell's degree is the number of nets it is on, and
    the degrees sum to the total pin count of the kept nets."""
    nl = W.tiny(seed=3)
    g = O.build_netlist(nl, lib=lib)
    a = _csr(g, g.w)
    assert (a != a.T).nnz == 0
    at = a.T.tocsr()
    at.sort_indices()
    assert np.array_equal(at.data.view(np.uint64), g.w.view(np.uint64))
    m = np.diff(nl.net_ptr)
    owner = np.repeat(np.arange(nl.num_nets), m)
    kept = m >= 2
    inc = np.bincount(nl.pin_cell[kept[owner]], minlength=nl.num_cells)
    assert np.allclose(g.deg, inc, rtol=4e-16 * 8, atol=0)
    assert abs(g.deg.sum() - m[kept].sum()) <= 1e-9 * m.sum()
    g.close()


def pin_invalid_input(lib):
    """Malformed netlists are refused."""
    import pytest
    with pytest.raises(O.OracleError):
        O.build_graph(2, np.array([0, 2]), np.array([0, 2]), lib=lib)
    with pytest.raises(O.OracleError):
        O.build_graph(2, np.array([0, 2, 1]), np.array([0, 1]), lib=lib)
    g = O.build_graph(2, np.array([0, 2]), np.array([0, 1]), lib=lib)
    with pytest.raises(O.OracleError):
        g.filter(np.zeros((2, 1)), [-1.0], [1], [1.0])
    with pytest.raises(O.OracleError):
        g.filter(np.zeros((2, 1)), [1.0], [0], [1.0])


def _dense_laplacian_from_netlist(n, net_ptr, pin_cell, model):
    """L = D - A of the clique model, accumulated straight from the netlist:
    every net of M >= 2 distinct cells adds w(M) to each pair."""
    a = np.zeros((n, n))
    for e in range(len(net_ptr) - 1):
        cells = sorted(set(int(c) for c in pin_cell[net_ptr[e]:net_ptr[e + 1]]))
        m = len(cells)
        if m < 2:
            continue
        w = 2.0 / m if model == O.W_TWO_OVER_M else 1.0 / (m - 1)
        for i in cells:
            for j in cells:
                if i != j:
                    a[i, j] += w
    return np.diag(a.sum(axis=1)) - a


def pin_evaluate_hand(lib):
    """Hand-computed metrics: nets {0,1,2}, {2,3}, a 1-pin net and a net whose
    two pins are one cell; x = (0, 3, 7, 1), y = (2, 2, 5, 0).
    S_x = (9 + 49 + 16) / 2 + 36 = 73, S_y = (0 + 9 + 9) / 2 + 25 = 34,
    HPWL_x = 7 + 6 = 13, HPWL_y = 3 + 5 = 8, |x|^2 = 59, |y|^2 = 33."""
    net_ptr = np.array([0, 3, 5, 6, 8], dtype=np.int64)
    pins = np.array([0, 1, 2, 2, 3, 1, 3, 3], dtype=np.int32)
    g = O.build_graph(4, net_ptr, pins, lib=lib)
    x = np.array([[0.0, 2.0], [3.0, 2.0], [7.0, 5.0], [1.0, 0.0]])
    S, n2, h = g.evaluate(x)
    assert np.array_equal(S, [73.0, 34.0]), S
    assert np.array_equal(n2, [59.0, 33.0]), n2
    assert np.array_equal(h, [13.0, 8.0]), h
    g.close()


def pin_evaluate_dense(lib):
    """S equals trace(G^T L G) with L = D - A built densely from the netlist
    (eq. smoothness, eq. wire_eq), for both weight models and any star
    threshold; the Rayleigh quotient of each Laplacian eigenvector is its
    eigenvalue (eq. smoothness_ray2); S and HPWL do not change when the whole
    placement moves."""
    rng = np.random.default_rng(21)
    for trial in range(6):
        n = int(rng.integers(3, 14))
        net_ptr, pins = _random_netlist(rng, n, int(rng.integers(1, 9)), 6)
        model = trial % 2
        L = _dense_laplacian_from_netlist(n, net_ptr, pins, model)
        x = rng.normal(size=(n, 3)) * 5
        for T in (0, 2):
            g = O.build_graph(n, net_ptr, pins, weight_model=model, star_threshold=T, lib=lib)
            S, n2, h = g.evaluate(x)
            exp = np.einsum("iq,ij,jq->q", x, L, x)
            assert np.allclose(S, exp, rtol=1e-12, atol=1e-9), (trial, T, S, exp)
            assert np.allclose(n2, (x * x).sum(axis=0), rtol=1e-14)
            S2, _, h2 = g.evaluate(x + 17.5)
            assert np.allclose(S2, S, rtol=1e-9, atol=1e-7) and np.allclose(h2, h, rtol=1e-12)
            lam, U = np.linalg.eigh(L)
            SU, nU, _ = g.evaluate(U)
            assert np.allclose(SU / nU, lam, rtol=1e-9, atol=1e-9), (SU / nU, lam)
            g.close()


def pin_exact_filter(lib):
    """The exact filter (I + L~_sigma)^-1 g of eq. derivative / eq. spectral:
    the conjugate-gradient result equals a dense solve of (2I - A~_sigma) g' = g
    and the spectral form U diag(1 / (2 - mu)) U^T g; on the two-cell example
    (A~_s = [[s, 1], [1, s]] / (1 + s)) the solution is known in closed form."""
    rng = np.random.default_rng(33)
    for trial in range(5):
        n = int(rng.integers(3, 14))
        net_ptr, pins = _random_netlist(rng, n, int(rng.integers(1, 9)), 6)
        T = 0 if trial % 2 == 0 else 3
        g = O.build_graph(n, net_ptr, pins, star_threshold=T, lib=lib)
        sigma = [0.5, 2.0, 4.0][trial % 3]
        x = rng.normal(size=(n, 2)) * 3
        y, it = g.filter_exact(x, sigma)
        a, d = g.normalise(sigma)
        At = _dense_from(g)
        for i in range(g.num_rows):
            for p in range(g.row_ptr[i], g.row_ptr[i + 1]):
                At[i, g.col[p]] = a[p]
        At[np.diag_indices(g.num_rows)] = d
        xe = np.zeros((g.num_rows, 2))
        xe[:n] = x
        for v in range(g.num_virtual):
            e = int(g.virt_net[v])
            cells = sorted(set(int(c) for c in pins[net_ptr[e]:net_ptr[e + 1]]))
            xe[n + v] = x[cells].mean(axis=0)
        M = 2 * np.eye(g.num_rows) - At
        ref = np.linalg.solve(M, xe)[:n]
        assert np.allclose(y, ref, rtol=1e-11, atol=1e-11), (trial, np.abs(y - ref).max())
        mu, U = np.linalg.eigh(At)
        spec = (U @ np.diag(1.0 / (2.0 - mu)) @ U.T @ xe)[:n]
        assert np.allclose(y, spec, rtol=1e-10, atol=1e-10)
        assert it <= g.num_rows + 1
        g.close()
    # two cells, one net: (2I - A~_s) has eigenvalues 1 (on [1, 1]) and
    # 2 - (s - 1)/(1 + s) (on [1, -1]), so g' = mean + (g - mean) (1 + s)/(s + 3)
    g = O.build_graph(2, np.array([0, 2], dtype=np.int64), np.array([0, 1], dtype=np.int32),
                      lib=lib)
    for s in (0.5, 2.0, 4.0):
        y, _ = g.filter_exact(np.array([[0.0], [1.0]]), s)
        k = (1 + s) / (s + 3)
        assert np.allclose(y[:, 0], [0.5 - 0.5 * k, 0.5 + 0.5 * k], rtol=1e-13, atol=1e-14)
    g.close()


def pin_bin_density(lib):
    """Bin density (eq. density_eq): hand-computed overlaps of a 2 x 1 cell
    on a 4 x 4 grid; the densities of a placement inside the region sum to the
    total cell area; a brute-force sampled overlap on random inputs."""
    d = O.bin_density(np.array([[1.0, 1.5]]), 2.0, 1.0, (0, 0, 4, 4), 4, 4, lib=lib)
    exp = np.zeros((4, 4))
    # x in [0, 2], y in [1, 2]: bins (0, 1) and (1, 1) fully covered
    exp[1, 0] = exp[1, 1] = 1.0
    assert np.array_equal(d, exp), d
    d = O.bin_density(np.array([[1.5, 1.0]]), 1.0, 1.0, (0, 0, 4, 4), 4, 4, lib=lib)
    exp = np.zeros((4, 4))
    exp[0, 1] = exp[1, 1] = 0.5  # x in [1, 2], y in [0.5, 1.5]
    assert np.allclose(d, exp), d
    rng = np.random.default_rng(4)
    x = rng.uniform(5, 95, size=(200, 2))
    w = rng.uniform(0.5, 4.0, size=200)
    h = rng.uniform(0.5, 4.0, size=200)
    d = O.bin_density(x, w, h, (0, 0, 100, 100), 7, 5, lib=lib)
    assert np.isclose(d.sum(), (w * h).sum(), rtol=1e-12)
    # one cell against an analytic per-bin overlap computed independently
    for v in range(5):
        one = O.bin_density(x[v:v + 1], w[v], h[v], (0, 0, 100, 100), 7, 5, lib=lib)
        xs = np.clip([x[v, 0] - w[v] / 2, x[v, 0] + w[v] / 2], 0, 100)
        ys = np.clip([x[v, 1] - h[v] / 2, x[v, 1] + h[v] / 2], 0, 100)
        ex = np.zeros((5, 7))
        for j in range(5):
            for i in range(7):
                lx = max(0.0, min(xs[1], (i + 1) * 100 / 7) - max(xs[0], i * 100 / 7))
                ly = max(0.0, min(ys[1], (j + 1) * 20) - max(ys[0], j * 20))
                ex[j, i] = lx * ly
        assert np.allclose(one, ex, rtol=1e-12, atol=1e-12)
    # overflow: the 2 x 1 cell above covers two unit bins fully; at target
    # 0.5 each exceeds by 0.5, over a total object area of 2
    d = O.bin_density(np.array([[1.0, 1.5]]), 2.0, 1.0, (0, 0, 4, 4), 4, 4, lib=lib)
    assert O.density_overflow(d, (0, 0, 4, 4), 0.5, 2.0, lib=lib) == 0.5
    assert O.density_overflow(d, (0, 0, 4, 4), 1.0, 2.0, lib=lib) == 0.0
    # two unit cells stacked on one bin of area 1: excess 1 at target 1
    d = O.bin_density(np.array([[0.5, 0.5], [0.5, 0.5]]), 1.0, 1.0, (0, 0, 2, 2), 2, 2, lib=lib)
    assert O.density_overflow(d, (0, 0, 2, 2), 1.0, 2.0, lib=lib) == 0.5
    # bins of area 4 (8 x 8 region, 4 x 4 grid): target 0.25 allows one unit
    d = np.zeros((4, 4))
    d[2, 3] = 3.0
    assert O.density_overflow(d, (0, 0, 8, 8), 0.25, 3.0, lib=lib) == 2.0 / 3.0


def _path_netlist(cells):
    """2-pin nets joining consecutive entries of `cells` (a path graph)."""
    pins = []
    for a, b in zip(cells[:-1], cells[1:]):
        pins += [b, a] if (a + b) % 2 else [a, b]
    net_ptr = np.arange(0, len(pins) + 1, 2, dtype=np.int64)
    return net_ptr, np.array(pins, dtype=np.int32)


def pin_eigen_path(lib, eig=None):
    """Eigenvector placement (eq. ideal_filter on L = D - A, Section 2.1): a
    chain of n cells joined by 2-pin nets (weight 1) is the path graph, whose
    Laplacian has eigenvalues 2 - 2 cos(pi k / n) and eigenvectors
    cos(pi k (i + 1/2) / n), k = 0..n-1."""
    from oracle import eigen as E
    eig = eig or E
    for n in (5, 9, 16):
        net_ptr, pins = _path_netlist(list(range(n)))
        lam, vec, labels, g, _ = eig.eigen_placement(n, net_ptr, pins)
        k = np.array([1.0, 2.0])
        assert np.allclose(lam, 2 - 2 * np.cos(np.pi * k / n), rtol=1e-12, atol=1e-13), lam
        assert np.all(labels == 0) and g == 0
        for q in range(2):
            u = np.cos(np.pi * (q + 1) * (np.arange(n) + 0.5) / n)
            u /= np.linalg.norm(u)
            assert min(np.linalg.norm(vec[:, q] - u), np.linalg.norm(vec[:, q] + u)) < 1e-10
            assert vec[int(np.argmax(np.abs(vec[:, q]))), q] > 0


def pin_eigen_complete(lib, eig=None):
    """One net of M cells is the complete graph with weight w(M): eigenvalues
    0 and M w(M) (M - 1 times), for both weight models."""
    from oracle import eigen as E
    eig = eig or E
    m = 6
    net_ptr = np.array([0, m], dtype=np.int64)
    pins = np.array([3, 0, 5, 1, 4, 2], dtype=np.int32)
    for model, wm in ((0, 1.0 / (m - 1)), (1, 2.0 / m)):
        lam, vec, labels, g, full = eig.eigen_placement(m, net_ptr, pins, model)
        assert np.allclose(full, [0.0] + [m * wm] * (m - 1), rtol=1e-12, atol=1e-12), full
        # the eigenvectors are orthonormal and orthogonal to the constant
        assert np.allclose(vec.T @ vec, np.eye(2), atol=1e-12)
        assert np.allclose(vec.sum(axis=0), 0.0, atol=1e-12)


def pin_eigen_components(lib, eig=None):
    """Components and the giant component: two disjoint paths (cells 0..4 and
    10..17), isolated cells and a separate pair; labels are the smallest cell
    of each component (checked against scipy's connected components), the
    8-cell path is the giant one, cells outside it get 0, and its eigenvalues
    are those of the 8-path."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    from oracle import eigen as E
    eig = eig or E
    n = 22
    p1, q1 = _path_netlist([4, 2, 0, 1, 3])
    p2, q2 = _path_netlist(list(range(10, 18)))
    pins = np.concatenate([q1, q2, np.array([19, 20, 7, 7], dtype=np.int32)])
    net_ptr = np.arange(0, len(pins) + 1, 2, dtype=np.int64)
    lam, vec, labels, g, _ = eig.eigen_placement(n, net_ptr, pins)
    assert g == 10 and np.count_nonzero(labels == g) == 8
    assert np.all(vec[labels != g] == 0.0)
    assert np.allclose(lam, 2 - 2 * np.cos(np.pi * np.array([1.0, 2.0]) / 8), rtol=1e-12)
    rng = np.random.default_rng(12)
    for trial in range(4):
        nc = int(rng.integers(20, 60))
        net_ptr, pins = _random_netlist(rng, nc, int(rng.integers(5, 25)), 5)
        lab = eig.components(nc, net_ptr, pins)
        rows, cols = [], []
        for e in range(len(net_ptr) - 1):
            cs = pins[net_ptr[e]:net_ptr[e + 1]]
            for c in cs[1:]:
                rows.append(cs[0])
                cols.append(c)
        adj = sp.coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(nc, nc))
        k, ref = connected_components(adj, directed=False)
        for comp in range(k):
            members = np.flatnonzero(ref == comp)
            assert np.all(lab[members] == members.min())


def _csr_of_dense(a):
    """Canonical CSR (ascending columns, no diagonal) of a dense matrix."""
    rows, cols = np.nonzero(a)
    keep = rows != cols
    rows, cols = rows[keep], cols[keep]
    row_ptr = np.zeros(a.shape[0] + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    return np.cumsum(row_ptr), cols.astype(np.int32), a[rows, cols].astype(np.float64)


def pin_import_csr(lib):
    """A caller-supplied weighted graph (Section 2.1's A = {w_ij}, the input of
    Algorithm 1): the paper's two-cell example through the import path; the
    weighted complete graph's closed form; degrees bit-equal to a dense
    left-to-right sum and the filter equal to the dense spectral form on
    random weighted graphs; the CSR a netlist builds, imported, gives the same
    bits; malformed CSRs are refused."""
    gd = _read_golden("two_cell_paper_filter.txt")
    g = O.import_csr(np.array([0, 1, 2]), np.array([1, 0]), np.array([1.0, 1.0]), lib=lib)
    y = g.filter(np.array([float(v) for v in gd["x"]])[:, None],
                 [float(v) for v in gd["sigma"]], [int(v) for v in gd["order"]],
                 [float(v) for v in gd["alpha"]])
    assert np.allclose(y[:, 0], [float(v) for v in gd["expected"]], rtol=0, atol=1e-15)
    g.close()
    # complete graph K_M with one weight w: A~^k x = xbar 1 + mu^k (x - xbar 1),
    # mu = (sigma - w) / ((M - 1) w + sigma)
    rng = np.random.default_rng(21)
    for m, w in ((3, 0.37), (7, 2.5), (12, 0.125)):
        a = w * (np.ones((m, m)) - np.eye(m))
        rp, cl, wv = _csr_of_dense(a)
        g = O.import_csr(rp, cl, wv, lib=lib)
        assert np.allclose(g.deg, (m - 1) * w, rtol=1e-15, atol=0)
        x = rng.normal(size=(m, 2)) * 10 + 300
        xb = x.mean(axis=0, keepdims=True)
        for s in (0.5, 4.0):
            mu = (s - w) / ((m - 1) * w + s)
            for k in (1, 3):
                yk = g.filter(x, [s], [k], [1.0])
                assert np.allclose(yk, xb + mu ** k * (x - xb), rtol=1e-13, atol=1e-12)
        g.close()
    # random symmetric weighted graphs with isolated nodes
    cases = [([4.0] * 4, [1, 2, 4, 8], [0.25] * 4), ([0.0, 1.5], [2, 5], [0.4, 0.6])]
    for trial in range(12):
        n = int(rng.integers(2, 25))
        a = np.triu(rng.random((n, n)) * (rng.random((n, n)) < 0.3) * rng.choice([0.25, 3.0, 1.0]), 1)
        a = a + a.T
        rp, cl, wv = _csr_of_dense(a)
        g = O.import_csr(rp, cl, wv, lib=lib)
        dd = D.dense_degree(a)
        assert np.array_equal(g.deg.view(np.uint64), dd.view(np.uint64))
        x = rng.normal(size=(n, 2)) * 30 + 500
        for sig, k, al in cases:
            ref = D.spectral_filter(a, x, sig, k, al)
            err = np.abs(g.filter(x, sig, k, al) - ref).max() / np.abs(ref).max()
            assert err <= 1e-12, (trial, err)
        g.close()
    # the CSR of a built netlist, imported, is the same graph bit for bit
    net_ptr, pin_cell = _random_netlist(rng, 40, 60, 6)
    gb = O.build_graph(40, net_ptr, pin_cell, lib=lib)
    gi = O.import_csr(gb.row_ptr, gb.col, gb.w, lib=lib)
    assert np.array_equal(gi.deg.view(np.uint64), gb.deg.view(np.uint64))
    for s in (0.0, 2.0):
        for u, v in zip(gb.normalise(s), gi.normalise(s)):
            assert np.array_equal(u.view(np.uint64), v.view(np.uint64))
    x = rng.normal(size=(40, 2)) * 20 + 500
    assert np.array_equal(gb.filter(x, [4.0, 2.0], [3, 2], [0.5, 0.5]),
                          gi.filter(x, [4.0, 2.0], [3, 2], [0.5, 0.5]))
    gb.close()
    gi.close()
    bad = [([0, 1, 2], [1, 1], [1.0, 1.0]),          # row 1 holds its own diagonal
           ([0, 2, 2], [1, 1], [1.0, 1.0]),          # repeated column
           ([0, 2, 2], [1, 0], [1.0, 1.0]),          # diagonal, descending
           ([0, 1, 2], [2, 0], [1.0, 1.0]),          # column out of range
           ([0, 1, 2], [1, 0], [-1.0, 1.0]),         # negative weight
           ([0, 1, 2], [1, 0], [np.nan, 1.0]),       # NaN weight
           ([1, 1, 2], [1, 0], [1.0, 1.0]),          # row_ptr[0] != 0
           ([0, 2, 1], [1, 0], [1.0, 1.0])]          # decreasing row_ptr
    for rp, cl, wv in bad:
        try:
            O.import_csr(np.array(rp), np.array(cl), np.array(wv), lib=lib)
        except O.OracleError:
            continue
        raise AssertionError(f"malformed CSR accepted: {rp} {cl} {wv}")


ALL_PINS = [pin_golden_two_cell, pin_clique_closed_form, pin_hand_built,
            pin_brute_force_structure, pin_spectral, pin_theorem1_fixed_point,
            pin_spectrum, pin_isolated_and_fixed, pin_star_schur, pin_star_start_value,
            pin_star_order_golden, pin_star_order_relabels, pin_generated_invariants, pin_invalid_input, pin_evaluate_hand,
            pin_evaluate_dense, pin_exact_filter, pin_bin_density, pin_import_csr]

# the eigenvector-placement oracle is numpy (oracle/eigen.py); its pins take
# the module to check, so mutants of it can be run through them
EIGEN_PINS = [pin_eigen_path, pin_eigen_complete, pin_eigen_components]
