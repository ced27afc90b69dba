"""Eigenvector placement, the comparison baseline of Section 3.3.1 (test
infrastructure only).

The classic eigenvector placer takes the eigenvectors of the second and third
smallest eigenvalues of the graph Laplacian L = D - A (Section 2.1, where the
GFT basis U diagonalises L) as the cells' x and y, i.e. the ideal low-pass
filter of eq. ideal_filter.  The graph is the clique net model (Section 3.2,
the paragraph after Algorithm 1) with weight w(M) per net.

A netlist graph is usually disconnected (isolated cells, small groups), and
every component adds a zero eigenvalue, so "second smallest" is read on the
largest connected component (most cells; ties go to the component with the
smallest cell index): its zero eigenvalue belongs to the constant vector, and
u_2, u_3 are the next two.  Cells outside that component get 0.

Plain definitions, evaluated densely: components by union-find over the nets,
the Laplacian of the component accumulated net by net, and a dense symmetric
eigendecomposition (numpy.linalg.eigh) as the one library step.  Only for
small graphs.
"""
from __future__ import annotations

from typing import Dict, List

import numpy as np


def _net_cells(net_ptr, pin_cell, e) -> List[int]:
    return sorted(set(int(c) for c in pin_cell[int(net_ptr[e]):int(net_ptr[e + 1])]))


def _weight(m: int, weight_model: int) -> float:
    return 2.0 / m if weight_model == 1 else 1.0 / (m - 1)


def components(num_cells: int, net_ptr, pin_cell) -> np.ndarray:
    """Component label of every cell: the smallest cell index of its
    connected component (cells are connected when they share a net of at
    least two distinct cells)."""
    parent = list(range(num_cells))

    def find(a: int) -> int:
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for e in range(len(net_ptr) - 1):
        cells = _net_cells(net_ptr, pin_cell, e)
        for c in cells[1:]:
            ra, rb = find(cells[0]), find(c)
            if ra != rb:
                parent[max(ra, rb)] = min(ra, rb)
    return np.array([find(i) for i in range(num_cells)], dtype=np.int64)


def row_labels(num_cells: int, net_ptr, pin_cell, star_threshold: int) -> np.ndarray:
    """Labels of all graph rows: cells, then one virtual row per star net
    (nets of more than star_threshold distinct cells, in net order), which
    takes the label of its cells."""
    lab = components(num_cells, net_ptr, pin_cell)
    extra = []
    for e in range(len(net_ptr) - 1):
        cells = _net_cells(net_ptr, pin_cell, e)
        if len(cells) >= 2 and star_threshold > 0 and len(cells) > star_threshold:
            extra.append(lab[cells[0]])
    return np.concatenate([lab, np.array(extra, dtype=np.int64)])


def giant_component(labels: np.ndarray) -> int:
    """Label of the largest component (most cells; ties: smallest label)."""
    counts: Dict[int, int] = {}
    for l in labels.tolist():
        counts[l] = counts.get(l, 0) + 1
    return min(counts, key=lambda l: (-counts[l], l))


def laplacian(num_cells: int, net_ptr, pin_cell, cells: List[int],
              weight_model: int = 0) -> np.ndarray:
    """Dense L = D - A of the clique model restricted to `cells` (sorted),
    accumulated one net at a time."""
    pos = {c: i for i, c in enumerate(cells)}
    n = len(cells)
    lap = np.zeros((n, n), dtype=np.float64)
    for e in range(len(net_ptr) - 1):
        cs = _net_cells(net_ptr, pin_cell, e)
        m = len(cs)
        if m < 2 or cs[0] not in pos:
            continue
        w = _weight(m, weight_model)
        for a in cs:
            for b in cs:
                if a != b:
                    lap[pos[a], pos[b]] -= w
                    lap[pos[a], pos[a]] += w
    return lap


def eigen_placement(num_cells: int, net_ptr, pin_cell, weight_model: int = 0):
    """(values[2], vectors N x 2, labels, giant label): lambda_2, lambda_3 of
    the giant component's Laplacian and their unit eigenvectors (zero outside
    the component; each vector's largest-magnitude entry made positive)."""
    labels = components(num_cells, net_ptr, pin_cell)
    g = giant_component(labels)
    cells = [i for i in range(num_cells) if labels[i] == g]
    lap = laplacian(num_cells, net_ptr, pin_cell, cells, weight_model)
    lam, vec = np.linalg.eigh(lap)
    out = np.zeros((num_cells, 2), dtype=np.float64)
    for q in range(2):
        v = vec[:, 1 + q]
        if v[int(np.argmax(np.abs(v)))] < 0:
            v = -v
        out[cells, q] = v
    return lam[1:3].copy(), out, labels, g, lam
