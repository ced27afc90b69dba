"""Dense brute-force checkers for tiny graphs (test infrastructure only).

These pin the C oracle to the paper's definitions by a different route:

* ``dense_adjacency`` accumulates the adjacency matrix straight from the
  clique net model (Section 3.2, after Algorithm 1) with Python loops, one net
  at a time in ascending net id, into a dense R x R array.
* ``spectral_filter`` applies the filter in the spectral domain
  (Section 2.1, eq. filter): it eigendecomposes the normalised Laplacian of the
  self-loop-augmented graph, L~_sigma = I - A~_sigma (Theorem 1 relates A~ to
  the filter h(lambda) = 1 - lambda, and Section 3.2.1 the k-th power to
  (1 - lambda)^k), and forms U diag(h(lambda)) U^T x with
  h(lambda) = sum_t alpha_t (1 - lambda)^{k_t} for each self-loop weight.

Nothing here calls the C oracle.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np


def net_cells(net_ptr, pin_cell, e) -> List[int]:
    return sorted(set(int(c) for c in pin_cell[int(net_ptr[e]):int(net_ptr[e + 1])]))


def dense_adjacency(num_cells: int, net_ptr, pin_cell, *, weight_model: int = 0,
                    star_threshold: int = 0) -> Tuple[np.ndarray, List[int]]:
    """Dense A (R x R, float64) and the net of every virtual row."""
    nets = [net_cells(net_ptr, pin_cell, e) for e in range(len(net_ptr) - 1)]
    star = [e for e, c in enumerate(nets)
            if len(c) >= 2 and star_threshold > 0 and len(c) > star_threshold]
    r = num_cells + len(star)
    a = np.zeros((r, r), dtype=np.float64)
    vid = {e: num_cells + i for i, e in enumerate(star)}
    for e, cells in enumerate(nets):
        m = len(cells)
        if m < 2:
            continue
        if e in vid:
            # A star: every cell of the net joined to one new node by M*w(M).
            g = 2.0 if weight_model == 1 else float(m) / float(m - 1)
            v = vid[e]
            for c in cells:
                a[c, v] += g
                a[v, c] += g
        else:
            w = 2.0 / float(m) if weight_model == 1 else 1.0 / float(m - 1)
            for i in cells:
                for j in cells:
                    if i != j:
                        a[i, j] += w
    return a, star


def dense_degree(a: np.ndarray) -> np.ndarray:
    """d_i = sum_j w_ij, summed left to right over ascending j."""
    d = np.zeros(a.shape[0], dtype=np.float64)
    for i in range(a.shape[0]):
        s = 0.0
        for j in range(a.shape[1]):
            if a[i, j] != 0.0:
                s = s + float(a[i, j])
        d[i] = s
    return d


def augmented_normalised(a: np.ndarray, sigma: float) -> np.ndarray:
    """A~_sigma = (D + sigma I)^-1/2 (A + sigma I) (D + sigma I)^-1/2; a row
    with d_i + sigma = 0 is all zero."""
    d = a.sum(axis=1)
    t = d + sigma
    s = np.where(t > 0, 1.0 / np.sqrt(np.where(t > 0, t, 1.0)), 0.0)
    return (s[:, None] * (a + sigma * np.eye(a.shape[0]))) * s[None, :]


def extend_signal(x: np.ndarray, net_ptr, pin_cell, star: Sequence[int]) -> np.ndarray:
    """Append one row per virtual node: the mean of its net's cells."""
    x = np.asarray(x, dtype=np.float64)
    rows = [x]
    for e in star:
        cells = net_cells(net_ptr, pin_cell, e)
        rows.append(x[cells].mean(axis=0, keepdims=True))
    return np.concatenate(rows, axis=0)


def spectral_filter(a: np.ndarray, x_ext: np.ndarray, sigma: Sequence[float],
                    order: Sequence[int], alpha: Sequence[float]) -> np.ndarray:
    """sum over self-loop weights of U h(Lambda) U^T x (eq. filter)."""
    x_ext = np.asarray(x_ext, dtype=np.float64)
    y = np.zeros_like(x_ext)
    for s in sorted(set(float(v) for v in sigma)):
        lap = np.eye(a.shape[0]) - augmented_normalised(a, s)
        lam, u = np.linalg.eigh(lap)
        h = np.zeros_like(lam)
        for st, k, al in zip(sigma, order, alpha):
            if float(st) == s:
                h += float(al) * (1.0 - lam) ** int(k)
        y += u @ (h[:, None] * (u.T @ x_ext))
    return y
