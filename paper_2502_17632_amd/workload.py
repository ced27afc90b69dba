"""Seeded synthetic netlists and placement signals.

This module only draws inputs: it holds none of the filter's arithmetic and is
shared by the device path, the CPU oracle, the tests and the benchmark.

The paper evaluates on the ISPD2014 contest designs (30k-155k cells, about one
net per cell; Section 4, Table 1).  They are not available here, so these
generators stand in for them with the same kind of structure: mostly 2-4 pin
nets with a heavy tail, index-local connectivity, fixed IO cells on the die
boundary and movable cells started at the die centre with Gaussian noise
(Section 3.2.2, Algorithm 1 step 1).

Reading of the recipe (all stated here so a reader can regenerate it):

* pin count per net: ``M = 2 + (Geom(p) - 1)`` or ``M = 2 + (Zipf(s) - 1)``,
  then ``min(M, cap)``; numpy's geometric and zipf start at 1, so the extra
  pin count starts at 0 and 2-pin nets are the most common kind.
* pins of one net are distinct cells.  ``uniform``: drawn uniformly over all
  cells.  ``local``: each net draws an anchor ``a``; each pin is, with
  probability 0.9, ``(a + U{-512..512}) mod N`` and otherwise uniform; pins that
  repeat a cell already on the net are drawn again with the same rule.
* cell ``i`` is fixed iff ``(i + 1) % step == 0`` and ``(i + 1) // step <=
  num_fixed`` with ``step = N // num_fixed``: IO cells are spread through the
  index range instead of sitting at one end of the locality window.
* fixed cells sit uniformly on the perimeter of the ``[0, die]^2`` die
  (arc length ``t ~ U[0, 4 die)``); movable cells at ``(die/2, die/2) +
  N(0, noise^2)`` per coordinate.
* every draw comes from one ``numpy.random.default_rng(seed)`` (PCG64) stream,
  in the order the code below makes them.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
from typing import List, Optional, Sequence

import numpy as np

DIE = 1000.0


@dataclasses.dataclass
class Netlist:
    """A hypergraph netlist in CSR-of-pins form.

    ``net_ptr[e] .. net_ptr[e+1]`` index the pins of net ``e`` in ``pin_cell``.
    ``fixed`` marks the fixed (IO) cells.
    """

    num_cells: int
    net_ptr: np.ndarray  # int64[E+1]
    pin_cell: np.ndarray  # int32[P]
    fixed: np.ndarray  # uint8[N]
    name: str = ""

    @property
    def num_nets(self) -> int:
        return int(self.net_ptr.shape[0] - 1)

    @property
    def num_pins(self) -> int:
        return int(self.pin_cell.shape[0])

    def digest(self) -> str:
        h = hashlib.sha256()
        h.update(np.int64(self.num_cells).tobytes())
        h.update(np.ascontiguousarray(self.net_ptr, dtype=np.int64).tobytes())
        h.update(np.ascontiguousarray(self.pin_cell, dtype=np.int32).tobytes())
        h.update(np.ascontiguousarray(self.fixed, dtype=np.uint8).tobytes())
        return h.hexdigest()


def _pin_counts(rng, num_nets: int, dist: str, param: float, cap: int) -> np.ndarray:
    if dist == "geometric":
        extra = rng.geometric(param, size=num_nets) - 1
    elif dist == "zipf":
        extra = rng.zipf(param, size=num_nets) - 1
    else:
        raise ValueError(f"unknown pin-count distribution {dist!r}")
    m = np.minimum(2 + extra, cap).astype(np.int64)
    return m


def _draw_pins(rng, n_cells: int, owner: np.ndarray, anchor: Optional[np.ndarray],
               window: int, p_local: float) -> np.ndarray:
    """One candidate cell per pin slot; ``owner`` is the net of each slot."""
    k = owner.shape[0]
    if anchor is None:
        return rng.integers(0, n_cells, size=k, dtype=np.int64)
    local = rng.random(k) < p_local
    off = rng.integers(-window, window + 1, size=k, dtype=np.int64)
    uni = rng.integers(0, n_cells, size=k, dtype=np.int64)
    near = (anchor[owner] + off) % n_cells
    return np.where(local, near, uni)


def make_netlist(num_movable: int, num_fixed: int, num_nets: int, *,
                 dist: str = "zipf", param: float = 2.2, cap: int = 1000,
                 locality: bool = True, window: int = 512, p_local: float = 0.9,
                 seed: int = 0, name: str = "") -> Netlist:
    """Draw a netlist with the recipe in the module docstring."""
    n = int(num_movable) + int(num_fixed)
    if n <= 0:
        raise ValueError("a netlist needs at least one cell")
    rng = np.random.default_rng(seed)
    m = _pin_counts(rng, num_nets, dist, param, cap)
    m = np.minimum(m, n)  # a net cannot hold more distinct cells than exist
    net_ptr = np.zeros(num_nets + 1, dtype=np.int64)
    np.cumsum(m, out=net_ptr[1:])
    p = int(net_ptr[-1])
    owner = np.repeat(np.arange(num_nets, dtype=np.int64), m)
    anchor = rng.integers(0, n, size=num_nets, dtype=np.int64) if locality else None
    cells = _draw_pins(rng, n, owner, anchor, window, p_local)
    # Redraw pins that repeat a cell already on their net until every net's
    # cells are distinct.  The first occurrence (in slot order) is kept.
    # After the first sweep only the slots of nets that still held a
    # repeated cell are examined again.
    active = np.arange(p, dtype=np.int64)
    for _ in range(100_000):
        own = owner[active]
        key = own * n + cells[active]
        order = np.argsort(key, kind="stable")
        sk = key[order]
        dup_sorted = np.zeros(active.shape[0], dtype=bool)
        if active.shape[0] > 1:
            dup_sorted[1:] = sk[1:] == sk[:-1]
        if not dup_sorted.any():
            break
        dup = active[order[dup_sorted]]
        cells[dup] = _draw_pins(rng, n, owner[dup], anchor, window, p_local)
        bad_nets = np.unique(owner[dup])
        active = active[np.isin(own, bad_nets)]
    else:  # pragma: no cover - the caps above make this unreachable
        raise RuntimeError("pin redraw did not converge")
    fixed = np.zeros(n, dtype=np.uint8)
    if num_fixed > 0:
        step = n // num_fixed
        idx = np.arange(step - 1, n, step)[:num_fixed]
        fixed[idx] = 1
    return Netlist(n, net_ptr, cells.astype(np.int32), fixed, name)


def make_signal(netlist: Netlist, noise: Sequence[float] = (10.0,), *, seed: int = 0,
                die: float = DIE) -> np.ndarray:
    """Initial locations, float64 ``[N, 2*len(noise)]`` row-major.

    Columns ``2q, 2q+1`` hold x, y of placement ``q``; fixed cells are at the
    same boundary position in every placement, movable cells at the die centre
    plus ``N(0, noise[q]^2)``.
    """
    rng = np.random.default_rng(seed + 7_919)
    n = netlist.num_cells
    fixed = netlist.fixed.astype(bool)
    nf = int(fixed.sum())
    t = rng.uniform(0.0, 4.0 * die, size=nf)
    side = np.minimum((t // die).astype(np.int64), 3)
    u = t - side * die
    fx = np.choose(side, [u, np.full(nf, die), die - u, np.zeros(nf)])
    fy = np.choose(side, [np.zeros(nf), u, np.full(nf, die), die - u])
    out = np.empty((n, 2 * len(noise)), dtype=np.float64)
    for q, s in enumerate(noise):
        g = rng.normal(0.0, float(s), size=(n, 2)) + die / 2.0
        g[fixed, 0] = fx
        g[fixed, 1] = fy
        out[:, 2 * q:2 * q + 2] = g
    return out


# --------------------------------------------------------------------------
# The five workloads.
# --------------------------------------------------------------------------

@dataclasses.dataclass
class FilterSpec:
    """(sigma, order, alpha) terms of a multi-order filter."""

    sigma: List[float]
    order: List[int]
    alpha: List[float]


def equal_terms(orders: Sequence[int], sigma: float = 4.0) -> FilterSpec:
    """One self-loop weight for all orders, equal combine weights."""
    k = len(orders)
    return FilterSpec([float(sigma)] * k, [int(o) for o in orders], [1.0 / k] * k)


# The paper's filter: alpha_0 A_2^2 + alpha_1 A_4^2 + alpha_2 A_4^4 with
# alpha = (0.1, 0.7, 0.2) (Section 3.2.1, eq. proposed_filter and
# A_formulation; coefficients from Section 4.1).
PAPER_DEFAULT = FilterSpec([2.0, 4.0, 4.0], [2, 2, 4], [0.1, 0.7, 0.2])


def tiny(seed: int = 0) -> Netlist:
    """2,000 movable + 200 fixed cells, 2,500 nets, 2 + Geom(0.5) pins <= 8,
    uniform pins."""
    return make_netlist(2000, 200, 2500, dist="geometric", param=0.5, cap=8,
                        locality=False, seed=seed, name="tiny")


def medium(seed: int = 0) -> Netlist:
    """200k movable + 2k fixed, 220k nets, 2 + Zipf(2.2) pins <= 1000,
    90% of pins within +-512 of a per-net anchor."""
    return make_netlist(200_000, 2_000, 220_000, seed=seed, name="medium")


def large(seed: int = 0) -> Netlist:
    """2M movable + 20k fixed, 2.1M nets, same generator as ``medium``."""
    return make_netlist(2_000_000, 20_000, 2_100_000, seed=seed, name="large")


def sized(num_movable: int, seed: int) -> Netlist:
    """The ``medium`` generator at another size: fixed = round(mov/100),
    nets = round(1.1 mov)."""
    nf = max(1, int(round(num_movable / 100.0)))
    ne = int(round(1.1 * num_movable))
    return make_netlist(num_movable, nf, ne, seed=seed, name=f"sized{num_movable}")


def batch_sizes(count: int = 64, lo: float = 10_000, hi: float = 300_000,
                seed: int = 1000) -> List[int]:
    """Log-uniform movable-cell counts for the batched workload."""
    rng = np.random.default_rng(seed)
    return [int(round(v)) for v in np.exp(rng.uniform(math.log(lo), math.log(hi), size=count))]


BATCH_NOISE = (5.0, 10.0, 20.0, 40.0)


def poisson_arrivals(count: int, rate_per_s: float, seed: int = 4242) -> np.ndarray:
    """Arrival times (s) of a Poisson stream."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=count))


def serving_sizes(count: int, lo: float = 5_000, hi: float = 2_000_000,
                  seed: int = 4243) -> List[int]:
    rng = np.random.default_rng(seed)
    return [int(round(v)) for v in np.exp(rng.uniform(math.log(lo), math.log(hi), size=count))]
