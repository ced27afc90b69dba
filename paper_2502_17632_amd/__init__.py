"""GiFt graph-filter placement on AMD MI355X (gfx950).

``build_graph`` turns a netlist into a resident normalised cell graph and
``filter_placement`` applies the multi-order low-pass filter of the paper
"The Power of Graph Signal Processing for Chip Placement Acceleration"
(ICCAD'24, Section 3.2.1, eq. proposed_filter).  Both run in the HIP library
``libgift.so``; importing this package does not require a GPU, calling it
does.
"""
from .api import (Batch, Graph, Server, bin_density, build_graph,  # noqa: F401
                  density_overflow, eigen_placement, evaluate_placement,
                  filter_exact, filter_placement, import_csr, make_terms, profile_collect,
                  profile_enable, profile_pause, set_allocator, TorchAllocator, use_torch_allocator)
from ._lib import GiftError, lib  # noqa: F401
