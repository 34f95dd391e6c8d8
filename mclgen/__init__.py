"""Seeded synthetic inputs shared by the oracle and the GPU library.

This package builds input graphs only: cluster sizes, edges, weights and
self-loops, emitted as sorted CSC arrays.  It holds none of the clustering
method's arithmetic (no column normalisation, products, pruning or
inflation); both sides of every comparison apply those themselves.
"""
from .planted import (  # noqa: F401
    CSC,
    planted_graph,
    planted_components,
    fit_cap_for_density,
    powerlaw_sizes,
    config0_graph,
    config1_graph,
    config3_graph,
    random_csc,
    random_symmetric_graph,
    clique_union,
    two_triangles,
    stripe_blocks,
)
