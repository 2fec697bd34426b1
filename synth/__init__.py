"""Seeded synthetic graph generators shared by the tests, the bench and the oracle checks.

This module only builds input graphs (CSR adjacency) and random point sets.
It holds none of the layout method's arithmetic: no distances sets, no
coarsening, no layout update. Every generator is deterministic in its seed.
"""
from .graphs import (  # noqa: F401
    Graph,
    csr_from_edges,
    largest_component,
    relabel,
    grid,
    path,
    cycle,
    star,
    complete_binary_tree,
    two_triangles,
    random_tree,
    rgg,
    rmat,
    delaunay,
    config_graph,
)
from .dynamic import churn_snapshot  # noqa: F401
from .batch import batch_graphs, concat  # noqa: F401
