"""Seeded synthetic graph generators shared by the tests, the oracle runs and the bench.

This module holds no arithmetic of the eigensolver: it only builds simple, connected,
undirected graphs (optionally weighted) in CSR form and seeded start vectors.
"""
from .generators import (  # noqa: F401
    CSRGraph,
    path_graph,
    cycle_graph,
    grid2d,
    grid3d,
    complete_graph,
    star_graph,
    hypercube,
    spider,
    whiskered_clique,
    random_connected,
    rmat,
    chung_lu,
    start_block,
    config_graph,
)
