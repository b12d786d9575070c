"""Seeded synthetic signed bipartite graphs (inputs only, no counting arithmetic).

This package is the one piece of code shared by the CPU oracle side and the HIP
side: it draws edge lists and nothing else.
"""
from .graphs import (  # noqa: F401
    SignedBipartiteGraph,
    uniform_graph,
    voting_graph,
    chung_lu_graph,
    chung_lu_graph_fast,
    serving_large_params,
    random_graph,
    complete_graph,
    batch_graph_params,
    batch_graph,
    WORKLOADS,
    workload,
)
