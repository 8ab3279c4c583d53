"""Seeded synthetic inputs for IMM: graph generators and edge-parameter encodings.

This package is shared by the CPU oracle's tests and by the GPU path's tests and
benchmark. It holds no arithmetic of the IMM method itself: it only builds
graphs (R-MAT, Chung-Lu), lays them out as CSC of in-edges, and encodes the
diffusion parameters as 32-bit integers (IC live-edge thresholds and LT
cumulative in-weight tables).
"""

from .graphs import (  # noqa: F401
    Graph,
    WORKLOADS,
    batch_instances,
    chung_lu_edges,
    ic_uniform_thresholds,
    ic_wc_thresholds,
    lt_cumulative,
    make_graph,
    make_graphs,
    rmat_edges,
    to_csc,
    tiny_graph,
    served_queries,
)
