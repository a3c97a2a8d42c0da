"""Seeded synthetic bipartite graphs.

This module only draws inputs.  It holds none of the decomposition
arithmetic, so both the CPU oracle (test infrastructure) and the HIP path
may take their inputs from it.

Every graph is returned as a U-side CSR: ``row_ptr`` (int64, length n_u+1)
and ``col_idx`` (int32, length m), with the V ids of each row strictly
increasing.  Edge ``e`` is slot ``e`` of ``col_idx``.

Generators
----------
``er(n_u, n_v, m, seed)``
    m distinct (u, v) pairs drawn uniformly from U x V.
``chung_lu(n_u, n_v, m, gamma, cap, seed)``
    Power-law expected degrees on both sides: rank weights
    (i+1)^(-1/(gamma-1)) scaled so that the capped weights sum to m, ids
    shuffled per side, endpoints drawn independently in proportion to the
    weights, duplicates rejected until m distinct edges remain.  Isolated
    vertices are kept.
``complete(a, b)``
    K_{a,b}.
``mixed_graph(gi, m_min, m_max)``
    Graph gi of a family of uneven sizes (half Erdos-Renyi, half Chung-Lu)
    for batched calls.

All randomness comes from numpy's counter-based Philox generator, keyed by
the seed, so a (generator, parameters, seed) triple names one graph.
"""
from .bipartite import (  # noqa: F401
    Graph,
    er,
    chung_lu,
    complete,
    from_edges,
    disjoint_union,
    random_small,
    mixed_graph,
    mixed_graphs,
    mixed_edges,
    config_graph,
    CONFIGS,
)
