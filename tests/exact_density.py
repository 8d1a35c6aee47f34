"""Exact maximum density rho* = max over nonempty S of |E(S)| / |S| (test infrastructure).

Independent of the oracle: it shares no code with it and is itself checked
against exhaustive enumeration and closed forms (test_oracle_exact.py).

Goldberg's min-cut construction decides whether some S has |E(S)| - g|S| > 0
for a rational g = a/b.  With capacities scaled by b to stay integral:
    s -> v : b * D                    (D >= max degree keeps every capacity >= 0)
    v -> t : b * D + 2a - b * deg(v)
    u -> v : b  for every adjacency entry (both directions of each edge)
a cut with source side {s} + S costs b*D*n + 2(a|S| - b|E(S)|), so the
minimum cut is below b*D*n exactly when such an S exists, and the source side
of a minimum cut maximises b|E(S)| - a|S|.  Dinkelbach's iteration starts at
the whole graph's density and replaces g by the density of the maximiser
until the maximum is 0; g then equals rho*.  It ends after finitely many
steps because g strictly increases over the finitely many values
|E(S)| / |S|.  scipy's Dinic max-flow is the max-flow step.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np
from scipy.sparse import csr_array
from scipy.sparse.csgraph import breadth_first_order, maximum_flow


def _induced_edges(offsets, adj, mask) -> int:
    src = np.repeat(np.arange(len(offsets) - 1), np.diff(offsets))
    return int(np.count_nonzero(mask[src] & mask[adj])) // 2


def _best_subset(offsets, adj, a: int, b: int):
    """Source side S (bool mask) of a minimum cut for g = a/b; it maximises b|E(S)| - a|S| (empty if 0 is the max)."""
    n = len(offsets) - 1
    deg = np.diff(offsets).astype(np.int64)
    D = int(deg.max()) if n else 0
    s, t = n, n + 1
    src = np.repeat(np.arange(n, dtype=np.int64), deg)
    rows = np.concatenate([np.full(n, s), np.arange(n), src])
    cols = np.concatenate([np.arange(n), np.full(n, t), np.asarray(adj, dtype=np.int64)])
    caps = np.concatenate([np.full(n, b * D), b * D + 2 * a - b * deg, np.full(len(adj), b)]).astype(np.int64)
    assert caps.min() >= 0 and int(caps.sum()) < 2**31 - 1, "capacities must fit scipy's int32 flows"
    cap = csr_array((caps.astype(np.int32), (rows, cols)), shape=(n + 2, n + 2))
    res = maximum_flow(cap, s, t, method="dinic")
    # residual arcs: capacity - flow > 0 (a reverse arc's capacity is 0, its flow negative)
    resid = (cap - res.flow).tocsr()
    resid.data = np.where(resid.data > 0, 1, 0).astype(np.int32)
    resid.eliminate_zeros()
    reach = breadth_first_order(resid, s, directed=True, return_predecessors=False)
    mask = np.zeros(n + 2, dtype=bool)
    mask[reach] = True
    assert not mask[t], "a maximum flow leaves the sink unreachable"
    return mask[:n]


def densest_exact(offsets, adj):
    """(rho* as a Fraction, a densest vertex set as a bool mask).  rho* = 0 for a graph without edges."""
    offsets = np.asarray(offsets, dtype=np.int64)
    adj = np.asarray(adj, dtype=np.int64)
    n = len(offsets) - 1
    m = len(adj) // 2
    mask = np.ones(n, dtype=bool)
    if m == 0:
        return Fraction(0), mask
    g = Fraction(m, n)
    while True:
        S = _best_subset(offsets, adj, g.numerator, g.denominator)
        k = int(S.sum())
        if k == 0:
            return g, mask
        e = _induced_edges(offsets, adj, S)
        h = Fraction(e, k)
        if h <= g:  # the maximiser only ties g: 0 is the maximum
            return g, mask
        g, mask = h, S
