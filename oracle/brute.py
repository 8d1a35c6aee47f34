"""Exhaustive checkers for tiny graphs (TEST INFRASTRUCTURE ONLY).

These compute quantities with a plain definition: the maximum density over
all non-empty vertex subsets (the densest-subgraph objective of Section 2),
and the number of induced edges of a given vertex set.  They do not use the
peeling algorithm, so they can pin it.
"""
from __future__ import annotations

import numpy as np


def edge_list(offsets, adj):
    """Undirected edges (u < v) of a symmetric CSR."""
    off = np.asarray(offsets, dtype=np.int64)
    a = np.asarray(adj, dtype=np.int64)
    n = len(off) - 1
    src = np.repeat(np.arange(n), np.diff(off))
    keep = src < a
    return np.stack([src[keep], a[keep]], axis=1)


def induced_edges(offsets, adj, mask) -> int:
    """|E(S)| for S = {v : mask[v]}, counted from the CSR."""
    e = edge_list(offsets, adj)
    m = np.asarray(mask, dtype=bool)
    if len(e) == 0:
        return 0
    return int(np.sum(m[e[:, 0]] & m[e[:, 1]]))


def densest_brute(offsets, adj):
    """Exact maximum density as an (edges, vertices) pair, by enumerating all 2^n - 1 subsets (n <= 20)."""
    n = len(offsets) - 1
    if n > 20:
        raise ValueError("brute force is limited to n <= 20")
    e = edge_list(offsets, adj)
    masks = np.arange(1, 1 << n, dtype=np.int64)
    sizes = np.zeros(len(masks), dtype=np.int64)
    for v in range(n):
        sizes += (masks >> v) & 1
    edges = np.zeros(len(masks), dtype=np.int64)
    for u, v in e:
        edges += ((masks >> u) & 1) & ((masks >> v) & 1)
    # maximise edges/sizes exactly: compare by cross-multiplication against the running best
    best_e, best_v = 0, 1
    # candidates: for each size keep the max edge count, then compare rationals exactly
    for s in range(1, n + 1):
        sel = sizes == s
        if not np.any(sel):
            continue
        es = int(edges[sel].max())
        if es * best_v > best_e * s:
            best_e, best_v = es, s
    return best_e, best_v


def core_numbers_brute(offsets, adj):
    """Core numbers by the definition: core(v) = max k such that v is in the k-core.

    The k-core is found by repeatedly deleting any vertex of degree < k
    (Section 2); done for every k from 0 up.
    """
    off = np.asarray(offsets)
    a = np.asarray(adj)
    n = len(off) - 1
    core = np.zeros(n, dtype=np.int64)
    k = 0
    while True:
        alive = np.ones(n, dtype=bool)
        changed = True
        while changed:
            changed = False
            for v in range(n):
                if alive[v] and sum(alive[a[off[v]:off[v + 1]]]) < k:
                    alive[v] = False
                    changed = True
        if not alive.any():
            break
        core[alive] = k
        k += 1
    return core
