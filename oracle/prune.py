"""Pruning-and-Refining framework (Algorithm 1, Section 3) with exact k-core pruning, on the CPU oracle.

TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the benchmark's CPU baseline, never by the
product path.

Algorithm 1 as written, with these readings (they bind the GPU path too):
  * cores, k_max <- Coreness(G) on the input graph; L <- ceil(k_max / 2); G <- getCore(G, cores, L), the subgraph
    induced by {v : core(v) >= L}; S <- G (the pruned graph is the initial answer; its density is (m_1, n_1)).
  * Refine is one Greedy++ iteration of the chosen variant (SEQ, PEEL or SORT) on the current G.  Loads persist
    across iterations for the vertices that stay; a vertex removed by a prune takes its load with it.  S' is the
    iteration's densest suffix (the Algorithm 3 maximum, ties to the smallest index).
  * If rho(S') > rho(S) (strict, exact cross-multiplication): S <- S', L <- max(L, rho(S)) and
    G <- getCore(G, cores, ceil(L)).  The cores are those of the input graph, and since L only grows each prune
    keeps a subset of the current G.  ceil(L) is an exact integer ceiling of the rational e/v.
  * Vertex ids of a pruned graph follow the input order (the induced subgraph keeps relative id order), so every
    lowest-id tie rule resolves as it would on the input ids.
  * Returned: the best (edges, vertices), the iteration that found it (0 = the initial pruned graph), its vertex
    set in input ids, the per-iteration (edges, vertices, index) of S', the size (n_i, m_i) of the graph each
    iteration ran on, k_max and the final core level ceil(L).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import State, coreness, run


@dataclass
class ParResult:
    core: np.ndarray
    kmax: int
    level: int
    best: tuple  # (edges, vertices, iteration)
    best_mask: np.ndarray
    hist: list = field(default_factory=list)  # per iteration (edges, vertices)
    hist_idx: list = field(default_factory=list)
    sizes: list = field(default_factory=list)  # per iteration (n_i, m_i) of the graph refined
    levels: list = field(default_factory=list)  # per iteration: the refined graph is the levels[i]-core
    prunes: int = 0


def get_core(offsets, adj, keep):
    """Subgraph induced by the vertices with keep[v], ids renumbered in input order: (offsets, adj, old_ids)."""
    offsets = np.asarray(offsets, dtype=np.int64)
    adj = np.asarray(adj, dtype=np.int64)
    keep = np.asarray(keep, dtype=bool)
    n = len(offsets) - 1
    old_ids = np.flatnonzero(keep)
    new_id = np.full(n, -1, dtype=np.int64)
    new_id[old_ids] = np.arange(len(old_ids))
    src = np.repeat(np.arange(n), np.diff(offsets))
    sel = keep[src] & keep[adj]
    new_src, new_dst = new_id[src[sel]], new_id[adj[sel]]
    counts = np.bincount(new_src, minlength=len(old_ids))
    new_off = np.zeros(len(old_ids) + 1, dtype=np.int32)
    np.cumsum(counts, out=new_off[1:])
    # the kept entries stay in input order, so rows stay sorted
    return new_off, new_dst.astype(np.int32), old_ids.astype(np.int64)


def ceil_div(a: int, b: int) -> int:
    return -((-a) // b)


def par_run(offsets, adj, T: int, variant: str, eps=(0, 1), lib=None) -> ParResult:
    offsets = np.asarray(offsets, dtype=np.int32)
    adj = np.asarray(adj, dtype=np.int32)
    n = len(offsets) - 1
    core, kmax = coreness(offsets, adj, lib=lib)
    level = ceil_div(kmax, 2)
    o, a, ids = get_core(offsets, adj, core >= level)
    loads = np.zeros(len(ids), dtype=np.int64)
    best = (int(o[-1]) // 2, len(ids), 0)
    mask = np.zeros(n, dtype=bool)
    mask[ids] = True
    res = ParResult(core=core, kmax=kmax, level=level, best=best, best_mask=mask)
    for t in range(1, T + 1):
        st = State.fresh(o)
        st.loads = loads.copy()
        st = run(o, a, 1, variant, eps, state=st, lib=lib)
        e, v = st.hist[-1]
        idx = st.hist_idx[-1]
        res.hist.append((int(e), int(v)))
        res.hist_idx.append(int(idx))
        res.sizes.append((len(ids), int(o[-1]) // 2))
        res.levels.append(res.level)
        loads = st.loads
        be, bv, _ = res.best
        if e * bv > be * v:
            res.best = (int(e), int(v), t)
            mask = np.zeros(n, dtype=bool)
            mask[ids[st.last_pos >= idx]] = True
            res.best_mask = mask
            new_level = max(res.level, ceil_div(int(e), int(v)))
            if new_level > res.level:
                res.level = new_level
                keep = core[ids] >= new_level
                o, a, sub = get_core(o, a, keep)
                ids = ids[sub]
                loads = loads[sub]
                res.prunes += 1
    return res
