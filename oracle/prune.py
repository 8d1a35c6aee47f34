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

Approximate k-core pruning (Definition "c-Approx k-Core Decomposition", Corollary apxkmax, and the two
approximate-pruning frameworks of Section 4, "Implementations"):
  * The paper cites an outside algorithm for the decomposition and does not describe it.  The reading here is
    round-synchronous peeling with a geometric, monotone degree bound: with c = c_num / c_den > 1, round r takes
    the current minimum degree mn_r among the alive vertices, sets D_r = max(D_{r-1}, floor(c * mn_r)) and peels
    every alive vertex of degree at most D_r (degrees at the start of the round; the decrements of a round apply
    after it).  The approximate core number of a vertex is the bound D of the round that peels it.
  * It is a c-approximate decomposition, in the stronger one-sided form core(v) <= khat(v) <= c * core(v):
    - the first vertex u of the core(v)-core to be peeled has degree >= core(v) at its round, and it is peeled
      there, so core(v) <= D at that round <= D at v's round;
    - D at v's round is floor(c * mn_s) for some round s no later than v's; every vertex alive at round s has
      degree >= mn_s among the alive vertices, so all of them, v included, have core number >= mn_s.
    With c = 1 it is exact bucketing, and khat equals the core numbers.
  * First cut (Corollary apxkmax): L = ceil(khat_max / (2c)), computed exactly as ceil(khat_max * c_den /
    (2 c_num)); G <- {v : khat(v) >= L}.  It keeps every densest subgraph: rho* >= k_max / 2 >= khat_max / (2c),
    and each vertex u of a densest subgraph has khat(u) >= core(u) >= ceil(rho*).
  * prune = "apx" (PaRApxSorting++: approximate pruning only): the re-cuts of Algorithm 1 use khat at level
    ceil(L), which keeps every densest subgraph for the same reason (khat >= core).
  * prune = "apx_exact" (PaRApxGreedy++: approximate, then exact pruning): after the approximate cut, exact core
    numbers are computed on the cut graph; L <- max(L, ceil(k_max / 2)) and G <- that L-core; the re-cuts use these
    exact numbers.  For every level >= the approximate L the cut graph has the same k-cores as the input (each such
    k-core lies inside it), so every refined graph is the one exact pruning refines, and the outputs other than the
    decomposition itself equal those of prune = "exact".
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
    apx_core: np.ndarray | None = None  # approximate core numbers (prune = "apx" / "apx_exact"), input ids
    apx_kmax: int = 0
    apx_level: int = 0  # the first cut's level ceil(khat_max / (2c))
    apx_size: tuple | None = None  # (n, m) of the approximate cut


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


def approx_coreness(offsets, adj, c=(3, 2)):
    """c-approximate core numbers by round-synchronous peeling with the bound D_r = max(D_{r-1}, floor(c * mn_r))
    (the reading in the module notes): (khat int32[n], khat_max).  c = (c_num, c_den) with c_num >= c_den >= 1."""
    c_num, c_den = int(c[0]), int(c[1])
    if c_den < 1 or c_num < c_den:
        raise ValueError("c must be a rational >= 1")
    offsets = np.asarray(offsets, dtype=np.int64)
    adj = np.asarray(adj, dtype=np.int64)
    n = len(offsets) - 1
    deg = np.diff(offsets)
    alive = np.ones(n, dtype=bool)
    khat = np.zeros(n, dtype=np.int64)
    D = 0
    while alive.any():
        mn = int(deg[alive].min())
        D = max(D, (c_num * mn) // c_den)
        frontier = np.flatnonzero(alive & (deg <= D))
        khat[frontier] = D
        alive[frontier] = False
        # the round's decrements, applied after it: every edge from a peeled vertex to a survivor
        lens = offsets[frontier + 1] - offsets[frontier]
        total = int(lens.sum())
        if total:
            # adjacency positions of the frontier's rows, row after row
            idx = np.repeat(offsets[frontier] - (np.cumsum(lens) - lens), lens) + np.arange(total)
            nbr = adj[idx]
            nbr = nbr[alive[nbr]]
            deg -= np.bincount(nbr, minlength=n)
    return khat.astype(np.int32), int(khat.max()) if n else 0


def par_run(offsets, adj, T: int, variant: str, eps=(0, 1), lib=None, prune: str = "exact", c=(3, 2)) -> ParResult:
    """Algorithm 1 with exact ("exact"), approximate ("apx") or approximate-then-exact ("apx_exact") pruning."""
    offsets = np.asarray(offsets, dtype=np.int32)
    adj = np.asarray(adj, dtype=np.int32)
    n = len(offsets) - 1
    if prune == "exact":
        core, kmax = coreness(offsets, adj, lib=lib)
        level = ceil_div(kmax, 2)
        o, a, ids = get_core(offsets, adj, core >= level)
        apx = None
    elif prune in ("apx", "apx_exact"):
        khat, khat_max = approx_coreness(offsets, adj, c)
        apx_level = ceil_div(khat_max * int(c[1]), 2 * int(c[0]))
        o, a, ids = get_core(offsets, adj, khat >= apx_level)
        apx = (khat, khat_max, apx_level, (len(ids), int(o[-1]) // 2))
        if prune == "apx":
            core, kmax, level = khat, khat_max, apx_level
        else:
            core1, kmax = coreness(o, a, lib=lib)
            core = np.zeros(n, dtype=np.int32)
            core[ids] = core1
            level = max(apx_level, ceil_div(kmax, 2))
            o, a, sub = get_core(o, a, core1 >= level)
            ids = ids[sub]
    else:
        raise ValueError(f"unknown pruning {prune!r}")
    loads = np.zeros(len(ids), dtype=np.int64)
    best = (int(o[-1]) // 2, len(ids), 0)
    mask = np.zeros(n, dtype=bool)
    mask[ids] = True
    res = ParResult(core=core, kmax=kmax, level=level, best=best, best_mask=mask)
    if apx is not None:
        res.apx_core, res.apx_kmax, res.apx_level, res.apx_size = apx
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
