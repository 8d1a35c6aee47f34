"""Pins of the oracle's Pruning-and-Refining framework (Algorithm 1) and its Coreness, against things other than
itself: networkx's core numbers and k-cores, brute-force optima and induced-edge recounts on small graphs, the
containment lemma for cores (Section 2.1), the k_max/2 lower bound, convergence to the optimum, and the cases where
pruning removes nothing and the framework reduces to plain Greedy++."""
import networkx as nx
import numpy as np
import pytest

import graphgen
import oracle
from oracle import brute, prune
from pins import _small_graphs


def _nx(o, a):
    n = len(o) - 1
    G = nx.Graph()
    G.add_nodes_from(range(n))
    src = np.repeat(np.arange(n), np.diff(o))
    G.add_edges_from((int(u), int(v)) for u, v in zip(src, a) if u < v)
    return G


def _graphs():
    gs = list(_small_graphs())
    gs.append(graphgen.config1(2))
    gs.append(graphgen.rmat(3, 11, 16 << 11))
    gs.append(graphgen.from_edges(30, [(i, i + 1) for i in range(20)]))  # a path and isolated vertices
    gs.append(graphgen.from_edges(1, []))
    gs.append(graphgen.complete(9))
    return gs


def test_core_numbers_match_networkx():
    """Coreness (Section 2) equals networkx.core_number, and {v: core(v) >= k} is networkx's k-core."""
    for o, a in _graphs():
        core, kmax = oracle.coreness(o, a)
        G = _nx(o, a)
        cn = nx.core_number(G)
        assert [cn[v] for v in range(len(o) - 1)] == core.tolist()
        assert kmax == (max(cn.values()) if cn else 0)
        for k in {0, 1, (kmax + 1) // 2, kmax}:
            assert set(np.flatnonzero(core >= k).tolist()) == set(nx.k_core(G, k).nodes())


def test_get_core_is_the_induced_subgraph():
    """getCore keeps exactly the edges between kept vertices, in input order (rows sorted, symmetric)."""
    rng = np.random.default_rng(3)
    for o, a in _graphs():
        n = len(o) - 1
        keep = rng.random(n) < 0.6
        so, sa, ids = prune.get_core(o, a, keep)
        assert np.array_equal(ids, np.flatnonzero(keep))
        sub = nx.relabel_nodes(_nx(o, a).subgraph(ids.tolist()), {int(v): i for i, v in enumerate(ids)})
        assert int(so[-1]) // 2 == sub.number_of_edges()
        for v in range(len(ids)):
            row = sa[so[v]:so[v + 1]]
            assert np.all(np.diff(row) > 0)
            assert set(row.tolist()) == set(sub.neighbors(v))


@pytest.mark.parametrize("variant,eps", [("seq", (0, 1)), ("peel", (1, 10)), ("peel", (0, 1)), ("sort", (0, 1))])
def test_framework_against_brute_force(variant, eps):
    """On small graphs: every refined graph is a ceil(L)-core that contains a densest subgraph (the core-containment
    lemma), the best never exceeds rho* and never decreases below the initial core's density, the initial core has
    density >= k_max / 2 (the folklore corollary), and the best mask recounts to the reported pair."""
    for o, a in _small_graphs():
        es, vs = brute.densest_brute(o, a)
        G = _nx(o, a)
        r = prune.par_run(o, a, 8, variant, eps)
        # a densest subgraph, by brute force over subsets
        n = len(o) - 1
        best_sets = [S for S in _all_densest(o, a, es, vs)]
        for t, lev in enumerate(r.levels):
            keep = set(np.flatnonzero(r.core >= lev).tolist())
            assert any(S <= keep for S in best_sets), "a densest subgraph was pruned away"
            K = nx.k_core(G, lev)
            assert r.sizes[t] == (K.number_of_nodes(), K.number_of_edges())
        be, bv, _ = r.best
        assert be * vs <= es * bv
        m1, n1 = r.sizes[0][1], r.sizes[0][0]
        assert be * n1 >= m1 * bv
        assert 2 * es >= r.kmax * vs  # rho* >= k_max / 2 (folklore corollary)
        L0 = (r.kmax + 1) // 2
        assert 2 * m1 >= L0 * n1  # every vertex of the L-core has degree >= L
        ids = np.flatnonzero(r.best_mask)
        assert len(ids) == bv and brute.induced_edges(o, a, r.best_mask) == be
        # replay the improvements: the level after each is max(L0, ceil(rho(S))), and the graph refined at
        # iteration t is the core of the level reached before it
        cur, lev = (m1, n1), L0
        for t, (e, v) in enumerate(r.hist):
            assert r.levels[t] == lev
            if e * cur[1] > cur[0] * v:
                cur, lev = (e, v), max(lev, -(-e // v))
        assert (be, bv) == cur and r.level == lev


def _all_densest(o, a, es, vs):
    n = len(o) - 1
    out = []
    for mask in range(1, 1 << n):
        sel = np.array([(mask >> v) & 1 for v in range(n)], dtype=bool)
        if sel.sum() * es == brute.induced_edges(o, a, sel) * vs and sel.sum() == vs:
            out.append(set(np.flatnonzero(sel).tolist()))
    return out


def test_framework_converges_to_the_optimum():
    """With enough iterations of sequential Greedy++ as Refine, the framework reaches rho* on small graphs."""
    for o, a in _small_graphs()[:5]:
        es, vs = brute.densest_brute(o, a)
        r = prune.par_run(o, a, 300, "seq")
        be, bv, _ = r.best
        assert be * vs == es * bv, (r.best, (es, vs))


def test_no_pruning_reduces_to_plain_greedy():
    """When the ceil(k_max/2)-core is the whole graph and no improvement raises the level (a clique: rho = (k-1)/2
    and ceil((k-1)/2) = ceil(k_max/2)), the framework is plain Greedy++ step for step."""
    for k in (3, 4, 7, 8):
        o, a = graphgen.complete(k)
        for variant, eps in [("seq", (0, 1)), ("peel", (1, 10)), ("sort", (0, 1))]:
            r = prune.par_run(o, a, 6, variant, eps)
            ref = oracle.run(o, a, 6, variant, eps)
            assert r.prunes == 0 and r.sizes == [(k, k * (k - 1) // 2)] * 6
            assert r.hist == ref.hist and r.hist_idx == ref.hist_idx
            assert (r.best[0], r.best[1]) == (int(ref.best[0]), int(ref.best[1]))


def test_isolated_vertices_are_pruned_first():
    """k_max >= 1 gives L >= 1, so the first prune drops every isolated vertex and nothing else when the rest is a
    forest (all core numbers 1): the refined graph is the input without its isolated vertices."""
    o, a = graphgen.from_edges(12, [(0, 3), (3, 5), (5, 9), (2, 7)])
    r = prune.par_run(o, a, 3, "peel", (1, 10))
    assert r.kmax == 1 and r.level == 1
    assert r.sizes[0] == (6, 4)
