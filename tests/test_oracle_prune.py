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


# ------------------------------------------------------------------ approximate k-core pruning
APX_RATIOS = [(3, 2), (2, 1), (11, 10), (5, 2)]


def _bigger_graphs():
    return [graphgen.config1(1), graphgen.rmat(3, 11, 16 << 11), graphgen.chunglu(5, 3000, 2.1, 10.0, 300.0),
            graphgen.er_planted(7, 500, 3000, 30, 1, 3)]


def test_approx_core_numbers_bracket_networkx():
    """core(v) <= khat(v) <= c * core(v) for every vertex (the c-approximate decomposition, in its one-sided form),
    with networkx's core numbers as the reference; c = 1 gives the core numbers themselves, and khat_max lies in
    [k_max, c * k_max]."""
    for o, a in _graphs() + _bigger_graphs():
        cn = nx.core_number(_nx(o, a))
        core = np.array([cn[v] for v in range(len(o) - 1)], dtype=np.int64)
        kmax = int(core.max()) if len(core) else 0
        exact, _ = prune.approx_coreness(o, a, (1, 1))
        assert np.array_equal(exact, core)
        for cn_, cd in APX_RATIOS:
            khat, khat_max = prune.approx_coreness(o, a, (cn_, cd))
            assert np.all(core <= khat) and np.all(cd * khat.astype(np.int64) <= cn_ * core)
            assert kmax <= khat_max and cd * khat_max <= cn_ * kmax


def test_approx_rounds_by_hand():
    """A path 0-1-2-3-4 and a triangle 5-6-7, c = 3/2.  Round 1: min degree 1 (the path's ends), D = 1: vertices 0
    and 4 go.  Round 2: the path 1-2-3 has degrees 1, 2, 1; D stays 1: 1 and 3 go.  Round 3: vertex 2 has degree 0,
    the triangle 2; min 0, D stays 1: vertex 2 goes.  Round 4: min 2, D = 3: the triangle.  khat = 1 on the path
    and 3 on the triangle, whose core number is 2 (3 <= 3/2 * 2)."""
    o, a = graphgen.from_edges(8, [(0, 1), (1, 2), (2, 3), (3, 4), (5, 6), (6, 7), (5, 7)])
    khat, khat_max = prune.approx_coreness(o, a, (3, 2))
    assert khat.tolist() == [1, 1, 1, 1, 1, 3, 3, 3] and khat_max == 3


def test_approx_cut_keeps_every_densest_subgraph():
    """Corollary apxkmax: S* lies in the ceil(khat_max / (2c))-approximate core.  Checked against every densest set
    found by brute force on the small graphs, and on the bigger ones against the exact densest set of Goldberg's
    min cut (rho* >= khat_max / (2c) as well)."""
    from exact_density import densest_exact

    for o, a in _small_graphs():
        es, vs = brute.densest_brute(o, a)
        sets = _all_densest(o, a, es, vs)
        for cn_, cd in APX_RATIOS:
            khat, khat_max = prune.approx_coreness(o, a, (cn_, cd))
            L = prune.ceil_div(khat_max * cd, 2 * cn_)
            keep = set(np.flatnonzero(khat >= L).tolist())
            assert all(S <= keep for S in sets)
            assert 2 * cn_ * es >= khat_max * cd * vs
    for o, a in _bigger_graphs():
        rho, mask = densest_exact(o, a)
        for cn_, cd in APX_RATIOS:
            khat, khat_max = prune.approx_coreness(o, a, (cn_, cd))
            L = prune.ceil_div(khat_max * cd, 2 * cn_)
            assert np.all(khat[mask] >= L)
            assert 2 * cn_ * rho >= khat_max * cd


@pytest.mark.parametrize("variant,eps", [("peel", (1, 10)), ("sort", (0, 1)), ("seq", (0, 1))])
def test_apx_then_exact_equals_exact_pruning(variant, eps):
    """Approximate, then exact pruning (PaRApxGreedy++) refines the same graphs as exact pruning (PaRGreedy++): its
    first level max(ceil(khat_max / 2c), ceil(k_max / 2)) is ceil(k_max / 2), and above the approximate level the
    cut graph has the input's k-cores.  Every output but the decomposition matches; the exact core numbers it
    computes on the cut graph equal networkx's on the input for every vertex at or above the approximate level."""
    for o, a in _graphs() + _bigger_graphs():
        ref = prune.par_run(o, a, 6, variant, eps)
        G = _nx(o, a)
        cn = nx.core_number(G)
        for c in APX_RATIOS[:2]:
            r = prune.par_run(o, a, 6, variant, eps, prune="apx_exact", c=c)
            assert (r.best, r.hist, r.hist_idx, r.sizes, r.levels, r.kmax, r.level, r.prunes) == \
                (ref.best, ref.hist, ref.hist_idx, ref.sizes, ref.levels, ref.kmax, ref.level, ref.prunes)
            assert np.array_equal(r.best_mask, ref.best_mask)
            hi = np.flatnonzero(r.apx_core >= r.apx_level)
            assert r.apx_size[0] == len(hi)
            for v in hi:
                if cn[int(v)] >= r.apx_level:
                    assert r.core[v] == cn[int(v)]
                else:
                    assert r.core[v] < r.apx_level


@pytest.mark.parametrize("variant,eps", [("sort", (0, 1)), ("peel", (1, 10))])
def test_apx_pruning_framework_against_brute_force(variant, eps):
    """Approximate pruning only (PaRApxSorting++ for SORT): every refined graph is {khat >= level} and contains a
    densest subgraph; the first is the approximate core of Corollary apxkmax; the best never exceeds rho*, the best
    mask recounts to the reported pair, and replaying the improvements gives the recorded levels."""
    for o, a in _small_graphs():
        es, vs = brute.densest_brute(o, a)
        sets = _all_densest(o, a, es, vs)
        for c in APX_RATIOS[:2]:
            r = prune.par_run(o, a, 8, variant, eps, prune="apx", c=c)
            khat, khat_max = prune.approx_coreness(o, a, c)
            assert np.array_equal(r.core, khat) and r.kmax == khat_max
            L0 = prune.ceil_div(khat_max * c[1], 2 * c[0])
            assert r.apx_level == L0 and r.levels[0] == L0
            for t, lev in enumerate(r.levels):
                keep = np.flatnonzero(khat >= lev)
                assert any(S <= set(keep.tolist()) for S in sets)
                sel = np.zeros(len(o) - 1, dtype=bool)
                sel[keep] = True
                assert r.sizes[t] == (len(keep), brute.induced_edges(o, a, sel))
            be, bv, _ = r.best
            assert be * vs <= es * bv
            assert int(r.best_mask.sum()) == bv and brute.induced_edges(o, a, r.best_mask) == be
            m1, n1 = r.sizes[0][1], r.sizes[0][0]
            cur, lev = (m1, n1), L0
            for t, (e, v) in enumerate(r.hist):
                assert r.levels[t] == lev
                if e * cur[1] > cur[0] * v:
                    cur, lev = (e, v), max(lev, -(-e // v))
            assert (be, bv) == cur and r.level == lev


def test_apx_pruning_reaches_the_optimum():
    """PaRApxSorting++ with enough iterations reaches rho* on the small graphs (the cuts never drop a densest set)."""
    for o, a in _small_graphs()[:5]:
        es, vs = brute.densest_brute(o, a)
        r = prune.par_run(o, a, 300, "sort", prune="apx")
        be, bv, _ = r.best
        assert be * vs == es * bv, (r.best, (es, vs))
