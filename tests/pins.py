"""Pins that tie the CPU oracle to facts the paper and the mathematics fix.

Each pin is a function ``pin_xxx(lib)``.  It takes an oracle library handle
(see ``oracle.load_library``) and raises AssertionError when the oracle
contradicts the fact.  ``test_oracle_pins.py`` runs every pin against the
real oracle.  ``test_oracle_mutants.py`` runs them against copies of the
oracle with a planted mistake, and each mutant must fail at least one pin.

Sources of the facts:
  * closed forms derived by hand from Algorithms 2/3 (complete graphs, stars,
    two disjoint cliques, the empty graph, a triangle and a path under
    round-synchronous peeling);
  * exhaustive enumeration (``oracle.brute``) for the exact optimum rho* on
    graphs with n <= 14, and Goldberg's min-cut construction (``exact_density``,
    scipy's max-flow as the step) on graphs of thousands of vertices;
  * Charikar's 2-approximation for the first iteration (Section 3.2), and
    the (1+eps)-relaxed form of it for round-synchronous peeling;
  * the dual bound rho* <= max_v l(v) / T: every edge of S* is charged to an
    endpoint inside S*;
  * Algorithm 3 invariants: the whole graph's edges equal B[0], the sum of
    the loads is T*m, and every suffix count B[i] equals a direct recount;
  * degeneracy order: the running maximum degree at peel time in the first
    sequential iteration gives the core numbers (Section 2, Coreness).  It is
    checked against networkx.core_number and against the k-core definition;
  * the ordering property of Section 3.2 / 3.3: for positions i < j,
    l(v_i) <= l(v_j) + Delta (eps = 0), and its (1+eps)-relaxed form;
  * the bucketing k-core algorithm of Section 3.1: with zero loads and
    eps = 0, the monotone-bound rounds are the core-number buckets;
  * the SplitMix64 known answer: from state 0 its first output is
    0xE220A8397B1DCDAF.
"""
from __future__ import annotations

import itertools

import numpy as np

import graphgen
import oracle
from oracle import brute


def _K(k):
    return graphgen.complete(k)


def _small_graphs():
    """A fixed family of small random graphs (seeded G(n, p))."""
    out = []
    for seed, n, pn, pd in [(1, 8, 1, 2), (2, 10, 2, 5), (3, 12, 1, 3), (4, 9, 3, 5), (5, 14, 1, 4), (6, 11, 1, 2),
                            (7, 13, 2, 7), (8, 7, 4, 5)]:
        out.append(graphgen.gnp(seed, n, pn, pd))
    # a graph with a dense part and a sparse tail
    out.append(graphgen.from_edges(12, [(i, j) for i in range(5) for j in range(i + 1, 5)] +
                                   [(4, 5), (5, 6), (6, 7), (7, 8), (8, 9), (9, 10), (10, 11), (3, 7)]))
    return out


# --------------------------------------------------------------------- closed forms
def pin_complete_graph_loads(lib):
    """K_k: after t = 2s+1 iterations l(i) = s(k-1) + (k-1-i); after t = 2s, l(i) = s(k-1).

    Derivation: with equal loads every vertex has priority k-1 and the
    lower id goes first, so vertex i is charged k-1-i.  The next iteration
    reverses the order and charges i, which equalises the loads again.  The
    whole graph stays the best, since every proper suffix is a smaller
    clique.
    """
    for k in (1, 2, 3, 5, 8):
        o, a = _K(k)
        for var, eps in (("seq", (0, 1)), ("peel", (0, 1)), ("sort", (0, 1)), ("peel", (1, 10))):
            if var == "peel" and eps == (1, 10) and k > 5:
                continue  # (1+eps) groups several vertices per round once k > 10
            for T in (1, 2, 3, 4):
                st = oracle.run(o, a, T, var, eps, lib=lib)
                s, odd = divmod(T, 2)
                expect = np.array([s * (k - 1) + ((k - 1 - i) if odd else 0) for i in range(k)])
                assert np.array_equal(st.loads, expect), (k, var, T, st.loads, expect)
                m = k * (k - 1) // 2
                assert tuple(st.best[:3]) == (m, k, 0), (k, var, st.best)
                assert all(h == (m, k) for h in st.hist), st.hist


def pin_sort_first_iteration_is_id_order(lib):
    """GreedySorting++ orders by start-of-iteration load.  With all loads 0 the order is id order,
    so vertex v is charged its number of higher-id neighbours."""
    for o, a in _small_graphs():
        st = oracle.run(o, a, 1, "sort", lib=lib)
        n = len(o) - 1
        assert np.array_equal(st.last_pos, np.arange(n))
        hi = np.array([np.sum(a[o[v]:o[v + 1]] > v) for v in range(n)])
        assert np.array_equal(st.loads, hi)


def pin_sort_second_iteration_orders_by_load(lib):
    """Iteration 2 of SORT visits vertices in (load after iteration 1, id) order."""
    for o, a in _small_graphs():
        st = oracle.run(o, a, 1, "sort", lib=lib)
        l1 = st.loads.copy()
        st = oracle.run(o, a, 1, "sort", state=st, lib=lib)
        n = len(o) - 1
        expect = sorted(range(n), key=lambda v: (l1[v], v))
        got = np.argsort(st.last_pos)
        assert list(got) == expect


def pin_star(lib):
    """K_{1,s}: rho* = s/(s+1) is the whole graph; it stays the best subgraph."""
    for s in (1, 2, 5, 9):
        o, a = graphgen.from_edges(s + 1, [(0, j) for j in range(1, s + 1)])
        for var, eps in (("seq", (0, 1)), ("peel", (1, 10)), ("sort", (0, 1))):
            st = oracle.run(o, a, 3, var, eps, lib=lib)
            assert tuple(st.best[:3]) == (s, s + 1, 0)
            assert st.loads.sum() == 3 * s


def pin_two_cliques(lib):
    """K_a + K_b disjoint, a > b: the first sequential iteration peels K_b first and finds K_a at index b."""
    for a_, b_ in ((5, 3), (6, 2), (7, 4)):
        edges = [(i, j) for i in range(a_) for j in range(i + 1, a_)]
        edges += [(a_ + i, a_ + j) for i in range(b_) for j in range(i + 1, b_)]
        o, a = graphgen.from_edges(a_ + b_, edges)
        st = oracle.run(o, a, 1, "seq", lib=lib)
        assert tuple(st.best) == (a_ * (a_ - 1) // 2, a_, 1, b_), st.best
        assert st.best_mask().sum() == a_ and st.best_mask()[:a_].all()


def pin_empty_graph(lib):
    """No edges: loads stay 0 and every candidate has density 0; the input graph stays best."""
    o = np.zeros(6, dtype=np.int32)
    a = np.zeros(0, dtype=np.int32)
    for var in ("seq", "peel", "sort"):
        st = oracle.run(o, a, 3, var, (1, 10), lib=lib)
        assert st.loads.sum() == 0
        assert tuple(st.best[:3]) == (0, 5, 0)
        assert st.hist == [(0, 5)] * 3 and st.hist_idx == [0, 0, 0]


def pin_triangle_round_ownership(lib):
    """Triangle, round-synchronous peeling with eps = 1/10.
    Iteration 1: one round, same-round edges go to the lower id: charges (2,1,0).
    Iteration 2: priorities (4,3,2) peel {2}, then {1}, then {0}: loads (2,2,2)."""
    o, a = _K(3)
    st = oracle.run(o, a, 1, "peel", (1, 10), lib=lib)
    assert list(st.loads) == [2, 1, 0] and st.rounds == [1]
    assert list(st.last_round) == [0, 0, 0] and list(st.last_pos) == [0, 1, 2]
    st = oracle.run(o, a, 1, "peel", (1, 10), state=st, lib=lib)
    assert list(st.loads) == [2, 2, 2] and st.rounds[-1] == 3
    assert list(st.last_round) == [2, 1, 0] and list(st.last_pos) == [2, 1, 0]


def pin_path_delayed_effects(lib):
    """Path 0-1-2-3, eps = 0.  Round 0 peels {0,3} (degree 1).  Their removal drops 1 and 2 to degree 1, so
    round 1 peels {1,2} and the edge 1-2 goes to vertex 1.  Loads (1,1,0,1); positions 0,3,1,2 -> 0,1,2,3.
    Sequential peeling instead takes 0,1,2,3 one by one: loads (1,1,1,0)."""
    o, a = graphgen.from_edges(4, [(0, 1), (1, 2), (2, 3)])
    st = oracle.run(o, a, 1, "peel", (0, 1), lib=lib)
    assert list(st.loads) == [1, 1, 0, 1]
    assert list(st.last_round) == [0, 1, 1, 0]
    assert list(st.last_pos) == [0, 2, 3, 1]
    assert st.hist == [(3, 4)] and st.hist_idx == [0]
    sq = oracle.run(o, a, 1, "seq", lib=lib)
    assert list(sq.loads) == [1, 1, 1, 0] and list(sq.last_pos) == [0, 1, 2, 3]


def pin_peel_huge_eps_is_id_order(lib):
    """eps so large that the first round takes everyone: the order is id order (same as SORT iteration 1)."""
    for o, a in _small_graphs():
        p = oracle.run(o, a, 1, "peel", (10 ** 9, 1), lib=lib)
        s = oracle.run(o, a, 1, "sort", lib=lib)
        assert p.rounds == [1]
        assert np.array_equal(p.loads, s.loads) and np.array_equal(p.last_pos, s.last_pos)


def pin_peel_eps0_unique_minima_equals_seq(lib):
    """With eps = 0 and a unique minimum in every round, round-synchronous peeling is the sequential
    load ordering.  Start loads (2 Delta + 1) * pi(v) for a permutation pi keep all priorities distinct
    through the iteration (degrees only move them by up to Delta).  So every round is a singleton, and
    PEEL(eps=0), SEQ and SORT all visit the vertices in pi order."""
    rng = np.random.default_rng(11)
    for o, a in _small_graphs():
        n = len(o) - 1
        delta = int(np.diff(o).max())
        pi = rng.permutation(n)
        res = {}
        for var in ("peel", "seq", "sort"):
            st = oracle.State.fresh(o)
            st.loads[:] = (2 * delta + 1) * pi
            res[var] = oracle.run(o, a, 1, var, (0, 1), state=st, lib=lib)
        assert res["peel"].rounds == [n]
        for var in ("seq", "sort"):
            assert np.array_equal(res["peel"].loads, res[var].loads), var
            assert np.array_equal(res["peel"].last_pos, res[var].last_pos), var
            assert res["peel"].hist == res[var].hist, var
        assert np.array_equal(res["peel"].last_pos, pi)


# ---------------------------------------------------------------- brute-force bounds
def pin_bounds_against_brute_force(lib):
    """For every variant and T: rho_best <= rho* <= max l / T (dual bound).
    Iteration 1 of SEQ: rho_best >= rho*/2 (Charikar); of PEEL: rho_best >= rho* / (2 (1 + eps)).
    Empirical width: ceil(rho*) <= max_v (load increase) <= Delta."""
    for o, a in _small_graphs():
        es, vs = brute.densest_brute(o, a)
        delta = int(np.diff(o).max())
        for var, eps in (("seq", (0, 1)), ("peel", (1, 10)), ("peel", (1, 2)), ("sort", (0, 1)),
                         ("peel_mono", (0, 1)), ("peel_mono", (1, 10))):
            st = None
            for T in range(1, 7):
                st = oracle.run(o, a, 1, var, eps, state=st, lib=lib)
                be, bv = int(st.best[0]), int(st.best[1])
                assert be * vs <= es * bv, "best exceeds the optimum"
                assert es * T <= int(st.loads.max()) * vs, "dual bound violated"
                w = st.width[-1]
                assert -(-es // vs) <= w <= delta, (w, es, vs, delta)
                if T == 1 and var == "seq":
                    assert 2 * be * vs >= es * bv, "Charikar bound"
                if T == 1 and var in ("peel", "peel_mono"):
                    q, p = eps[1], eps[0]
                    assert 2 * (q + p) * be * vs >= q * es * bv, "relaxed Charikar bound"


_MEDIUM_EXACT = {}


def _medium_graphs_exact():
    """Medium graphs with rho* from the max-flow tool (exact_density), cached: config 1 (ER n=2000 plus a planted
    50-set), R-MAT scale 11, a Chung-Lu graph and a small planted ER graph."""
    from exact_density import densest_exact

    if not _MEDIUM_EXACT:
        for name, (o, a) in [("config1", graphgen.config1(1)), ("rmat11", graphgen.rmat(3, 11, 16 << 11)),
                             ("chunglu3000", graphgen.chunglu(5, 3000, 2.1, 10.0, 300.0)),
                             ("planted500", graphgen.er_planted(7, 500, 3000, 30, 1, 3))]:
            r, _ = densest_exact(o, a)
            _MEDIUM_EXACT[name] = (o, a, r.numerator, r.denominator)
    return _MEDIUM_EXACT


def pin_bounds_against_exact_medium(lib):
    """The brute-force bounds carried to graphs of thousands of vertices, with rho* = es/vs from Goldberg's
    min-cut construction (exact_density, itself checked against brute force):
      rho_best <= rho* <= max l / T for every variant and T (every edge of S* is charged inside S*);
      iteration 1: SEQ rho_best >= rho*/2 (Charikar), PEEL and PEEL_MONO rho_best >= rho* / (2 (1 + eps));
      the empirical width of every iteration is at least ceil(rho*);
      k_max / 2 <= rho* <= k_max (the k_max-core has minimum degree k_max; every vertex of S* has at least
      rho* neighbours in S*, so S* lies in the ceil(rho*)-core).
    Sequential Greedy++ converges to rho* (observed here within 20 iterations on every graph)."""
    for name, (o, a, es, vs) in _medium_graphs_exact().items():
        _, kmax = oracle.coreness(o, a, lib=lib)
        assert kmax * vs <= 2 * es and es <= kmax * vs, (name, kmax, es, vs)
        for var, eps in (("seq", (0, 1)), ("peel", (1, 10)), ("sort", (0, 1)), ("peel_mono", (1, 20))):
            st = None
            for T in range(1, 21):
                st = oracle.run(o, a, 1, var, eps, state=st, lib=lib)
                be, bv = int(st.best[0]), int(st.best[1])
                assert be * vs <= es * bv, (name, var, T, "best exceeds the optimum")
                assert es * T <= int(st.loads.max()) * vs, (name, var, T, "dual bound violated")
                assert -(-es // vs) <= st.width[-1], (name, var, T, "width below ceil(rho*)")
                if T == 1 and var == "seq":
                    assert 2 * be * vs >= es * bv, (name, "Charikar bound")
                if T == 1 and var in ("peel", "peel_mono"):
                    q, p = eps[1], eps[0]
                    assert 2 * (q + p) * be * vs >= q * es * bv, (name, "relaxed Charikar bound")
            if var == "seq":
                assert int(st.best[0]) * vs == es * int(st.best[1]), (name, st.best[:2], (es, vs))


def pin_convergence(lib):
    """Sequential Greedy++ converges to rho*: after enough iterations the best found equals the
    optimum on these small graphs, and the best density never decreases."""
    for o, a in _small_graphs()[:5]:
        es, vs = brute.densest_brute(o, a)
        st = None
        prev = (0, 1)
        for _ in range(30):
            st = oracle.run(o, a, 10, "seq", lib=lib, state=st)
            be, bv = int(st.best[0]), int(st.best[1])
            assert be * prev[1] >= prev[0] * bv
            prev = (be, bv)
        assert prev[0] * vs == es * prev[1], (prev, (es, vs))


# ------------------------------------------------------------------ Algorithm 3 facts
def pin_suffix_counts_recount(lib):
    """Algorithm 3: B[i] is |E(S_i)| for S_i the suffix of the order from position i (direct recount),
    B[0] = m, and the iteration record is the densest suffix with ties to the smallest i."""
    rng = np.random.default_rng(5)
    for o, a in _small_graphs():
        n = len(o) - 1
        for _ in range(3):
            pos = rng.permutation(n).astype(np.int32)
            A, B, (e, v, i) = oracle.alg3(o, a, pos, lib=lib)
            assert B[0] == len(a) // 2
            for k in range(n):
                assert B[k] == brute.induced_edges(o, a, pos >= k)
            dens = [(int(B[k]), n - k) for k in range(n)]
            bi = 0
            for k in range(1, n):
                if dens[k][0] * dens[bi][1] > dens[bi][0] * dens[k][1]:
                    bi = k
            assert (e, v, i) == (dens[bi][0], dens[bi][1], bi)


def pin_load_sum_and_best_mask(lib):
    """Each edge charges exactly one endpoint per iteration: sum of loads = T*m.  The best mask
    recounted from the CSR has exactly (best edges, best vertices)."""
    for o, a in _small_graphs() + [graphgen.config1(3)]:
        m = len(a) // 2
        for var, eps in (("seq", (0, 1)), ("peel", (1, 10)), ("sort", (0, 1)), ("peel_mono", (1, 10))):
            st = oracle.run(o, a, 5, var, eps, lib=lib)
            assert st.loads.sum() == 5 * m
            mask = st.best_mask()
            assert mask.sum() == st.best[1]
            assert brute.induced_edges(o, a, mask) == st.best[0]


def pin_fused_equals_decoupled(lib):
    """Algorithm 2 run fused (density checked before every single peel) and decoupled (ordering, then
    Algorithm 3) agree exactly: loads, per-iteration records and best."""
    for o, a in _small_graphs() + [graphgen.config1(2)]:
        for var, eps in (("seq", (0, 1)), ("peel", (1, 10)), ("peel", (0, 1)), ("sort", (0, 1)),
                         ("peel_mono", (0, 1)), ("peel_mono", (1, 10))):
            d = oracle.run(o, a, 4, var, eps, lib=lib)
            f = oracle.run_fused(o, a, 4, var, eps, lib=lib)
            assert np.array_equal(d.loads, f.loads), var
            assert d.hist == f.hist and d.hist_idx == f.hist_idx, var
            assert np.array_equal(d.best, f.best), var
            assert np.array_equal(d.best_mask(), f.best_mask()), var


def pin_resume(lib):
    """The state carries across calls: run(a) then run(b) equals run(a + b)."""
    o, a = graphgen.config1(4)
    for var in ("seq", "peel", "sort", "peel_mono"):
        one = oracle.run(o, a, 5, var, (1, 10), lib=lib)
        two = oracle.run(o, a, 2, var, (1, 10), lib=lib)
        two = oracle.run(o, a, 3, var, (1, 10), state=two, lib=lib)
        assert np.array_equal(one.loads, two.loads) and one.hist == two.hist
        assert np.array_equal(one.best, two.best) and one.digests == two.digests


# ------------------------------------------------------------------- orderings
def pin_degeneracy_order_gives_core_numbers(lib):
    """First sequential iteration (loads 0) is a degeneracy ordering: the running maximum of the degree at
    peel time equals the core number (Coreness, Section 2).  It is checked against networkx.core_number
    and against the k-core definition.  The best density is also >= k_max / 2 (the k_max-core is a
    suffix)."""
    import networkx as nx

    graphs = _small_graphs() + [graphgen.config1(1), graphgen.gnp(9, 40, 1, 6)]
    for gi, (o, a) in enumerate(graphs):
        n = len(o) - 1
        st = oracle.run(o, a, 1, "seq", lib=lib)
        order = np.argsort(st.last_pos)
        D = 0
        core = np.zeros(n, dtype=np.int64)
        for v in order:
            D = max(D, int(st.loads[v]))  # load after iteration 1 = degree when peeled
            core[v] = D
        G = nx.Graph()
        G.add_nodes_from(range(n))
        G.add_edges_from(brute.edge_list(o, a).tolist())
        cn = nx.core_number(G)
        assert all(core[v] == cn[v] for v in range(n))
        if n <= 14:
            assert np.array_equal(core, brute.core_numbers_brute(o, a))
        kmax = int(core.max())
        assert 2 * int(st.best[0]) >= kmax * int(st.best[1])


def pin_ordering_property(lib):
    """For positions i < j with start-of-iteration loads: SEQ, SORT and PEEL with eps = 0 satisfy
    l(v_i) <= l(v_j) + Delta (Sections 3.2-3.3); PEEL with eps = p/q satisfies
    q l(v_i) <= (q + p)(l(v_j) + Delta).  So does PEEL_MONO: the bound a vertex v_i is peeled under
    is (1 + eps) times the minimum of some earlier round, when v_j was alive with priority at most
    l(v_j) + Delta."""
    for o, a in _small_graphs() + [graphgen.config1(1)]:
        delta = int(np.diff(o).max())
        for var, eps in (("seq", (0, 1)), ("sort", (0, 1)), ("peel", (0, 1)), ("peel", (1, 10)),
                         ("peel_mono", (0, 1)), ("peel_mono", (1, 10))):
            st = None
            for _ in range(4):
                start = np.zeros(len(o) - 1, dtype=np.int64) if st is None else st.loads.copy()
                st = oracle.run(o, a, 1, var, eps, state=st, lib=lib)
                seq = start[np.argsort(st.last_pos)]
                run_max = np.maximum.accumulate(seq)
                p, q = eps
                assert np.all(q * run_max <= (q + p) * (seq + delta))


def pin_peel_mono_rounds_are_core_buckets(lib):
    """PEEL_MONO with eps = 0 in the first iteration (loads 0) is the bucketing k-core algorithm of
    Section 3.1 (peel everything of degree at most d, raise d when nothing is left at or below it): the
    vertices of one round share one core number k (networkx.core_number, and the k-core definition on
    the smallest graphs), k never falls from one round to the next, and a round takes exactly the alive
    vertices whose current degree is at most k.  Plain PEEL takes only those at the round minimum, so it
    needs more rounds wherever the minimum drops below the core number reached (checked to happen)."""
    import networkx as nx

    graphs = _small_graphs() + [graphgen.config1(1), graphgen.gnp(9, 40, 1, 6), graphgen.rmat(3, 8, 6 << 8)]
    separated = False
    for o, a in graphs:
        n = len(o) - 1
        G = nx.Graph()
        G.add_nodes_from(range(n))
        G.add_edges_from(brute.edge_list(o, a).tolist())
        cn = nx.core_number(G)
        core = np.array([cn[v] for v in range(n)], dtype=np.int64)
        if n <= 14:
            assert np.array_equal(core, brute.core_numbers_brute(o, a))
        st = oracle.run(o, a, 1, "peel_mono", (0, 1), lib=lib)
        rnd = st.last_round
        src = np.repeat(np.arange(n), np.diff(o))
        alive = np.ones(n, dtype=bool)
        prev_k = -1
        for r in range(st.rounds[0]):
            members = np.flatnonzero(rnd == r)
            ks = set(core[members].tolist())
            assert len(ks) == 1, (r, ks)
            k = ks.pop()
            assert k >= prev_k
            prev_k = k
            cur = np.bincount(src, weights=alive[np.asarray(a)], minlength=n)
            expect = np.flatnonzero(alive & (cur <= k))
            assert np.array_equal(members, expect), r
            alive[members] = False
        assert not alive.any()
        plain = oracle.run(o, a, 1, "peel", (0, 1), lib=lib)
        assert plain.rounds[0] >= st.rounds[0]
        separated |= plain.rounds[0] > st.rounds[0]
    assert separated


def pin_seq_is_greedy_min(lib):
    """Sequential order: every peeled vertex minimises load + current degree among the vertices left,
    with ties to the lowest id (checked step by step from the returned order)."""
    for o, a in _small_graphs():
        n = len(o) - 1
        st = None
        for _ in range(3):
            start = np.zeros(n, dtype=np.int64) if st is None else st.loads.copy()
            st = oracle.run(o, a, 1, "seq", state=st, lib=lib)
            order = np.argsort(st.last_pos)
            left = set(range(n))
            for v in order:
                pri = {u: start[u] + sum(1 for w in a[o[u]:o[u + 1]] if w in left) for u in left}
                best = min(left, key=lambda u: (pri[u], u))
                assert v == best
                left.remove(v)


def pin_digest_known_answer(lib):
    """Digest of a one-vertex order is mix64(0), the first SplitMix64 output from state 0."""
    assert oracle.digest(np.zeros(1, dtype=np.int32), lib=lib) == 0xE220A8397B1DCDAF
    o = np.zeros(2, dtype=np.int32)
    a = np.zeros(0, dtype=np.int32)
    st = oracle.run(o, a, 1, "seq", lib=lib)
    assert st.digests == [0xE220A8397B1DCDAF]


ALL_PINS = [v for k, v in sorted(globals().items()) if k.startswith("pin_")]
