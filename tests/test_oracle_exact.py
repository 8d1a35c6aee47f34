"""The exact-density tool (Goldberg's min cut with Dinkelbach iteration) against brute force and closed forms.

The tool pins the oracle on graphs too large to enumerate (pins.py), so it is
pinned itself first: it must equal exhaustive enumeration on every small
graph of the pin family and the closed forms of cliques, stars, two disjoint
cliques and the empty graph, and the vertex set it returns must have the
density it reports.
"""
from fractions import Fraction

import numpy as np
import pytest

import graphgen
from exact_density import densest_exact
from oracle import brute
from pins import _small_graphs


def _density(o, a, mask):
    src = np.repeat(np.arange(len(o) - 1), np.diff(o))
    e = int(np.count_nonzero(mask[src] & mask[a])) // 2
    return Fraction(e, int(mask.sum()))


@pytest.mark.parametrize("i", range(len(_small_graphs())))
def test_exact_equals_brute_force(i):
    o, a = _small_graphs()[i]
    r, mask = densest_exact(o, a)
    e, v = brute.densest_brute(o, a)
    assert r == Fraction(e, v)
    assert _density(o, a, mask) == r


def test_exact_closed_forms():
    for k in (2, 3, 6, 11):
        assert densest_exact(*graphgen.complete(k))[0] == Fraction(k - 1, 2)
    for s in (1, 4, 9):
        o, a = graphgen.from_edges(s + 1, [(0, j) for j in range(1, s + 1)])
        assert densest_exact(o, a)[0] == Fraction(s, s + 1)
    # K_7 and K_4 disjoint: the larger clique, and only it
    edges = [(i, j) for i in range(7) for j in range(i + 1, 7)] + [(7 + i, 7 + j) for i in range(4) for j in range(i + 1, 4)]
    r, mask = densest_exact(*graphgen.from_edges(11, edges))
    assert r == 3 and mask.tolist() == [True] * 7 + [False] * 4
    assert densest_exact(np.zeros(6, np.int32), np.zeros(0, np.int32))[0] == 0


def test_exact_planted_set_is_found():
    """Config 1: the planted 50-vertex set (pair probability 1/2, about 12 internal neighbours per vertex) is far
    denser than the ER background (density 10); the densest set returned has the planted set's size."""
    o, a = graphgen.config1(1)
    r, mask = densest_exact(o, a)
    assert int(mask.sum()) == 50 and _density(o, a, mask) == r
    assert r > Fraction(20000, 2000)


@pytest.mark.parametrize("variant,eps", [("seq", (0, 1)), ("peel", (1, 10)), ("peel", (0, 1)), ("sort", (0, 1)),
                                         ("peel_mono", (1, 20))])
def test_load_certificate_is_sound(variant, eps):
    """The stopping certificate's bound rho* <= L_t / t (L_t = largest load after t iterations): every iteration of
    every ordering charges each edge to one of its endpoints, so the loads inside a densest set S* grow by at least
    |E(S*)| per iteration.  Checked against the exact rho* after each of 12 iterations on the pin family, config 1
    and a small R-MAT graph; the best density found never exceeds rho* either."""
    import oracle

    graphs = list(_small_graphs()) + [graphgen.config1(2), graphgen.rmat(6, 9, 16 << 9)]
    for o, a in graphs:
        r, _ = densest_exact(o, a)
        st = None
        for t in range(1, 13):
            st = oracle.run(o, a, 1, variant, eps, state=st)
            lmax = int(st.loads.max()) if len(st.loads) else 0
            assert r * t <= lmax, (variant, t)
            e, v = int(st.best[0]), int(st.best[1])
            assert Fraction(e, v) <= r
