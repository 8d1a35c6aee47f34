"""Hub order (DSG_HUB_ORDER): the graph renumbers its vertices by degree inside the library; every output, in the
caller's ids, must still equal the oracle bit for bit.  Ties between vertices peeled in one round, in SEQ's argmin
and in SORT's order all go to the smaller caller id, which the renumbered CSR has to carry through (the flag bit of
its entries, the sorts' caller-order input).  Covers every variant and round-loop path (full-list and near-list
select, bucketed and direct decrements, coarse and fine chunks), the degenerate graphs, mixed-variant resumes, and
a graph large enough for several radix passes and owner ranges."""
import numpy as np
import pytest

import graphgen
import oracle
from gpu_helpers import assert_same, log
from test_gpu_parity import VARIANTS, edge_cases

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dsg():
    import torch

    import paper_2311_04333_amd as dsg

    assert torch.cuda.is_available()
    dsg.library()
    return dsg


@pytest.fixture(scope="module")
def ctx(dsg):
    c = dsg.Context(0)
    yield c
    c.close()


def _cases():
    ec = edge_cases()
    cases = {k: ec[k] for k in ["single_vertex", "no_edges_n7", "one_edge", "triangle", "K40", "star_3000",
                                "path_50", "isolated_mix", "two_cliques", "gnp_0", "gnp_3"]}
    cases["config1"] = graphgen.config1(7)
    cases["ragged_4097"] = graphgen.er_planted(11, 4097, 30000, 60, 1, 2)
    cases["rmat16"] = graphgen.rmat(12, 16, 16 << 16)
    cases["chunglu_200k"] = graphgen.chunglu(13, 200_000, 2.1, 30.0, 10_000.0)
    return cases


@pytest.mark.parametrize("name", list(_cases().keys()))
def test_hub_order_all_variants(dsg, ctx, name):
    o, a = _cases()[name]
    n = len(o) - 1
    for variant, eps in VARIANTS:
        if variant == "seq" and n > 16000:
            continue
        log(f"hub case={name} variant={variant} eps={eps}")
        ref = oracle.run(o, a, 4, variant, eps)
        g = dsg.Graph(ctx, o, a, t_cap=8, hub_order=True)
        assert g.hub_order
        g.run(4, eps, variant)
        assert_same(g, ref, f"hub/{name}/{variant}/{eps}")
        g.close()


@pytest.mark.parametrize("name", ["isolated_mix", "config1", "rmat16", "chunglu_200k"])
def test_hub_order_round_loop_paths(dsg, ctx, name):
    """PEEL and PEEL_MONO under hub order with every select mode and the bucketed / coarse paths forced on or off."""
    o, a = _cases()[name]
    for variant, eps in [("peel", (1, 10)), ("peel", (0, 1)), ("peel_mono", (0, 1))]:
        ref = oracle.run(o, a, 3, variant, eps)
        for sel in [0, 1]:
            for bkt, coarse in [(0, 0), (1 << 62, 1 << 62), (0, 1 << 62)]:
                log(f"hub paths case={name} {variant} eps={eps} select={sel} bucket={bkt} coarse={coarse}")
                g = dsg.Graph(ctx, o, a, t_cap=4, hub_order=True).set_peel_select(sel).set_peel_tuning(bkt, coarse)
                g.run(3, eps, variant)
                assert_same(g, ref, f"hubpaths/{name}/{variant}/{eps}/{sel}/{bkt}/{coarse}")
                g.close()


def test_hub_order_resume_mixed_variants(dsg, ctx):
    o, a = graphgen.config1(4)
    g = dsg.Graph(ctx, o, a, t_cap=32, hub_order=True)
    ref = None
    for T, variant, eps in [(2, "peel", (1, 10)), (3, "sort", (0, 1)), (1, "seq", (0, 1)), (2, "peel", (1, 20)),
                            (2, "peel_mono", (0, 1)), (2, "peel", (1, 10))]:
        log(f"hub resume T={T} variant={variant}")
        g.run(T, eps, variant)
        ref = oracle.run(o, a, T, variant, eps, state=ref)
    assert_same(g, ref, "hub resume")
    g.reset().run(2, (0, 1), "sort")
    assert_same(g, oracle.run(o, a, 2, "sort"), "hub reset")


def test_hub_order_large_equals_plain(dsg, ctx):
    """R-MAT scale 20 (2^20 vertices, more than 2^16 for the four-pass sort by round, 256 owner ranges): hub
    order and the plain layout give identical outputs for PEEL (both selects) and SORT; PEEL also equals the
    oracle."""
    o, a = graphgen.rmat(21, 20, 16 << 20)
    ref = oracle.run(o, a, 2, "peel", (1, 10))
    for sel in [0, 1]:
        log(f"hub rmat20 peel select={sel}")
        g = dsg.Graph(ctx, o, a, t_cap=4, hub_order=True).set_peel_select(sel)
        g.run(2, (1, 10), "peel")
        assert_same(g, ref, f"hub rmat20 peel select={sel}")
        g.close()
    h = dsg.Graph(ctx, o, a, t_cap=4, hub_order=True).run(3, (0, 1), "sort")
    p = dsg.Graph(ctx, o, a, t_cap=4, hub_order=False).run(3, (0, 1), "sort")
    assert np.array_equal(h.loads(), p.loads())
    assert h.digests() == p.digests() and h.best() == p.best() and h.iter_densities() == p.iter_densities()
    assert np.array_equal(h.best_mask(), p.best_mask())
    hr, hp, hn = h.order()
    pr, pp, pn = p.order()
    assert np.array_equal(hr, pr) and np.array_equal(hp, pp) and hn == pn
    h.close()
    p.close()


@pytest.mark.parametrize("variant", ["peel", "sort", "seq"])
def test_hub_order_graph_replay_and_bounds(dsg, ctx, variant):
    """Under hub order a run captured into a HIP graph (with the caller-order gathers of the sorts) replays to the
    oracle's results, with eager work between replays; the width and load bounds and the certificate stop equal the
    oracle's too."""
    eps = (1, 10) if variant == "peel" else (0, 1)
    o, a = graphgen.er_planted(23, 3000, 24000, 40, 1, 2)
    ref = oracle.run(o, a, 4, variant, eps)
    other = dsg.Graph(ctx, *graphgen.rmat(4, 12, 16 << 12), t_cap=4, hub_order=True)
    g = dsg.Graph(ctx, o, a, t_cap=8, hub_order=True).set_graph_replay(True)
    for rep in range(3):
        g.reset().run(4, eps, variant)
        assert g.graph_replay_state() == 1
        assert_same(g, ref, f"hub {variant} replay {rep}")
        other.reset().run(2, (1, 10), "peel")
        other.sync()
    g.close()
    other.close()
    h = dsg.Graph(ctx, o, a, t_cap=8, hub_order=True).run(4, eps, variant)
    p = dsg.Graph(ctx, o, a, t_cap=8, hub_order=False).run(4, eps, variant)
    assert h.iter_bounds() == p.iter_bounds()
    h.close()
    p.close()
    st, stop = None, None
    for t in range(1, 31):
        st = oracle.run(o, a, 1, variant, eps, state=st)
        if int(st.loads.max()) * int(st.best[1]) * 100 <= t * int(st.best[0]) * 101:
            stop = t
            break
    g = dsg.Graph(ctx, o, a, t_cap=30, hub_order=True)
    it, ok = g.run_until(30, eps, variant, (1, 100))
    assert ok == (stop is not None) and it == (stop if stop is not None else 30)
    assert_same(g, st, f"hub run_until {variant}")
    g.close()
