"""Pruning-and-Refining (Algorithm 1) on the GPU against the oracle's framework, bit for bit: core numbers, k_max,
every refined graph's size and core level, the per-iteration (edges, vertices, index) of S', the best pair, the
iteration that found it, the best set, the final level and the number of prunes."""
import numpy as np
import pytest

import graphgen
from gpu_helpers import log
from oracle import prune
from test_gpu_parity import edge_cases

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


def assert_par_same(g, r, what):
    assert g.kmax == r.kmax, f"{what}: kmax {g.kmax} vs {r.kmax}"
    assert np.array_equal(g.core, r.core), f"{what}: core numbers differ at {np.flatnonzero(g.core != r.core)[:10]}"
    assert g.sizes == r.sizes, f"{what}: refined graph sizes {g.sizes} vs {r.sizes}"
    assert g.levels == r.levels, f"{what}: levels differ"
    assert g.hist == r.hist, f"{what}: per-iteration densities differ"
    assert g.hist_idx == r.hist_idx, f"{what}: per-iteration indices differ"
    assert g.best == r.best, f"{what}: best {g.best} vs {r.best}"
    assert np.array_equal(g.best_mask, r.best_mask), f"{what}: best set differs"
    assert g.level == r.level and g.prunes == r.prunes, f"{what}: level/prunes {g.level, g.prunes} vs {r.level, r.prunes}"


def _cases():
    ec = edge_cases()
    cases = {k: ec[k] for k in ["single_vertex", "no_edges_n7", "one_edge", "triangle", "K8", "K40", "star_3000",
                                "path_50", "isolated_mix", "two_cliques", "gnp_0", "gnp_8"]}
    cases["config1_s1"] = graphgen.config1(1)
    cases["config1_s2"] = graphgen.config1(2)
    cases["ragged_12289"] = graphgen.er_planted(7 + 12289, 12289, 60000, 60, 1, 2)
    cases["rmat12"] = graphgen.rmat(3, 12, 16 << 12)
    cases["rmat16"] = graphgen.rmat(5, 16, 16 << 16)
    cases["chunglu_200k"] = graphgen.chunglu(5, 200_000, 2.1, 30.0, 10_000.0)
    return cases


VARIANTS = [("peel", (1, 10)), ("peel", (0, 1)), ("sort", (0, 1)), ("peel_mono", (1, 20))]


@pytest.mark.parametrize("name", list(_cases().keys()))
def test_par_against_oracle(dsg, ctx, name):
    o, a = _cases()[name]
    n = len(o) - 1
    vs = VARIANTS + ([("seq", (0, 1))] if n <= 16000 else [])
    for variant, eps in vs:
        log(f"par case={name} variant={variant} eps={eps}")
        ref = prune.par_run(o, a, 8, variant, eps)
        g = dsg.par_run(ctx, o, a, 8, eps, variant)
        assert_par_same(g, ref, f"{name}/{variant}/{eps}")


def test_par_zero_iterations(dsg, ctx):
    """T = 0: only the initial prune; the best is the ceil(k_max/2)-core."""
    o, a = graphgen.config1(3)
    ref = prune.par_run(o, a, 0, "peel", (1, 10))
    g = dsg.par_run(ctx, o, a, 0, (1, 10), "peel")
    assert g.best == ref.best and g.kmax == ref.kmax and np.array_equal(g.best_mask, ref.best_mask)


def test_par_rmat22_full_size(dsg, ctx):
    """R-MAT scale 22 (n = 4,194,304), PEEL eps = 1/10, T = 20, in the configuration bench.py times."""
    log("par: generating R-MAT scale 22")
    o, a = graphgen.config2(1)
    log("par: oracle framework (coreness + cuts + 20 refinements)")
    ref = prune.par_run(o, a, 20, "peel", (1, 10))
    log(f"par: oracle done, k_max={ref.kmax} sizes {ref.sizes[0]} .. {ref.sizes[-1]}")
    g = dsg.par_run(ctx, o, a, 20, (1, 10), "peel")
    assert_par_same(g, ref, "rmat22")


def test_par_invalid_arguments(dsg, ctx):
    o, a = graphgen.complete(4)
    with pytest.raises(dsg.DsgError):
        dsg.par_run(ctx, o, a, -1, (1, 10), "peel")
    bad_o, bad_a = np.array([0, 1, 2], np.int32), np.array([0, 1], np.int32)  # self-loops
    with pytest.raises(dsg.DsgError):
        dsg.par_run(ctx, bad_o, bad_a, 2, (1, 10), "peel")


@pytest.mark.parametrize("name", ["single_vertex", "no_edges_n7", "triangle", "K40", "star_3000", "path_50",
                                  "isolated_mix", "config1_s1", "rmat16", "chunglu_200k"])
def test_coreness_against_oracle(dsg, ctx, name):
    """dsg_coreness equals the oracle's sequential Coreness (core numbers are unique)."""
    import oracle

    o, a = _cases()[name]
    core, kmax, rounds, _ = dsg.coreness(ctx, o, a)
    ref, rk = oracle.coreness(o, a)
    assert kmax == rk and np.array_equal(core, ref)
    assert rounds >= 1


def test_coreness_chunglu_40m(dsg, ctx):
    """Core numbers of the 40M-vertex Chung-Lu graph (1.1 billion adjacency entries) against the oracle."""
    import oracle

    log("coreness: generating Chung-Lu n=40M")
    o, a = graphgen.config3(1)
    log("coreness: GPU")
    core, kmax, rounds, ms = dsg.coreness(ctx, o, a, validate=False, timed=True)
    log(f"coreness: k_max={kmax}, {rounds} rounds, {ms:.1f} ms; oracle")
    ref, rk = oracle.coreness(o, a)
    assert kmax == rk and np.array_equal(core, ref)


# ------------------------------------------------------------------ approximate k-core pruning
def assert_apx_same(g, r, what):
    assert_par_same(g, r, what)
    assert np.array_equal(g.apx_core, r.apx_core), \
        f"{what}: approximate core numbers differ at {np.flatnonzero(g.apx_core != r.apx_core)[:10]}"
    assert (g.apx_kmax, g.apx_level, g.apx_size) == (r.apx_kmax, r.apx_level, r.apx_size), \
        f"{what}: approximate cut {(g.apx_kmax, g.apx_level, g.apx_size)} vs {(r.apx_kmax, r.apx_level, r.apx_size)}"


APX_CASES = ["single_vertex", "no_edges_n7", "one_edge", "triangle", "K40", "star_3000", "path_50", "isolated_mix",
             "two_cliques", "gnp_8", "config1_s1", "config1_s2", "ragged_12289", "rmat12", "rmat16", "chunglu_200k"]


@pytest.mark.parametrize("name", APX_CASES)
def test_par_apx_against_oracle(dsg, ctx, name):
    """PaRApxSorting++ (approximate pruning, SORT) and PaRApxGreedy++ (approximate then exact pruning, PEEL), plus
    the crossed pairs, at c = 3/2 and c = 2, against the oracle's frameworks bit for bit, including the approximate
    core numbers of every vertex."""
    o, a = _cases()[name]
    for prune_mode, variant, eps in [("apx", "sort", (0, 1)), ("apx_exact", "peel", (1, 10)),
                                     ("apx", "peel", (1, 20)), ("apx_exact", "sort", (0, 1))]:
        for c in [(3, 2), (2, 1)]:
            log(f"par apx case={name} prune={prune_mode} variant={variant} eps={eps} c={c}")
            ref = prune.par_run(o, a, 8, variant, eps, prune=prune_mode, c=c)
            g = dsg.par_run(ctx, o, a, 8, eps, variant, prune=prune_mode, c=c)
            assert_apx_same(g, ref, f"{name}/{prune_mode}/{variant}/{c}")


def test_par_apx_rmat22_full_size(dsg, ctx):
    """R-MAT scale 22: PaRApxGreedy++ (PEEL eps = 1/10) and PaRApxSorting++ (SORT), c = 3/2, T = 20."""
    log("par apx: generating R-MAT scale 22")
    o, a = graphgen.config2(1)
    for prune_mode, variant, eps in [("apx_exact", "peel", (1, 10)), ("apx", "sort", (0, 1))]:
        log(f"par apx rmat22: oracle {prune_mode}/{variant}")
        ref = prune.par_run(o, a, 20, variant, eps, prune=prune_mode, c=(3, 2))
        g = dsg.par_run(ctx, o, a, 20, eps, variant, prune=prune_mode, c=(3, 2))
        assert_apx_same(g, ref, f"rmat22/{prune_mode}/{variant}")


def test_par_apx_invalid_ratio(dsg, ctx):
    o, a = graphgen.complete(5)
    for c in [(1, 1), (2, 3), (3, 0)]:
        with pytest.raises(dsg.DsgError):
            dsg.par_run(ctx, o, a, 2, (1, 10), "peel", prune="apx", c=c)
