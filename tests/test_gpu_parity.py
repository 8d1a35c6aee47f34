"""GPU path (through the C ABI) against the CPU oracle, bit for bit.

Every case runs the HIP library and the oracle on the same seeded input and
compares every output exactly: loads, per-iteration (edges, vertices, index),
best pair, best vertex set, order digests, rounds per iteration, and the last
iteration's rounds and positions.  Sizes span several tiles and sweep chunks
with ragged tails, plus the degenerate cases: one vertex, no edges, stars,
cliques, paths, isolated vertices, and rounds that hold a single vertex or
every vertex.
"""
import numpy as np
import pytest

import graphgen
import oracle
from gpu_helpers import assert_same, log
from pins import _small_graphs

pytestmark = pytest.mark.gpu

VARIANTS = [("seq", (0, 1)), ("peel", (1, 10)), ("peel", (0, 1)), ("peel", (1, 20)), ("sort", (0, 1)),
            ("peel_mono", (0, 1)), ("peel_mono", (1, 10))]


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


def run_both(dsg, ctx, o, a, T, variant, eps, t_cap=64):
    g = dsg.Graph(ctx, o, a, t_cap=t_cap)
    g.run(T, eps, variant)
    ref = oracle.run(o, a, T, variant, eps)
    return g, ref


def edge_cases():
    cases = {
        "single_vertex": (np.array([0, 0], np.int32), np.zeros(0, np.int32)),
        "no_edges_n7": (np.zeros(8, np.int32), np.zeros(0, np.int32)),
        "one_edge": graphgen.from_edges(2, [(0, 1)]),
        "triangle": graphgen.complete(3),
        "K8": graphgen.complete(8),
        "K40": graphgen.complete(40),
        "star_9": graphgen.from_edges(10, [(0, j) for j in range(1, 10)]),
        "star_3000": graphgen.from_edges(3001, [(0, j) for j in range(1, 3001)]),
        "path_50": graphgen.from_edges(50, [(i, i + 1) for i in range(49)]),
        "isolated_mix": graphgen.from_edges(30, [(3, 7), (7, 11), (3, 11), (20, 21), (21, 29)]),
        "two_cliques": graphgen.from_edges(11, [(i, j) for i in range(6) for j in range(i + 1, 6)] +
                                           [(6 + i, 6 + j) for i in range(5) for j in range(i + 1, 5)]),
    }
    for i, (o, a) in enumerate(_small_graphs()):
        cases[f"gnp_{i}"] = (o, a)
    return cases


@pytest.mark.parametrize("name", list(edge_cases().keys()))
def test_edge_cases_all_variants(dsg, ctx, name):
    o, a = edge_cases()[name]
    for variant, eps in VARIANTS:
        log(f"case={name} variant={variant} eps={eps}")
        g, ref = run_both(dsg, ctx, o, a, 6, variant, eps)
        assert_same(g, ref, f"{name}/{variant}/{eps}")
        g.close()


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_config1_all_variants(dsg, ctx, seed):
    """ER n=2000, m=20000 + planted 50-set, T=10: sequential and eps-peeling semantics."""
    o, a = graphgen.config1(seed)
    for variant, eps in VARIANTS:
        log(f"config1 seed={seed} variant={variant} eps={eps}")
        g, ref = run_both(dsg, ctx, o, a, 10, variant, eps)
        assert_same(g, ref, f"config1/{seed}/{variant}")
        g.close()


@pytest.mark.parametrize("n,m", [(4097, 30000), (8191, 90000), (12289, 60000), (40000, 400000)])
def test_ragged_multi_tile(dsg, ctx, n, m):
    """Sizes that are not multiples of the 4096-element tiles or the 2048-edge chunks."""
    o, a = graphgen.er_planted(7 + n, n, m, 60, 1, 2)
    for variant, eps in VARIANTS:
        if variant == "seq" and n > 16000:
            continue
        log(f"ragged n={n} m={m} variant={variant} eps={eps}")
        g, ref = run_both(dsg, ctx, o, a, 4, variant, eps)
        assert_same(g, ref, f"ragged/{n}/{variant}")
        g.close()


@pytest.mark.parametrize("scale", [12, 16])
def test_rmat_skewed(dsg, ctx, scale):
    """R-MAT (hubs, many isolated vertices) with the configuration's quadrant probabilities."""
    o, a = graphgen.rmat(3, scale, 16 << scale)
    for variant, eps in [("peel", (1, 10)), ("peel", (1, 20)), ("peel", (0, 1)), ("sort", (0, 1)),
                         ("peel_mono", (0, 1)), ("peel_mono", (1, 20))]:
        log(f"rmat scale={scale} variant={variant} eps={eps}")
        g, ref = run_both(dsg, ctx, o, a, 5, variant, eps)
        assert_same(g, ref, f"rmat{scale}/{variant}/{eps}")
        g.close()


def test_rmat_large_slices(dsg, ctx):
    """R-MAT scale 20 (1M vertices): each of the 256 round-loop blocks owns more than 4096 alive vertices in the
    first rounds, so the select phase runs several full tiles per block."""
    o, a = graphgen.rmat(4, 20, 16 << 20)
    for variant, eps in [("peel", (1, 10)), ("sort", (0, 1)), ("peel_mono", (1, 10))]:
        log(f"rmat scale=20 variant={variant}")
        g, ref = run_both(dsg, ctx, o, a, 3, variant, eps)
        assert_same(g, ref, f"rmat20/{variant}")
        g.close()


def test_chunglu_small(dsg, ctx):
    """Chung-Lu power law (the shape of the 40M-vertex configuration) at n=200k."""
    o, a = graphgen.chunglu(5, 200_000, 2.1, 30.0, 10_000.0)
    for variant, eps in [("peel", (1, 20)), ("sort", (0, 1)), ("peel_mono", (1, 20))]:
        log(f"chunglu n=200k variant={variant}")
        g, ref = run_both(dsg, ctx, o, a, 3, variant, eps)
        assert_same(g, ref, f"chunglu/{variant}")
        g.close()


def test_resume_and_mixed_variants(dsg, ctx):
    """run(a) then run(b) appends; mixing variants and eps between calls matches the oracle doing the same."""
    o, a = graphgen.config1(4)
    g = dsg.Graph(ctx, o, a, t_cap=32)
    ref = None
    for T, variant, eps in [(2, "peel", (1, 10)), (3, "sort", (0, 1)), (1, "seq", (0, 1)), (2, "peel", (1, 20)),
                            (0, "peel", (1, 10)), (2, "peel_mono", (0, 1)), (2, "peel", (1, 10))]:
        log(f"resume step T={T} variant={variant}")
        g.run(T, eps, variant)
        ref = oracle.run(o, a, T, variant, eps, state=ref)
    assert_same(g, ref, "resume")
    one = dsg.Graph(ctx, o, a, t_cap=32).run(7, (1, 10), "peel")
    two = dsg.Graph(ctx, o, a, t_cap=32).run(3, (1, 10), "peel").run(4, (1, 10), "peel")
    assert np.array_equal(one.loads(), two.loads()) and one.best() == two.best()
    assert one.digests() == two.digests()


def test_reset(dsg, ctx):
    o, a = graphgen.config1(5)
    g = dsg.Graph(ctx, o, a, t_cap=16).run(4, (1, 10), "peel")
    g.reset().run(3, (0, 1), "sort")
    assert_same(g, oracle.run(o, a, 3, "sort"), "reset")


@pytest.mark.parametrize("variant", ["peel", "sort", "seq"])
def test_kernel_timing(dsg, ctx, variant):
    """Kernel timing (events around each iteration's dominant kernel) changes no result and counts one launch per
    iteration of the last run; with timing off it reports nothing."""
    o, a = graphgen.er_planted(21, 3000, 24000, 40, 1, 2)
    ref = oracle.run(o, a, 4, variant, (1, 10))
    g = dsg.Graph(ctx, o, a, t_cap=8).set_kernel_timing(True).run(4, (1, 10), variant)
    ms, launches = g.kernel_timing()
    assert launches == 4 and ms > 0.0
    assert_same(g, ref, f"timed {variant}")
    g.set_kernel_timing(False).run(1, (1, 10), variant)
    assert g.kernel_timing() == (0.0, 0)
    assert_same(g, oracle.run(o, a, 5, variant, (1, 10)), f"untimed {variant} after timed")


@pytest.mark.parametrize("variant", ["peel", "sort", "seq", "peel_mono"])
def test_bounds_against_exact_density(dsg, ctx, variant):
    """Independent of the oracle: on config 1 and R-MAT scale 11 the GPU's best density never exceeds the exact
    rho* (Goldberg's min cut), rho* <= max load / T holds after every iteration, and sequential Greedy++
    reaches rho* within 20 iterations."""
    from exact_density import densest_exact

    eps = (1, 10) if variant in ("peel", "peel_mono") else (0, 1)
    for name, (o, a) in [("config1", graphgen.config1(1)), ("rmat11", graphgen.rmat(3, 11, 16 << 11))]:
        r, _ = densest_exact(o, a)
        es, vs = r.numerator, r.denominator
        g = dsg.Graph(ctx, o, a, t_cap=20)
        for T in range(1, 21):
            g.run(1, eps, variant)
            be, bv = g.best()[:2]
            assert be * vs <= es * bv, (name, T)
            assert es * T <= int(g.loads().max()) * vs, (name, T)
        if variant == "seq":
            assert be * vs == es * bv, (name, (be, bv), (es, vs))
        log(f"{name} {variant}: best {be}/{bv} vs rho* {es}/{vs}")
        g.close()


@pytest.mark.parametrize("variant", ["peel", "sort", "seq", "peel_mono"])
def test_graph_replay(dsg, ctx, variant):
    """A run captured into a HIP graph and replayed gives the oracle's results on every replay, with other eager work
    and synchronisations between the replays; a different T, or a run continuing the history, captures anew."""
    eps = (1, 10) if variant in ("peel", "peel_mono") else (0, 1)
    o, a = graphgen.er_planted(23, 3000, 24000, 40, 1, 2)
    ref = oracle.run(o, a, 4, variant, eps)
    other = dsg.Graph(ctx, *graphgen.rmat(4, 12, 16 << 12), t_cap=4)
    g = dsg.Graph(ctx, o, a, t_cap=8).set_graph_replay(True)
    states = []
    for rep in range(4):
        g.reset().run(4, eps, variant)
        states.append(g.graph_replay_state())
        assert_same(g, ref, f"{variant} replay {rep}")
        other.reset().run(2, (1, 10), "peel")  # eager work on the same stream between the replays
        other.sync()
    log(f"{variant}: replay states {states}")
    assert states == [1, 1, 1, 1]
    g.reset().run(3, eps, variant)
    assert_same(g, oracle.run(o, a, 3, variant, eps), f"{variant} recaptured for T=3")
    g.run(2, eps, variant)
    assert_same(g, oracle.run(o, a, 5, variant, eps), f"{variant} continued history")
    g.set_graph_replay(False).reset().run(4, eps, variant)
    assert g.graph_replay_state() == 0
    assert_same(g, ref, f"{variant} eager again")
    g.close()
    other.close()


def test_deterministic(dsg, ctx):
    """Atomics only commute integers: two runs are bit-identical."""
    o, a = graphgen.rmat(9, 14, 16 << 14)
    r1 = dsg.Graph(ctx, o, a, t_cap=8).run(5, (1, 10), "peel")
    r2 = dsg.Graph(ctx, o, a, t_cap=8).run(5, (1, 10), "peel")
    assert np.array_equal(r1.loads(), r2.loads())
    assert r1.digests() == r2.digests() and r1.best() == r2.best()


def test_invalid_csr_rejected(dsg, ctx):
    """Validation turns every broken CSR property into DSG_EINVAL before any peeling kernel runs."""
    good_o, good_a = graphgen.from_edges(4, [(0, 1), (1, 2), (2, 3)])
    bad = {
        "asymmetric": (good_o, np.array([1, 0, 2, 1, 3, 1], np.int32)),
        "self_loop": (np.array([0, 1, 2], np.int32), np.array([0, 1], np.int32)),
        "unsorted": (np.array([0, 2, 3, 4], np.int32), np.array([2, 1, 0, 0], np.int32)),
        "out_of_range": (good_o, np.array([1, 0, 2, 1, 3, 9], np.int32)),
        "offsets_decrease": (np.array([0, 3, 2, 6, 6], np.int32), good_a),
        "offsets_end": (np.array([0, 1, 3, 5, 5], np.int32), good_a),
    }
    for name, (o, a) in bad.items():
        log(f"invalid csr case={name}")
        with pytest.raises(dsg.DsgError) as ei:
            dsg.Graph(ctx, o, a, t_cap=4)
        assert ei.value.status == -1, name


def test_guards(dsg, ctx):
    """Overflow guard, history capacity and the SEQ size limit fail cleanly without running kernels."""
    o, a = graphgen.from_edges(1 << 16, [(0, j) for j in range(1, 1 << 16)])
    g = dsg.Graph(ctx, o, a, t_cap=40000)
    with pytest.raises(dsg.DsgError) as ei:
        g.run(33000, (1, 10), "peel")  # (33000 + 1) * 65535 >= 2^31
    assert ei.value.status == -4
    with pytest.raises(dsg.DsgError) as ei:
        g.run(1, (1, 10), "seq")  # n = 65536 > 16000
    assert ei.value.status == -1
    small = dsg.Graph(ctx, *graphgen.complete(5), t_cap=2)
    small.run(2, (0, 1), "sort")
    with pytest.raises(dsg.DsgError):
        small.run(1, (0, 1), "sort")


def _bucket_cases():
    ec = edge_cases()
    cases = {k: ec[k] for k in ["single_vertex", "no_edges_n7", "triangle", "K40", "star_3000", "isolated_mix"]}
    cases["config1"] = graphgen.config1(6)
    cases["ragged_4097"] = graphgen.er_planted(11, 4097, 30000, 60, 1, 2)
    cases["rmat16"] = graphgen.rmat(12, 16, 16 << 16)
    cases["chunglu_200k"] = graphgen.chunglu(13, 200_000, 2.1, 30.0, 10_000.0)
    return cases


@pytest.mark.parametrize("name", list(_bucket_cases().keys()))
def test_peel_bucket_paths(dsg, ctx, name):
    """PEEL round-loop paths against the oracle: owner buckets in every round or in none, and coarse (4096-edge) or
    fine (1024-edge) sweep chunks in every round.  Covers partial last ranges, empty rounds and isolated vertices."""
    o, a = _bucket_cases()[name]
    for eps in [(1, 10), (0, 1)]:
        ref = oracle.run(o, a, 4, "peel", eps)
        for bkt, coarse in [(0, 0), (0, 1 << 62), (1 << 62, 0), (1 << 62, 1 << 62)]:
            log(f"bucket case={name} eps={eps} bucket_min={bkt} coarse_min={coarse}")
            g = dsg.Graph(ctx, o, a, t_cap=8).set_peel_tuning(bkt, coarse)
            g.run(4, eps, "peel")
            assert_same(g, ref, f"bucket/{name}/{eps}/{bkt}/{coarse}")
            g.close()


def test_peel_bucket_more_ranges_than_blocks(dsg, ctx):
    """n = 12M vertices: 367 owner ranges of 32768 ids, more than the round loop's blocks, so blocks apply several
    ranges per bucketed round (and the last range is partial).  Under hub order the graph takes the narrow apply
    (256 line-dealt ranges of 2^16 ids with 16-bit counters, the hubs' counters apart)."""
    o, a = graphgen.er_planted(14, 12_000_000, 14_000_000, 60, 1, 2)
    ref = oracle.run(o, a, 2, "peel", (1, 10))
    for thr in [0, 1 << 62]:
        for hub in [False, True]:
            log(f"bucket n=12M threshold={thr} hub_order={hub}")
            g = dsg.Graph(ctx, o, a, t_cap=4, hub_order=hub).set_peel_tuning(thr, thr)
            g.run(2, (1, 10), "peel")
            assert_same(g, ref, f"bucket12M/{thr}/{hub}")
            g.close()


@pytest.mark.parametrize("name", list(_bucket_cases().keys()))
def test_sort_coarse_rank_paths(dsg, ctx, name):
    """SORT with the coarse position classes forced on and off: both equal the oracle (the classes only order
    edges whose endpoints differ in class; equal classes fall back to the full positions)."""
    o, a = _bucket_cases()[name]
    ref = oracle.run(o, a, 5, "sort")
    for coarse in [1, 0]:
        log(f"sort coarse case={name} coarse={coarse}")
        g = dsg.Graph(ctx, o, a, t_cap=8).set_sort_tuning(coarse)
        g.run(5, (0, 1), "sort")
        assert_same(g, ref, f"sortcoarse/{name}/{coarse}")
        g.close()


@pytest.mark.parametrize("name", ["K40", "star_3000", "isolated_mix", "config1", "ragged_4097", "rmat16"])
def test_width_and_load_bounds(dsg, ctx, name):
    """Per-iteration empirical width (largest load increase) and largest load equal the oracle's, for every
    variant; the load bound rho* <= L_t / t is then the oracle's too."""
    o, a = _bucket_cases()[name]
    n = len(o) - 1
    for variant, eps in VARIANTS:
        if variant == "seq" and n > 16000:
            continue
        log(f"bounds case={name} variant={variant}")
        g = dsg.Graph(ctx, o, a, t_cap=8).run(5, eps, variant)
        st, ref = None, []
        for _ in range(5):
            st = oracle.run(o, a, 1, variant, eps, state=st)
            ref.append((st.width[-1], int(st.loads.max()) if n > 0 else 0))
        assert g.iter_bounds() == ref, f"{name}/{variant}: {g.iter_bounds()} vs {ref}"
        g.close()


def _near_cases():
    ec = edge_cases()
    cases = {k: ec[k] for k in ["single_vertex", "no_edges_n7", "one_edge", "triangle", "K40", "star_3000",
                                "path_50", "isolated_mix", "two_cliques", "gnp_0", "gnp_5"]}
    cases["config1"] = graphgen.config1(4)
    cases["ragged_12289"] = graphgen.er_planted(17, 12289, 70000, 60, 1, 2)
    cases["rmat16"] = graphgen.rmat(21, 16, 16 << 16)
    cases["chunglu_300k"] = graphgen.chunglu(23, 300_000, 2.1, 30.0, 15_000.0)
    return cases


@pytest.mark.parametrize("name", list(_near_cases().keys()))
def test_peel_near_select(dsg, ctx, name):
    """The near-list select against the oracle: PEEL and PEEL_MONO at several eps (eps = 0 gives many rounds with
    tiny frontiers, where the near list runs empty and rounds rescan the full list for the exact minimum), with
    owner buckets in every round or in none, over 5 iterations (loads make later priorities tie densely)."""
    o, a = _near_cases()[name]
    for variant, eps in [("peel", (1, 10)), ("peel", (0, 1)), ("peel", (1, 20)), ("peel_mono", (0, 1)),
                         ("peel_mono", (1, 10))]:
        ref = oracle.run(o, a, 5, variant, eps)
        for bkt in (0, 1 << 62):
            log(f"near case={name} variant={variant} eps={eps} bucket_min={bkt}")
            g = dsg.Graph(ctx, o, a, t_cap=8).set_peel_select(1).set_peel_tuning(bkt, -1)
            g.run(5, eps, variant)
            assert_same(g, ref, f"near/{name}/{variant}/{eps}/{bkt}")
            g.close()


def test_peel_select_modes_agree_large(dsg, ctx):
    """A 2M-vertex Chung-Lu graph (thousands of owner-range entries per block, a near list of millions): both
    selects give the same results, and those of the oracle."""
    o, a = graphgen.chunglu(29, 2_000_000, 2.1, 20.0, 100_000.0)
    ref = oracle.run(o, a, 3, "peel", (1, 20))
    for mode in (0, 1):
        log(f"select mode={mode} on Chung-Lu 2M")
        g = dsg.Graph(ctx, o, a, t_cap=4).set_peel_select(mode)
        g.run(3, (1, 20), "peel")
        assert_same(g, ref, f"chunglu2M/select{mode}")
        g.close()


@pytest.mark.parametrize("variant,eps", [("peel", (1, 10)), ("sort", (0, 1)), ("seq", (0, 1)), ("peel_mono", (1, 20))])
def test_run_until_certificate(dsg, ctx, variant, eps):
    """dsg_run_until stops at the first iteration whose load certificate L_t * v * den <= t * e * (den + num) holds,
    computed here from the oracle's own loads and best pair one iteration at a time, and leaves exactly the
    oracle's state after that many iterations (or after T_max when the certificate never holds)."""
    cases = [("config1", graphgen.config1(2), (1, 50), 40), ("K40", graphgen.complete(40), (0, 1), 5),
             ("rmat12", graphgen.rmat(8, 12, 16 << 12), (1, 20), 30), ("rmat12_tight", graphgen.rmat(8, 12, 16 << 12),
                                                                        (0, 1), 6)]
    for name, (o, a), (tn, td), tmax in cases:
        if variant == "seq" and len(o) - 1 > 16000:
            continue
        st, stop = None, None
        for t in range(1, tmax + 1):
            st = oracle.run(o, a, 1, variant, eps, state=st)
            lmax = int(st.loads.max())
            e, v = int(st.best[0]), int(st.best[1])
            if lmax * v * td <= t * e * (td + tn):
                stop = t
                break
        log(f"run_until case={name} variant={variant} tol={tn}/{td}: oracle stops at {stop}")
        g = dsg.Graph(ctx, o, a, t_cap=tmax)
        it, ok = g.run_until(tmax, eps, variant, (tn, td))
        assert ok == (stop is not None), name
        assert it == (stop if stop is not None else tmax), (name, it, stop)
        assert_same(g, st, f"run_until/{name}/{variant}")
        g.close()
