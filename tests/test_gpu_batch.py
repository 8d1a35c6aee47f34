"""Batched persistent kernel: every graph of a batch matches the oracle (and the single-graph path) bit for bit.

The batch mixes the three families of the batched workload (Erdos-Renyi,
R-MAT, ER with a planted dense block) with uneven sizes, plus degenerate
graphs.  Graphs may have different T and eps.  Checked outputs: loads,
per-iteration densities and indices, best pair and set, order digests and
round counts.
"""
import numpy as np
import pytest

import graphgen
import oracle
from gpu_helpers import assert_same, bad_csrs, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dsg():
    import torch

    import paper_2311_04333_amd as dsg

    assert torch.cuda.is_available()
    return dsg


@pytest.fixture(scope="module")
def ctx(dsg):
    c = dsg.Context(0)
    yield c
    c.close()


def mix_small(seed, count, nmax):
    """Graphs of the batched mix (same sampler), keeping those with n <= nmax so the oracle stays fast."""
    out, i = [], 0
    while len(out) < count:
        kind, n, d, gseed = graphgen.mix_params(seed, i)
        if n <= nmax:
            out.append(graphgen.mix_graph(seed, i))
        i += 1
    return out


def degenerate():
    return [
        (np.array([0, 0], np.int32), np.zeros(0, np.int32)),
        (np.zeros(6, np.int32), np.zeros(0, np.int32)),
        graphgen.complete(9),
        graphgen.from_edges(40, [(0, j) for j in range(1, 40)]),
        graphgen.from_edges(30, [(i, i + 1) for i in range(29)]),
    ]


@pytest.mark.parametrize("cfg", [0, 1, 2])
def test_batch_matches_oracle(dsg, ctx, cfg):
    graphs = mix_small(11, 30, 20000) + degenerate()
    T, eps = 4, (1, 10)
    log(f"batch cfg={cfg}: {len(graphs)} graphs")
    b = dsg.Batch(ctx, graphs, T=T, eps=eps, t_cap=16).set_config(cfg, 4)
    b.run()
    b.last_run_ms()
    for i, (o, a) in enumerate(graphs):
        ref = oracle.run(o, a, T, "peel", eps)
        assert_same(b.view(i), ref, f"batch cfg={cfg} graph {i}", check_order=False)
    b.close()


def test_batch_equals_alone(dsg, ctx):
    """Each graph's batched result equals its result run alone through the single-graph path."""
    graphs = mix_small(23, 12, 60000)
    b = dsg.Batch(ctx, graphs, T=5, eps=(1, 10), t_cap=8).run()
    for i, (o, a) in enumerate(graphs):
        g = dsg.Graph(ctx, o, a, t_cap=8).run(5, (1, 10), "peel")
        v = b.view(i)
        assert np.array_equal(v.loads(), g.loads()), i
        assert v.best() == g.best(), i
        assert np.array_equal(v.best_mask(), g.best_mask()), i
        assert v.iter_densities() == g.iter_densities(), i
        assert v.digests() == g.digests(), i
        g.close()


def test_batch_per_graph_T_eps_and_resume(dsg, ctx):
    graphs = mix_small(5, 16, 15000)
    Ts = [1 + (i % 5) for i in range(len(graphs))]
    epss = [(1, 10), (1, 20), (0, 1), (3, 7)] * 4
    b = dsg.Batch(ctx, graphs, T=Ts, eps=epss, t_cap=16)
    b.run().run()  # two launches: every graph does 2*T iterations
    for i, (o, a) in enumerate(graphs):
        ref = oracle.run(o, a, 2 * Ts[i], "peel", epss[i])
        assert_same(b.view(i), ref, f"graph {i} T={Ts[i]} eps={epss[i]}", check_order=False)
    b.reset().run()
    for i, (o, a) in enumerate(graphs):
        ref = oracle.run(o, a, Ts[i], "peel", epss[i])
        assert_same(b.view(i), ref, f"after reset graph {i}", check_order=False)


def test_batch_history_guard(dsg, ctx):
    graphs = mix_small(7, 3, 5000)
    b = dsg.Batch(ctx, graphs, T=3, t_cap=4).run()
    with pytest.raises(dsg.DsgError) as ei:
        b.run()
    assert ei.value.status == -1


def test_batch_validation(dsg, ctx):
    """DSG_VALIDATE on a batch: valid graphs (empty rows, hubs spanning many chunks) pass and match the oracle,
    and every broken CSR property anywhere in the batch is DSG_EINVAL."""
    good = [graphgen.rmat(5, 14, 16 << 14), graphgen.from_edges(6, [(0, 5), (2, 5)]),
            graphgen.from_edges(3, []), graphgen.chunglu(7, 50_000, 2.1, 20.0, 8000.0)]
    b = dsg.Batch(ctx, good, T=3, eps=(1, 10), t_cap=4, validate=True).run()
    for i, (o, a) in enumerate(good):
        ref = oracle.run(o, a, 3, "peel", (1, 10))
        assert b.best(i) == tuple(int(x) for x in ref.best), i
    b.close()
    for name, (o, a) in bad_csrs().items():
        log(f"batch validation case={name}")
        with pytest.raises(dsg.DsgError) as ei:
            dsg.Batch(ctx, [good[1], (o, a)], T=2, eps=(1, 10), t_cap=2, validate=True)
        assert ei.value.status == -1, name
