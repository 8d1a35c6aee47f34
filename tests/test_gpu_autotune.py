"""The autotuners choose among settings that change speed but never results: after tuning, the batch and the
single-graph PEEL round loop still equal the oracle bit for bit, and the choice is one of the candidates (and is
read back from the cache on the next call)."""
import os

import pytest

import graphgen
import oracle
from gpu_helpers import assert_same, log
from test_gpu_batch import mix_small

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


def test_tune_peel_then_parity(dsg, ctx, tmp_path, monkeypatch):
    from paper_2311_04333_amd import autotune

    monkeypatch.setenv("DSG_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    o, a = graphgen.chunglu(13, 200_000, 2.1, 30.0, 10_000.0)
    for hub in (False, True):
        g = dsg.Graph(ctx, o, a, t_cap=8, hub_order=hub)
        sel, bkt, coarse, timings = autotune.tune_peel(ctx, g, T=2, eps=(1, 10), log=log)
        assert (sel, bkt, coarse) in autotune.PEEL_CANDIDATES and len(timings) == len(autotune.PEEL_CANDIDATES)
        again = autotune.tune_peel(ctx, g, T=2, eps=(1, 10))  # cached
        assert again[:3] == (sel, bkt, coarse)
        g.run(3, (1, 10), "peel")
        assert_same(g, oracle.run(o, a, 3, "peel", (1, 10)), f"tuned peel hub_order={hub}")
        g.close()
    assert os.path.exists(tmp_path / "tune.json")


def test_tune_batch_then_parity(dsg, ctx, tmp_path, monkeypatch):
    from paper_2311_04333_amd import autotune

    monkeypatch.setenv("DSG_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    graphs = mix_small(31, 24, 20000)
    cfg, bpc, timings = autotune.tune_batch(ctx, graphs, T=2, eps=(1, 10), log=log)
    assert (cfg, bpc) in autotune.CANDIDATES and len(timings) == len(autotune.CANDIDATES)
    b = dsg.Batch(ctx, graphs, T=3, eps=(1, 10), t_cap=4).set_config(cfg, bpc).run()
    for i, (o, a) in enumerate(graphs):
        assert_same(b.view(i), oracle.run(o, a, 3, "peel", (1, 10)), f"tuned batch graph {i}", check_order=False)
    b.close()
