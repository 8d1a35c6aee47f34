"""The largest graphs of the batched mix, at full size, through the batched persistent kernel and through the
serving loop, bit for bit against stored oracle results.

tests/golden/mix_large.json (written by tests/golden/make_golden.py from the oracle alone) holds, for the 8 largest
graphs of the 4096-graph mix (ER with a planted block of 5% of the vertices at p = 0.3: about 18M edges each) and the
2 largest ER and R-MAT graphs, PEEL eps = 1/10, T = 20: per-iteration (edges, vertices, index), order digests and
round counts, the best pair, and SHA-256 of the loads and of the best-set mask.  These graphs are far above the
sizes of the other batch and serving tests.
"""
import hashlib
import json
import os
import time

import numpy as np
import pytest

import graphgen
from gpu_helpers import log

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


@pytest.fixture(scope="module")
def golden():
    with open(os.path.join(HERE, "golden", "mix_large.json")) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def graphs(golden):
    out = []
    for gd in golden["graphs"]:
        o, a = graphgen.mix_graph(1, gd["mix_index"])
        assert sha(o) + sha(a) == gd["csr_sha256"], f"generator output changed for mix graph {gd['mix_index']}"
        out.append((o, a))
    log(f"mix_large: {len(out)} graphs, m = {sum(len(a) // 2 for _, a in out)}")
    return out


@pytest.fixture(scope="module")
def ctx():
    import torch

    import paper_2311_04333_amd as dsg

    assert torch.cuda.is_available()
    c = dsg.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("cfg", [0, 2])
def test_mix_large_batched(ctx, golden, graphs, cfg):
    import paper_2311_04333_amd as dsg

    log(f"mix_large batched cfg={cfg}")
    b = dsg.Batch(ctx, graphs, T=20, eps=(1, 10), t_cap=20).set_config(cfg, 4)
    b.run()
    log(f"mix_large batched cfg={cfg}: {b.last_run_ms():.1f} ms")
    for i, gd in enumerate(golden["graphs"]):
        what = f"mix graph {gd['mix_index']} (cfg {cfg})"
        dens = b.iter_densities(i)
        assert [[e, v] for e, v, _ in dens] == gd["hist"], what
        assert [x for _, _, x in dens] == gd["hist_idx"], what
        digests, rounds = b.digests(i)
        assert rounds == gd["rounds"], what
        assert [str(d) for d in digests] == gd["digests"], what
        assert list(b.best(i)) == gd["best"], what
        loads = b.loads(i)
        assert int(loads.sum()) == gd["loads_sum"], what
        assert sha(loads.astype(np.int64)) == gd["loads_sha256"], what
        assert sha(b.best_mask(i).astype(np.uint8)) == gd["best_mask_sha256"], what
    b.close()


def test_mix_large_served(ctx, golden, graphs):
    """The same graphs as requests to the server, submitted back to back while earlier ones run."""
    import paper_2311_04333_amd as dsg

    srv = dsg.Server(ctx, 8 << 30, ring_size=64).start(cfg=1, blocks_per_cu=1, idle_seconds=60, max_seconds=600)
    try:
        tickets = {}
        for i, (o, a) in enumerate(graphs):
            t = srv.submit(o, a, 20, (1, 10))
            assert t is not None, i
            tickets[t] = i
        results = {}
        t0 = time.time()
        while len(results) < len(graphs) and time.time() - t0 < 240:
            for t in srv.poll():
                results[tickets[t]] = srv.fetch(t, loads=True)
                srv.release(t)
            time.sleep(0.005)
        assert len(results) == len(graphs), f"{len(graphs) - len(results)} requests did not finish"
        log(f"mix_large served in {time.time() - t0:.1f} s")
    finally:
        srv.stop()
        srv.close()
    for i, gd in enumerate(golden["graphs"]):
        what = f"served mix graph {gd['mix_index']}"
        res = results[i]
        assert [list(h) for h in res["hist"]] == gd["hist"], what
        assert res["hist_idx"] == gd["hist_idx"], what
        assert res["rounds"] == gd["rounds"], what
        assert [str(d) for d in res["digests"]] == gd["digests"], what
        assert list(res["best"]) == gd["best"], what
        assert sha(res["loads"].astype(np.int64)) == gd["loads_sha256"], what
