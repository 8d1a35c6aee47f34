"""Full-size parity, in the launch configuration that bench.py times.

* R-MAT scale 22 (n = 4,194,304, m = 64,156,259), PEEL eps = 1/10 and
  SORT, T = 20.  Checked bit for bit against stored oracle results
  (tests/golden/config2*.json, written by tests/golden/make_golden.py from
  the oracle alone).  The comparison covers per-iteration densities and
  indices, order digests, round counts, best pair, and SHA-256 of the loads,
  of the best-set mask, and of the last iteration's rounds and positions.
* Chung-Lu n = 40M, gamma 2.1 (the 5 GB configuration), SORT T = 50 and PEEL
  eps = 1/20 T = 50, bit for bit against stored oracle results
  (tests/golden/config3_{sort,peel}.json, the same fields as above).  This is
  the only configuration whose edge positions pass 2^30, whose owner ranges
  exceed the bucketed path's limit and whose SORT class table lives outside
  L2.  Beside it, properties that hold at any size: sum of loads = T*m, the
  best mask recounted from the CSR on the host equals (edges, vertices),
  per-iteration width <= Delta, positions form a permutation, and the
  ordering property of the last iteration holds.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import graphgen
import oracle
from gpu_helpers import log

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


@pytest.fixture(scope="module")
def dsg():
    import torch

    import paper_2311_04333_amd as dsg

    assert torch.cuda.is_available()
    return dsg


@pytest.fixture(scope="module")
def config2():
    log("generating R-MAT scale 22")
    return graphgen.config2(1)


@pytest.mark.parametrize("hub", [True, False])
@pytest.mark.parametrize("golden_name", ["config2", "config2_sort"])
def test_config2_against_golden(dsg, config2, golden_name, hub):
    path = os.path.join(HERE, "golden", golden_name + ".json")
    with open(path) as f:
        gd = json.load(f)
    o, a = config2
    assert sha(o) + sha(a) == gd["csr_sha256"], "generator output changed"
    ctx = dsg.Context(0)
    g = dsg.Graph(ctx, o, a, t_cap=gd["T"], hub_order=hub)
    log(f"{golden_name}: running {gd['variant']} T={gd['T']} hub_order={hub}")
    g.run(gd["T"], tuple(gd["eps"]), gd["variant"])
    g.sync()
    dens = g.iter_densities()
    assert [[e, v] for e, v, _ in dens] == gd["hist"]
    assert [i for _, _, i in dens] == gd["hist_idx"]
    digests, rounds = g.digests()
    assert rounds == gd["rounds"]
    assert [str(d) for d in digests] == gd["digests"]
    assert list(g.best()) == gd["best"]
    loads = g.loads()
    assert int(loads.sum()) == gd["loads_sum"]
    assert sha(loads.astype(np.int64)) == gd["loads_sha256"]
    assert sha(g.best_mask().astype(np.uint8)) == gd["best_mask_sha256"]
    rnd, pos, _ = g.order()
    assert sha(rnd.astype(np.int32)) == gd["last_round_sha256"]
    assert sha(pos.astype(np.int32)) == gd["last_pos_sha256"]


def _recount(o, a, mask):
    src = np.repeat(np.arange(len(o) - 1, dtype=np.int64), np.diff(o))
    sel = mask[src] & mask[a] & (src < a)
    return int(sel.sum())


@pytest.fixture(scope="module")
def config3():
    log("generating Chung-Lu n=40M")
    return graphgen.config3(1)


def _compare_golden(g, gd, what):
    dens = g.iter_densities()
    assert [[e, v] for e, v, _ in dens] == gd["hist"], what
    assert [i for _, _, i in dens] == gd["hist_idx"], what
    digests, rounds = g.digests()
    assert rounds == gd["rounds"], what
    assert [str(d) for d in digests] == gd["digests"], what
    assert list(g.best()) == gd["best"], what
    loads = g.loads()
    assert int(loads.sum()) == gd["loads_sum"], what
    assert sha(loads.astype(np.int64)) == gd["loads_sha256"], what
    assert sha(g.best_mask().astype(np.uint8)) == gd["best_mask_sha256"], what
    rnd, pos, _ = g.order()
    assert sha(rnd.astype(np.int32)) == gd["last_round_sha256"], what
    assert sha(pos.astype(np.int32)) == gd["last_pos_sha256"], what


@pytest.mark.parametrize("hub", [True, False])
@pytest.mark.parametrize("golden_name", ["config3_sort", "config3_peel"])
def test_config3_against_golden(dsg, config3, golden_name, hub):
    with open(os.path.join(HERE, "golden", golden_name + ".json")) as f:
        gd = json.load(f)
    o, a = config3
    assert sha(o) + sha(a) == gd["csr_sha256"], "generator output changed"
    ctx = dsg.Context(0)
    g = dsg.Graph(ctx, o, a, t_cap=gd["T"], validate=False, hub_order=hub)
    log(f"{golden_name}: running {gd['variant']} eps={gd['eps']} T={gd['T']} hub_order={hub}")
    g.run(gd["T"], tuple(gd["eps"]), gd["variant"])
    g.sync()
    _compare_golden(g, gd, golden_name)
    g.close()
    ctx.close()


@pytest.mark.parametrize("variant,eps,T", [("sort", (0, 1), 50), ("peel", (1, 20), 10)])
def test_config3_properties(dsg, config3, variant, eps, T):
    o, a = config3
    n, m = len(o) - 1, len(a) // 2
    delta = int(np.diff(o).max())
    ctx = dsg.Context(0)
    g = dsg.Graph(ctx, o, a, t_cap=T)
    if variant == "sort":
        g.run(1, eps, variant)
        ref = oracle.run(o, a, 1, variant, eps)
        assert np.array_equal(g.loads(), ref.loads)
        assert [(e, v) for e, v, _ in g.iter_densities()] == ref.hist
        assert g.digests()[0] == ref.digests
        g.reset()
    log(f"config3 {variant}: T={T}")
    prev_loads = None
    for t in range(T):
        if t == T - 1:
            prev_loads = g.loads()
        g.run(1, eps, variant)
    g.sync()
    loads = g.loads()
    assert int(loads.sum()) == T * m
    inc = loads - prev_loads
    assert inc.min() >= 0 and inc.max() <= delta
    e, v, it, idx = g.best()
    mask = g.best_mask()
    assert int(mask.sum()) == v and _recount(o, a, mask) == e
    rnd, pos, _ = g.order()
    assert np.array_equal(np.sort(pos), np.arange(n))
    start = prev_loads[np.argsort(pos)]
    run_max = np.maximum.accumulate(start)
    p, q = eps
    assert np.all(q * run_max <= (q + p) * (start + delta))
    dens = g.iter_densities()
    for (de, dv, di) in dens:
        assert 0 < dv <= n and 0 <= di < n and de <= m
