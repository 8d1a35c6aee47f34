"""Serving (continuous batching): each request's result is the same alone and in the mix.

Requests arrive while others are on the GPU.  Every result must match the
oracle run of that graph with the same T and eps.  That is also the result
of the graph run alone (the batched tests pin alone == batched).  Admission
refuses requests beyond the pool or the ring (DSG_EBUSY) and accepts them
again once earlier results are released.
"""
import time

import numpy as np
import pytest

import graphgen
import oracle
from gpu_helpers import bad_csrs, log

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


def small_mix(seed, count, nmax=12000):
    out, i = [], 0
    while len(out) < count:
        kind, n, d, gseed = graphgen.mix_params(seed, i)
        if n <= nmax:
            out.append(graphgen.mix_graph(seed, i))
        i += 1
    return out


def check_result(res, o, a, T, eps, what):
    ref = oracle.run(o, a, T, "peel", eps)
    assert res["best"] == tuple(int(x) for x in ref.best), what
    assert res["hist"] == ref.hist and res["hist_idx"] == ref.hist_idx, what
    assert res["digests"] == ref.digests and res["rounds"] == ref.rounds, what
    if res["loads"] is not None:
        assert np.array_equal(res["loads"], ref.loads), what


def drain(srv, pending, results, timeout=120.0):
    t0 = time.time()
    while pending and time.time() - t0 < timeout:
        for t in srv.poll():
            results[t] = srv.fetch(t, loads=True)
            srv.release(t)
            pending.discard(t)
        time.sleep(0.001)
    assert not pending, f"{len(pending)} requests did not finish"


def test_serve_mixed_stream(dsg, ctx):
    graphs = small_mix(31, 40)
    Ts = [1 + (i * 7) % 9 for i in range(len(graphs))]
    epss = [(1, 10), (1, 20)] * 20
    srv = dsg.Server(ctx, 2 << 30, ring_size=64).start(cfg=1, blocks_per_cu=1, idle_seconds=30, max_seconds=300)
    try:
        tickets, pending, results = {}, set(), {}
        for i, (o, a) in enumerate(graphs):
            t = srv.submit(o, a, Ts[i], epss[i])
            assert t is not None
            tickets[t] = i
            pending.add(t)
            if i % 5 == 4:  # let some finish while the rest arrive
                for done in srv.poll():
                    results[done] = srv.fetch(done, loads=True)
                    srv.release(done)
                    pending.discard(done)
                time.sleep(0.002)
        drain(srv, pending, results)
        log(f"served {len(results)} requests")
        for t, i in tickets.items():
            o, a = graphs[i]
            check_result(results[t], o, a, Ts[i], epss[i], f"request {i}")
    finally:
        srv.stop()
        srv.close()


def test_serve_admission_and_restart(dsg, ctx):
    graphs = small_mix(41, 6, nmax=5000)
    T = 3
    f = [dsg.Server.footprint(len(o) - 1, len(a), T) for o, a in graphs]
    # room for the first two requests only (512 bytes of the pool hold the server's own counters)
    srv = dsg.Server(ctx, 512 + f[0] + f[1] + 128, ring_size=64).start(cfg=0, blocks_per_cu=1, idle_seconds=30,
                                                                       max_seconds=300)
    try:
        t0 = srv.submit(*graphs[0], T)
        t1 = srv.submit(*graphs[1], T)
        assert t0 is not None and t1 is not None
        assert srv.submit(*graphs[2], T) is None  # pool full: DSG_EBUSY
        results = {}
        drain(srv, {t0, t1}, results)
        t2 = srv.submit(*graphs[2], T)  # memory released: admitted
        assert t2 is not None
        drain(srv, {t2}, results)
        srv.stop()
        srv.start(cfg=1, blocks_per_cu=1, idle_seconds=30, max_seconds=300)  # restart never replays old tickets
        t3 = srv.submit(*graphs[0], T)  # fits: graph 0 was admitted into this pool before
        assert t3 is not None and t3 > t2
        drain(srv, {t3}, results)
        for t, i in ((t0, 0), (t1, 1), (t2, 2), (t3, 0)):
            check_result(results[t], *graphs[i], T, (1, 10), f"request {i}")
    finally:
        srv.stop()
        srv.close()


def test_serve_ring_slot_guard(dsg, ctx):
    """Ticket t lives in ring slot t % ring_size: with two slots, ticket 2 waits for ticket 0's release."""
    graphs = small_mix(43, 4, nmax=3000)
    srv = dsg.Server(ctx, 1 << 28, ring_size=2).start(cfg=0, blocks_per_cu=1, idle_seconds=30, max_seconds=300)
    try:
        a = srv.submit(*graphs[0], 2)
        b = srv.submit(*graphs[1], 2)
        assert a is not None and b is not None
        done, t_end = set(), time.time() + 60
        while len(done) < 2 and time.time() < t_end:
            done |= set(srv.poll())
            time.sleep(0.001)
        assert done == {a, b}
        srv.fetch(b)
        srv.release(b)
        assert srv.submit(*graphs[2], 2) is None  # slot 0 still held by ticket a
        res_a = srv.fetch(a)
        srv.release(a)
        c = srv.submit(*graphs[2], 2)
        assert c is not None
        results = {}
        drain(srv, {c}, results)
        check_result(results[c], *graphs[2], 2, (1, 10), "ring reuse")
        check_result(dict(res_a, loads=None), *graphs[0], 2, (1, 10), "first request")
    finally:
        srv.stop()
        srv.close()


def test_serve_registered_graphs(dsg, ctx):
    """Resident graphs: many requests against a few registered CSRs, overlapping on the device."""
    graphs = small_mix(47, 5, nmax=8000)
    srv = dsg.Server(ctx, 1 << 30, ring_size=256)
    try:
        gids = [srv.register(o, a) for o, a in graphs]
        srv.start(cfg=1, blocks_per_cu=1, idle_seconds=30, max_seconds=300)
        plan = [(gids[i % 5], 2 + i % 6, [(1, 10), (1, 20), (0, 1)][i % 3]) for i in range(60)]
        tickets, pending, results = {}, set(), {}
        for j, (gid, T, eps) in enumerate(plan):
            t = srv.submit_registered(gid, T, eps)
            assert t is not None
            tickets[t] = j
            pending.add(t)
        drain(srv, pending, results)
        refs = {}
        for t, j in tickets.items():
            gid, T, eps = plan[j]
            key = (gid, T, eps)
            if key not in refs:
                refs[key] = True
                check_result(results[t], *graphs[gid], T, eps, f"registered request {j}")
        # identical requests give identical results regardless of their place in the mix
        by_key = {}
        for t, j in tickets.items():
            by_key.setdefault(plan[j], []).append(results[t])
        for key, rs in by_key.items():
            assert all(r["digests"] == rs[0]["digests"] and r["best"] == rs[0]["best"] for r in rs), key
    finally:
        srv.stop()
        srv.close()


def test_serve_register_validation(dsg, ctx):
    """Registering with validation rejects every broken CSR property (DSG_EINVAL) and accepts valid graphs."""
    srv = dsg.Server(ctx, 1 << 28, ring_size=8)
    try:
        for name, (o, a) in bad_csrs().items():
            log(f"register validation case={name}")
            with pytest.raises(dsg.DsgError) as ei:
                srv.register(o, a, validate=True)
            assert ei.value.status == -1, name
        assert srv.register(*graphgen.rmat(5, 14, 16 << 14), validate=True) == 0
    finally:
        srv.close()


def test_serve_restart_runs_unclaimed(dsg, ctx):
    """A kernel that leaves when idle, and requests submitted around its exits.

    With a very short idle limit the persistent kernel keeps exiting between
    bursts; a submit then reports DSG_ESTATE and the server is started again.
    A request published just as the last block left (after the submit's
    running check) was never claimed: the next start must run it, so every
    ticket handed out finishes and matches the oracle.
    """
    graphs = small_mix(41, 12, nmax=3000)
    srv = dsg.Server(ctx, 1 << 30, ring_size=32)
    srv.start(cfg=1, blocks_per_cu=1, idle_seconds=0.002, max_seconds=60)
    tickets, pending, results, restarts = {}, set(), {}, 0
    try:
        for burst in range(30):
            for k in range(2):
                i = (2 * burst + k) % len(graphs)
                o, a = graphs[i]
                while True:
                    try:
                        t = srv.submit(o, a, 2, (1, 10))
                    except dsg.DsgError as e:
                        assert e.status == -5, e  # the kernel left: start it again
                        srv.start(cfg=1, blocks_per_cu=1, idle_seconds=0.002, max_seconds=60)
                        restarts += 1
                        continue
                    break
                if t is None:  # ring or pool full: collect results first
                    drain(srv, pending, results, timeout=60)
                    continue
                tickets[t] = i
                pending.add(t)
            time.sleep(0.001 * (burst % 4))
            for t in srv.poll():
                results[t] = srv.fetch(t, loads=True)
                srv.release(t)
                pending.discard(t)
        # whatever is still unclaimed runs once the server is started again
        try:
            srv.stop()
        except dsg.DsgError:
            pass
        srv.start(cfg=1, blocks_per_cu=1, idle_seconds=5, max_seconds=60)
        drain(srv, pending, results, timeout=60)
    finally:
        srv.stop()
        srv.close()
    log(f"restart test: {len(tickets)} requests, {restarts} restarts")
    for t, i in tickets.items():
        o, a = graphs[i]
        check_result(results[t], o, a, 2, (1, 10), f"ticket {t} graph {i}")
