"""Autotuners: the batched persistent kernel's schedule, and the single-graph PEEL round loop's settings.

The batch kernel has three block/chunk shapes (cfg 0: 256 threads with
1024-edge sweep chunks and a 2048-slot LDS decrement table; cfg 1: 512 /
2048 / 4096; cfg 2: 1024 / 4096 / 8192).  It also has a cap on resident
blocks per CU.  Which is fastest depends on the mix of graph sizes: small
graphs want many resident blocks, and large ones want wider blocks and
larger chunks.  The tuner times each candidate on a systematic sample of
the batch and keeps the fastest.  The answer is cached per device name and
size bucket, which is the rounded log2 of the sample's mean and maximum edge
counts.

For one large graph, tune_peel times the PEEL round loop's settings that
change speed but never results: the select (full list or near list), the
frontier size from which a round applies decrements through owner buckets
(the hub threshold: below it, decrements go to per-target device atomics
after the per-chunk LDS aggregation), and the frontier size from which a
round sweeps 4096-edge chunks.

The cache lives in $DSG_AUTOTUNE_CACHE (default
~/.cache/paper_2311_04333_amd/autotune.json).  Delete it to retune.
"""
from __future__ import annotations

import json
import math
import os
import time

CANDIDATES = [(0, 4), (0, 2), (1, 2), (1, 1), (2, 1)]


def cache_path() -> str:
    return os.environ.get("DSG_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_2311_04333_amd", "autotune.json"))


def size_bucket(graphs) -> str:
    m = [max(1, len(a) // 2) for _, a in graphs]
    mean = sum(m) / len(m)
    return f"mean{int(round(math.log2(mean)))}_max{int(round(math.log2(max(m))))}"


def _load_cache():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(c):
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(c, f, indent=1)
    os.replace(tmp, path)


def tune_batch(ctx, graphs, T: int = 2, eps=(1, 10), sample: int = 256, use_cache: bool = True, log=None):
    """Pick (cfg, blocks_per_cu) for a batch like `graphs`; returns (cfg, bpc, {candidate: ms})."""
    import torch

    import paper_2311_04333_amd as dsg

    step = max(1, len(graphs) // sample)
    samp = graphs[::step][:sample]
    dev = torch.cuda.get_device_name(ctx.device)
    key = f"{dev}|{size_bucket(samp)}|T{T}"
    cache = _load_cache() if use_cache else {}
    if key in cache:
        e = cache[key]
        return e["cfg"], e["blocks_per_cu"], e.get("timings_ms", {})
    b = dsg.Batch(ctx, samp, T=T, eps=eps, t_cap=2 * T + 2, validate=False)
    timings = {}
    for cfg, bpc in CANDIDATES:
        b.set_config(cfg, bpc)
        b.reset().run()
        b.last_run_ms()  # warm
        b.reset().run()
        ms = b.last_run_ms()
        timings[f"{cfg},{bpc}"] = ms
        if log:
            log(f"autotune cfg={cfg} blocks/CU={bpc}: {ms:.2f} ms on {len(samp)} graphs")
    b.close()
    best = min(timings, key=timings.get)
    cfg, bpc = (int(x) for x in best.split(","))
    if use_cache:
        cache[key] = {"cfg": cfg, "blocks_per_cu": bpc, "timings_ms": timings, "tuned_at": time.time()}
        _store_cache(cache)
    return cfg, bpc, timings


# Single-graph PEEL round loop: (select, bucket_min_edges, coarse_min_edges).  select 0 = full-list, 1 = near-list;
# the two thresholds count a round's frontier adjacency entries (owner buckets, 4096-edge chunks from that size).
PEEL_CANDIDATES = [(s, b, c) for s in (0, 1) for b in (1 << 14, 1 << 17, 1 << 20, 1 << 62) for c in (1 << 18, 1 << 20)]


def peel_size_bucket(n: int, nnz: int) -> str:
    return f"n{int(round(math.log2(max(n, 1))))}_e{int(round(math.log2(max(nnz, 1))))}"


def tune_peel(ctx, graph, T: int = 2, eps=(1, 10), use_cache: bool = True, log=None):
    """Pick (select, bucket_min_edges, coarse_min_edges) for PEEL on `graph` (a dsg.Graph, whose state is reset
    afterwards) by timing T iterations of each candidate (after one warm-up run).  Results do not depend on the
    choice; only speed does.  Cached per device, size bucket, eps and T.  Returns (select, bucket, coarse,
    {candidate: ms})."""
    import torch

    dev = torch.cuda.get_device_name(ctx.device)
    key = f"{dev}|peel|{peel_size_bucket(graph.n, graph.nnz)}|eps{eps[0]}/{eps[1]}|T{T}"
    cache = _load_cache() if use_cache else {}
    if key in cache:
        e = cache[key]
        return e["select"], e["bucket_min_edges"], e["coarse_min_edges"], e.get("timings_ms", {})
    timings = {}
    for sel, bkt, coarse in PEEL_CANDIDATES:
        graph.set_peel_select(sel).set_peel_tuning(bkt, coarse)
        graph.reset().run(T, eps, "peel")
        graph.sync()
        graph.reset().run(T, eps, "peel")
        ms = graph.last_run_ms()
        timings[f"{sel},{bkt},{coarse}"] = ms
        if log:
            log(f"autotune peel select={sel} bucket_min={bkt} coarse_min={coarse}: {ms:.2f} ms for T={T}")
    best = min(timings, key=timings.get)
    sel, bkt, coarse = (int(x) for x in best.split(","))
    graph.set_peel_select(sel).set_peel_tuning(bkt, coarse)
    graph.reset()
    if use_cache:
        cache[key] = {"select": sel, "bucket_min_edges": bkt, "coarse_min_edges": coarse, "timings_ms": timings,
                      "tuned_at": time.time()}
        _store_cache(cache)
    return sel, bkt, coarse, timings
