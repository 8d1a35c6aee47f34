#!/usr/bin/env python
"""Benchmark: Greedy++ peeling (PaRGreedy++ ordering) on one MI355X.

Default workload: the Chung-Lu power-law graph with n = 40,000,000 vertices,
degree exponent 2.1, mean degree 30 and degrees capped at 2M (m = 555,487,662
edges after deduplication; a 4.4 GB int32 CSR resident in HBM).  One step is
one full run of the hot path: reset the state, then T = 50 Greedy++
iterations of round-synchronous peeling with eps = 1/20.  Each iteration
does init, the persistent round loop (select, sweep with the charges and the
delayed degree decrements, the order by round), Algorithm 3, and the load
and best updates.  `--workload rmat22` runs R-MAT scale 22 with PEEL
eps = 1/10, T = 20 per step instead.  Both graphs are bound with hub order
(vertices renumbered by degree inside the library, `--hub`); the renumbering
is part of graph creation, outside the timed steps, and its time is printed
under `setup`.

Metric: edge-visits/s = 2m * T * steps / wall time of the timed steps.

Also printed, on the same JSON line:
  roofline      the dominant kernel (the persistent round loop).  Its
                average launch time comes from HIP events recorded on the
                library's stream around every launch of the timed steps.
                Its algorithmic bytes per launch are 16m + 16n: each CSR
                entry read once (8m) plus one 4-byte neighbour-state access
                per entry (8m), and four int32 per-vertex accesses (priority,
                row bounds, round, order).  The iteration's other 16n
                (degree init, loads, Algorithm 3's A and suffix scan) are in
                the smaller kernels; `iteration` gives 16m + 32n over the
                whole iteration time beside it.  `traffic` is the HBM bytes
                per launch from committed rocprofv3 FETCH_SIZE / WRITE_SIZE
                summaries, while they match the kernel sources.
  cpu_baseline  the CPU oracle (single thread) timed on a bounded sample of
                the same workload (see --cpu-*), and beside it (all_cores)
                the oracle's multi-threaded timing build on every usable
                host core, with the host's core count, CPU model and memory.
  legs          (default workload) the sort-based ordering on the same graph,
                both orderings with exact k-core pruning, and both with
                approximate k-core pruning (c = 3/2), one timed run each,
                with the best density each reaches.
  check         sum of loads = T*m, the best set's size, and, at the stored
                sizes, equality with the oracle's stored results.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c3|rmat22|batch|serve|par]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """SHA-256 prefix over the sources the timed kernels are compiled from (the kernel translation unit and its
    headers); a committed PMC summary applies only while it matches."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2311_04333_amd", "csrc")
    for name in ("dsg_device.h", "dsg_internal.h", "dsg_kernels.hip"):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(workload: str, kernel: str):
    """HBM bytes per launch from committed rocprofv3 PMC summaries, if they match the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        p = json.load(f)
    if p.get("kernel_source_hash") != kernel_source_hash():
        log(f"traffic: {path} was taken on other kernel sources; reporting null")
        return None
    return p.get("hbm_bytes_per_launch")


def host_info():
    """Cores, CPU model and memory of the host the oracle runs on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    mem = None
    try:
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    mem = round(int(line.split()[1]) / 2 ** 20, 1)
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"nproc": usable, "cpu_model": model, "mem_gib": mem}


def sha(a) -> str:
    import numpy as np

    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def golden_check(g, gd, T):
    """Compare a finished run with a stored oracle result (tests/golden/*.json)."""
    import numpy as np

    loads = g.loads()
    digests, rounds = g.digests()
    dens = g.iter_densities()
    rnd, pos, _ = g.order()
    return bool([list(x[:2]) for x in dens] == gd["hist"] and [x[2] for x in dens] == gd["hist_idx"] and
                [str(d) for d in digests] == gd["digests"] and rounds == gd["rounds"] and
                list(g.best()) == gd["best"] and sha(loads.astype(np.int64)) == gd["loads_sha256"] and
                sha(g.best_mask().astype(np.uint8)) == gd["best_mask_sha256"] and
                sha(rnd.astype(np.int32)) == gd["last_round_sha256"] and
                sha(pos.astype(np.int32)) == gd["last_pos_sha256"] and int(loads.sum()) == T * (g.nnz // 2))


def read_golden(name):
    path = os.path.join(ROOT, "tests", "golden", name + ".json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3", choices=["c3", "rmat22", "batch", "serve", "par"],
                    help="c3: the 40M-vertex Chung-Lu graph, PEEL eps=1/20, T=50 (default); rmat22: one R-MAT "
                         "scale-22 graph, PEEL eps=1/10, T=20; batch: the 4096-graph batched mix; serve: Poisson "
                         "request stream through the continuous-batching server; par: Pruning-and-Refining (exact "
                         "k-core pruning) on the R-MAT scale-22 graph")
    ap.add_argument("--rates", default="100,300,1000,3000,5000", help="serve: offered request rates (req/s)")
    ap.add_argument("--requests", type=int, default=2000, help="serve: measured requests per rate (after warm-up)")
    ap.add_argument("--serve-warmup", type=int, default=200, help="serve: warm-up requests per rate (not measured)")
    ap.add_argument("--variant", default="peel", choices=["peel", "sort"])
    ap.add_argument("--select", type=int, default=-1, choices=[-1, 0, 1],
                    help="PEEL select: -1 = by size (near list from 2^23 vertices), 0 = full list, 1 = near list")
    ap.add_argument("--hub", default="auto", choices=["auto", "on", "off"],
                    help="hub order (vertices renumbered by degree inside the library): auto = from 2^22 vertices")
    ap.add_argument("--count", type=int, default=4096, help="graphs in the batched mix")
    ap.add_argument("--plain-sample", type=int, default=256, help="graphs of the mix timed on the plain path")
    ap.add_argument("--T", type=int, default=None, help="iterations per step (default: 50 for c3, 20 otherwise)")
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--no-legs", action="store_true", help="c3: skip the SORT and pruned legs")
    ap.add_argument("--cpu-iters", type=int, default=None,
                    help="single graph: oracle iterations timed for cpu_baseline (default 6 for c3 on the "
                         "sample graph, 8 for rmat22; 0 = skip)")
    ap.add_argument("--cpu-sample-n", type=int, default=4_000_000,
                    help="c3: vertices of the Chung-Lu sample graph the oracle is timed on (same generator, "
                         "exponent and mean degree as the 40M-vertex graph, degree cap scaled with n)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="batch: oracle runs of whole graphs (T iterations each) until this much CPU time (0 = skip)")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); how the path would "
              "shard over several GPUs is described, not built", file=sys.stderr)
        sys.exit(2)
    if args.T is None:
        args.T = 50 if args.workload == "c3" else 20

    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "par":
        return bench_par(args)
    return bench_graph(args)


def bench_graph(args):
    import numpy as np
    import torch

    import graphgen
    import paper_2311_04333_amd as dsg

    c3 = args.workload == "c3"
    if args.variant == "peel":
        eps = (1, 20) if c3 else (1, 10)
    else:
        eps = (0, 1)
    T = args.T
    t0 = time.time()
    if c3:
        log("generating Chung-Lu n=40M (one to two minutes)")
        offsets, adj = graphgen.config3(1)
        name = f"chunglu40m_{args.variant}"
        desc = "Chung-Lu n=40M, degree exponent 2.1, mean degree 30, degree cap 2M"
    else:
        offsets, adj = graphgen.rmat(1, args.scale, 16 << args.scale, 57, 19, 19)
        name = f"rmat{args.scale}_{args.variant}"
        desc = f"R-MAT scale {args.scale}, edge factor 16, (a,b,c,d)=(.57,.19,.19,.05)"
    n, m = len(offsets) - 1, len(adj) // 2
    log(f"generated {desc}: n={n} m={m} in {time.time() - t0:.1f}s")

    if args.copy_calib_mib > 0:
        src = torch.ones(args.copy_calib_mib << 18, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    ctx = dsg.Context(0)
    o_dev = torch.from_numpy(offsets).cuda()
    a_dev = torch.from_numpy(adj).cuda()
    torch.cuda.synchronize()
    t_create = time.perf_counter()
    g = dsg.Graph(ctx, o_dev, a_dev, t_cap=T, validate=False, hub_order=hub_arg(args))
    create_ms = 1e3 * (time.perf_counter() - t_create)
    log(f"graph created in {create_ms:.1f} ms (hub order: {g.hub_order})")
    g.set_kernel_timing(True)
    g.set_peel_select(args.select)
    near = args.select == 1 or (args.select < 0 and n >= (1 << 23))
    torch.cuda.synchronize()

    for w in range(args.warmup):
        g.reset().run(T, eps, args.variant)
        g.sync()
        log(f"warmup {w + 1}/{args.warmup}: {g.last_run_ms():.2f} ms device")

    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        g.reset().run(T, eps, args.variant)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    run_ms = g.last_run_ms()
    kern_ms, launches = g.kernel_timing()
    g.sync()

    ms_per_step = 1e3 * elapsed / max(args.steps, 1)
    value = 2.0 * m * T * args.steps / elapsed
    kernel = ("k_peel_rounds_near" if near else "k_peel_rounds") if args.variant == "peel" else "k_sweep_sort"
    # algorithmic bytes per launch of the dominant kernel, and per iteration
    if args.variant == "peel":
        alg_bytes, alg_model = 16.0 * m + 16.0 * n, "16m+16n"
        it_bytes, it_model = 16.0 * m + 32.0 * n, "16m+32n"
    else:
        alg_bytes, alg_model = 16.0 * m + 12.0 * n, "16m+12n"
        it_bytes, it_model = 16.0 * m + 88.0 * n, "16m+(16P+24)n, P=4 radix passes"
    avg_launch_s = (kern_ms / launches) / 1e3 if launches else float("nan")
    achieved = alg_bytes / avg_launch_s / 1e9
    if g.hub_order:
        name += "_hub"
    traffic = load_traffic(name, kernel)
    iter_s = elapsed / max(args.steps, 1) / T
    log(f"timed {args.steps} steps: {ms_per_step:.2f} ms/step (last run {run_ms:.2f} ms device), "
        f"{kernel}: {kern_ms / max(launches, 1):.3f} ms/launch over {launches} launches")

    check = None
    if not args.no_check:
        loads = g.loads()
        best = g.best()
        mask = g.best_mask()
        check = {"sum_loads_eq_Tm": bool(int(loads.sum()) == T * m), "best_set_size_ok": bool(mask.sum() == best[1])}
        gname = ("config3" + ("_peel" if args.variant == "peel" else "_sort")) if c3 else \
            ("config2" + ("" if args.variant == "peel" else "_sort"))
        gd = read_golden(gname)
        if gd is not None and gd["n"] == n and gd["m"] == m and gd["T"] == T and tuple(gd["eps"]) == eps \
                and gd["variant"] == args.variant:
            check["matches_oracle_golden"] = golden_check(g, gd, T)
        if not all(check.values()):
            log(f"RESULT CHECK FAILED: {check}")
    g.close()

    legs = None
    if c3 and not args.no_legs:
        legs = c3_legs(args, dsg, ctx, o_dev, a_dev, n, m, T)

    cpu = cpu_baseline_graph(args, c3, offsets, adj, n, m, T, eps)

    line = {
        "metric": "edge-visits/s per Greedy++ iteration (PaRGreedy++ peeling)" if args.variant == "peel"
        else "edge-visits/s per Greedy++ iteration (GreedySorting++)",
        "value": value,
        "unit": "edge-visits/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"{desc} (n={n}, m={m}), {args.variant} eps={eps[0]}/{eps[1]}, T={T} per step",
                   "peel_select": ("near list" if near else "full list") if args.variant == "peel" else None},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": kernel,
                     "avg_launch_ms": kern_ms / max(launches, 1), "launches": launches,
                     "alg_bytes_per_launch": alg_bytes, "alg_bytes_model": alg_model,
                     "alg_bytes_split": "the dominant kernel's share of the per-iteration bytes; the rest of the "
                                        "iteration's model is in the init and Algorithm 3 kernels (see iteration)",
                     "iteration": {"alg_bytes": it_bytes, "alg_bytes_model": it_model, "ms": iter_s * 1e3,
                                   "achieved": it_bytes / iter_s / 1e9,
                                   "frac": it_bytes / iter_s / 1e9 / HBM_PEAK_GBS}},
        "cpu_baseline": cpu,
        "setup": {"hub_order": g.hub_order, "graph_create_ms": create_ms,
                  "note": "graph creation (CSR binding, static item list and, with hub order, the degree "
                          "renumbering) runs once per graph, outside the timed steps"},
        "legs": legs,
        "check": check,
    }
    ctx.close()
    print(json.dumps(line), flush=True)


def hub_arg(args):
    """auto: the binding's size rule (hub order from 2^22 vertices)."""
    return {"auto": "auto", "on": True, "off": False}[args.hub]


def c3_legs(args, dsg, ctx, o_dev, a_dev, n, m, T):
    """The sort-based ordering on the same graph, both orderings with exact k-core pruning (Algorithm 1), and the
    approximate-pruning frameworks (PaRApxSorting++, PaRApxGreedy++): one run each after one warm-up run of one
    iteration, with the best density each reaches."""
    import torch

    out = {}
    g = dsg.Graph(ctx, o_dev, a_dev, t_cap=T, validate=False, hub_order=hub_arg(args))
    g.run(1, (0, 1), "sort")
    g.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g.reset().run(T, (0, 1), "sort")
    g.sync()
    sec = time.perf_counter() - t1
    e, v = g.best()[:2]
    rec = {"seconds": sec, "edge_visits_per_s": 2.0 * m * T / sec, "best": [e, v], "density": e / v}
    gd = read_golden("config3_sort")
    if gd is not None and gd["n"] == n and gd["T"] == T:
        rec["matches_oracle_golden"] = golden_check(g, gd, T)
    g.close()
    out["sort"] = rec
    log(f"sort leg: {sec:.2f} s for T={T} ({2.0 * m * T / sec / 1e9:.1f} G edge-visits/s), best {e}/{v}")
    ws = torch.empty(dsg.par_workspace_bytes(n, int(a_dev.numel()), T) + 256, dtype=torch.uint8, device="cuda")
    # PaRSorting++ / PaRGreedy++ (exact k-core pruning), then PaRApxSorting++ (approximate pruning only) and
    # PaRApxGreedy++ (approximate, then exact pruning), with the ratio c = 3/2 of the paper's experiments
    for name, variant, eps, prune in (("par_sort", "sort", (0, 1), "exact"), ("par_peel", "peel", (1, 20), "exact"),
                                      ("par_apx_sort", "sort", (0, 1), "apx"),
                                      ("par_apx_peel", "peel", (1, 20), "apx_exact")):
        dsg.par_run(ctx, o_dev, a_dev, 1, eps, variant, validate=False, workspace=ws, prune=prune)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r = dsg.par_run(ctx, o_dev, a_dev, T, eps, variant, validate=False, workspace=ws, prune=prune)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t1
        out[name] = {"seconds": sec, "best": list(r.best[:2]), "density": r.best[0] / r.best[1],
                     "k_max": r.kmax, "first_cut": r.sizes[0] if r.sizes else None, "last_cut": r.final_size}
        if prune != "exact":
            out[name]["apx"] = {"khat_max": r.apx_kmax, "level": r.apx_level, "cut": r.apx_size}
        log(f"{name} leg: {sec:.2f} s for T={T}, best {r.best[0]}/{r.best[1]}, k_max {r.kmax}, "
            f"cuts {r.sizes[0] if r.sizes else None} -> {r.final_size}")
    del ws
    return out


def cpu_baseline_graph(args, c3, offsets, adj, n, m, T, eps):
    """The oracle, single thread, on a bounded sample of the workload.  For the 40M-vertex graph one oracle PEEL
    iteration takes minutes, so the sample is a smaller graph from the same generator with the same exponent and
    mean degree (degree cap scaled with n); for R-MAT scale 22 it is the first iterations of the same run."""
    iters = args.cpu_iters if args.cpu_iters is not None else (6 if c3 else 8)
    if iters <= 0:
        return None
    import graphgen
    import oracle

    if c3:
        ns = args.cpu_sample_n
        o, a = graphgen.config3(1, n=ns, max_deg=2_000_000.0 * ns / 40_000_000)
        sample = (f"Chung-Lu n={len(o) - 1} (m={len(a) // 2}; same generator, exponent and mean degree as the timed "
                  f"graph, degree cap scaled with n), {iters} {args.variant} iteration(s)")
    else:
        o, a = offsets, adj
        sample = f"first {iters} of the {T} iterations of the same run (same graph)"
    t1 = time.perf_counter()
    ref = oracle.run(o, a, iters, args.variant, eps)
    cpu_s = time.perf_counter() - t1
    log(f"cpu oracle: {iters} iterations in {cpu_s:.1f}s")
    info = host_info()
    # the multi-threaded timing build of the same iterations on every usable host core, checked equal to the oracle
    cores = info["nproc"] or 1
    t1 = time.perf_counter()
    par = oracle.run_omp(o, a, iters, args.variant, eps, threads=cores)
    par_s = time.perf_counter() - t1
    same = par.hist == ref.hist and par.digests == ref.digests and list(par.best) == list(ref.best)
    log(f"cpu timing build: {iters} iterations in {par_s:.1f}s on {cores} threads (equal to the oracle: {same})")
    return {"value": 2.0 * (len(a) // 2) * iters / cpu_s, "unit": "edge-visits/s", "cores": 1, "kind": "oracle",
            "sample": f"{sample}, single thread, {cpu_s:.1f} s", "host": info,
            "all_cores": {"value": 2.0 * (len(a) // 2) * iters / par_s, "unit": "edge-visits/s", "cores": cores,
                          "kind": "OpenMP timing build of the oracle (oracle/timing_omp.c), same sample",
                          "seconds": par_s, "equals_oracle": bool(same)}}


def bench_batch(args):
    """The batched workload: --count graphs of the mix (n log-uniform 100..200k, mean degree 4..64; ER, R-MAT,
    ER + planted block), PEEL eps=1/10, T=20, in one persistent launch.  This is compared with the plain path
    (one dsg_run per graph, back to back) on a systematic sample of the same graphs."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    import torch

    import graphgen
    import paper_2311_04333_amd as dsg
    from paper_2311_04333_amd import autotune

    T, eps = args.T, (1, 10)
    t0 = time.time()
    workers = min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(workers) as ex:
        graphs = list(ex.map(lambda i: graphgen.mix_graph(1, i), range(args.count)))
    n_tot = sum(len(o) - 1 for o, _ in graphs)
    m_tot = sum(len(a) // 2 for _, a in graphs)
    log(f"generated {args.count} graphs (n={n_tot}, m={m_tot}) in {time.time() - t0:.1f}s with {workers} threads")
    ctx = dsg.Context(0)
    cfg, bpc, timings = autotune.tune_batch(ctx, graphs, T=2, eps=eps, log=log)
    log(f"autotuned schedule: cfg={cfg} blocks/CU={bpc}")
    t1 = time.time()
    b = dsg.Batch(ctx, graphs, T=T, eps=eps, t_cap=T, validate=False).set_config(cfg, bpc)
    torch.cuda.synchronize()
    log(f"batch resident in HBM in {time.time() - t1:.1f}s")
    for w in range(args.warmup):
        b.reset().run()
        log(f"warmup {w + 1}: {b.last_run_ms():.1f} ms")
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for _ in range(args.steps):
        b.reset().run()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - ts
    kern_ms = b.last_run_ms()
    graphs_per_s = args.count * args.steps / elapsed
    ev_per_s = 2.0 * m_tot * T * args.steps / elapsed
    alg_bytes = sum(16.0 * (len(a) // 2) + 16.0 * (len(o) - 1) for o, a in graphs) * T
    achieved = alg_bytes / (kern_ms / 1e3) / 1e9
    log(f"batched: {elapsed / args.steps * 1e3:.1f} ms/step, {graphs_per_s:.1f} graphs/s, {ev_per_s / 1e9:.2f} G edge-visits/s")

    # plain path on a systematic sample: one dsg_run per graph, enqueued back to back
    step = max(1, args.count // args.plain_sample)
    idx = list(range(0, args.count, step))[:args.plain_sample]
    plain = [dsg.Graph(ctx, *graphs[i], t_cap=T, validate=False) for i in idx]
    for g in plain[:4]:
        g.reset().run(T, eps, "peel")
    torch.cuda.synchronize()
    tp = time.perf_counter()
    for g in plain:
        g.reset().run(T, eps, "peel")
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - tp
    m_samp = sum(len(graphs[i][1]) // 2 for i in idx)
    plain_gps = len(idx) / plain_s
    plain_evs = 2.0 * m_samp * T / plain_s
    # bit-equality of batched and alone results on the sample
    same = all(np.array_equal(b.loads(i), g.loads()) and b.best(i) == g.best() and b.digests(i) == g.digests()
               for i, g in zip(idx[:32], plain[:32]))
    log(f"plain: {len(idx)} graphs in {plain_s:.2f}s = {plain_gps:.1f} graphs/s; batched/plain = "
        f"{graphs_per_s / plain_gps:.1f}x; alone == batched on {min(32, len(idx))} graphs: {same}")

    cpu = None
    if args.cpu_seconds > 0:
        import oracle

        # whole graphs of the same systematic sample, T iterations each, until the time budget is spent
        tc = time.perf_counter()
        done, m_c = 0, 0
        for i in idx:
            oracle.run(*graphs[i], T, "peel", eps)
            done += 1
            m_c += len(graphs[i][1]) // 2
            if time.perf_counter() - tc >= args.cpu_seconds:
                break
        cpu_s = time.perf_counter() - tc
        cpu = {"value": 2.0 * m_c * T / cpu_s, "unit": "edge-visits/s", "cores": 1, "kind": "oracle",
               "sample": f"the first {done} graphs of the plain-path sample, T={T} each, in {cpu_s:.1f} s: "
                         f"{done / cpu_s:.2f} graphs/s"}
        log(f"cpu oracle: {done} graphs x {T} iterations in {cpu_s:.1f}s")
    line = {
        "metric": "graphs/s, batched persistent launch (edge-visits/s beside it); batched vs plain",
        "value": graphs_per_s,
        "unit": "graphs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"{args.count} mixed graphs (n={n_tot}, m={m_tot}), PEEL eps=1/10, T={T}",
                   "schedule": {"cfg": cfg, "blocks_per_cu": bpc, "autotune_ms": timings}},
        "edge_visits_per_s": ev_per_s,
        "plain": {"graphs_per_s": plain_gps, "edge_visits_per_s": plain_evs, "sample_graphs": len(idx)},
        "batched_over_plain": graphs_per_s / plain_gps,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "k_batch_peel",
                     "avg_launch_ms": kern_ms, "alg_bytes_per_launch": alg_bytes},
        "cpu_baseline": cpu,
        "check": {"alone_equals_batched": bool(same)},
    }
    print(json.dumps(line), flush=True)


def bench_serve(args):
    """Serving: Poisson arrivals at each offered rate for a fixed window.  98% of requests draw a graph from the
    batched mix (a pool of 256 resident graphs) and 2% draw an R-MAT scale-20 graph.  T ~ U{5..50} and eps is 1/20
    or 1/10 with equal probability.  Requests are admitted under the HBM budget (min(200 GB, 80% of free HBM)).
    Per rate: served graphs/s = completions during the last three quarters of the arrival window divided by that
    time (the offered rate when the server keeps up, its capacity when it saturates); p50/p99 latency (arrival to
    result fetched on the host) over every request, after the stream drains.  The plain baseline runs a sample of
    the same requests one at a time through the single-graph path."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    import torch

    import graphgen
    import paper_2311_04333_amd as dsg

    rng = np.random.default_rng(2026)
    workers = min(16, os.cpu_count() or 1)
    t0 = time.time()
    with ThreadPoolExecutor(workers) as ex:
        mix = list(ex.map(lambda i: graphgen.mix_graph(7, i), range(256)))
        big = list(ex.map(lambda i: graphgen.rmat(100 + i, 20, 16 << 20), range(4)))
    log(f"request pool: 256 mix graphs + 4 R-MAT scale-20 graphs in {time.time() - t0:.1f}s")
    ctx = dsg.Context(0)
    free, _ = torch.cuda.mem_get_info()
    budget = int(min(200e9, 0.8 * free))
    srv = dsg.Server(ctx, budget, ring_size=16384)
    gids_mix = [srv.register(o, a, validate=False) for o, a in mix]
    gids_big = [srv.register(o, a, validate=False) for o, a in big]
    graphs = {g: ga for g, ga in zip(gids_mix + gids_big, mix + big)}
    from paper_2311_04333_amd import autotune

    cfg, bpc, _ = autotune.tune_batch(ctx, mix[:128], T=2, log=log)
    log(f"serving schedule (autotuned on the mix): cfg={cfg} blocks/CU={bpc}")
    srv.start(cfg=cfg, blocks_per_cu=bpc, idle_seconds=60, max_seconds=1100)
    results = []
    served_sample = {}
    try:
        for rate in [float(r) for r in args.rates.split(",")]:
            N = args.serve_warmup + args.requests
            arrivals = np.cumsum(rng.exponential(1.0 / rate, N))
            W = float(arrivals[-1])
            plan = [((gids_big[rng.integers(4)] if rng.random() < 0.02 else gids_mix[rng.integers(256)]),
                     int(rng.integers(5, 51)), (1, 20) if rng.random() < 0.5 else (1, 10)) for _ in range(N)]
            lat = np.zeros(N)
            tdone = np.zeros(N)
            ticket_of = {}
            start = time.perf_counter()
            i, done_cnt, last_done = 0, 0, 0.0
            while done_cnt < N:
                now = time.perf_counter() - start
                while i < N and arrivals[i] <= now:
                    t = srv.submit_registered(*plan[i])
                    if t is None:
                        break  # pool or ring full: retry once results are released
                    ticket_of[t] = i
                    i += 1
                for t in srv.poll():
                    j = ticket_of.pop(t)
                    res = srv.fetch(t)
                    srv.release(t)
                    last_done = time.perf_counter() - start
                    lat[j] = last_done - arrivals[j]
                    tdone[j] = last_done
                    done_cnt += 1
                    if len(served_sample) < 48 and plan[j] not in served_sample:
                        served_sample[plan[j]] = res
                if time.perf_counter() - start > 240:
                    raise RuntimeError(f"rate {rate}: stream did not drain in 240 s ({done_cnt}/{N} done)")
            # measured: the requests after the warm-up ones; throughput over the span of their arrivals
            meas = np.arange(args.serve_warmup, N)
            w0, w1 = float(arrivals[args.serve_warmup]), W
            thr = float(np.count_nonzero((tdone > w0) & (tdone <= w1))) / max(w1 - w0, 1e-9)
            small = np.array([plan[j][0] not in gids_big for j in meas])
            lm = lat[meas]
            rec = {"rate": rate, "requests": int(len(meas)), "warmup_requests": args.serve_warmup,
                   "arrival_span_s": W, "graphs_per_s": thr, "drained_s": last_done,
                   "p50_ms": float(np.percentile(lm, 50) * 1e3),
                   "p99_ms": float(np.percentile(lm, 99) * 1e3),
                   "p99_small_ms": float(np.percentile(lm[small], 99) * 1e3) if small.any() else None}
            results.append(rec)
            log(f"rate {rate:6.0f}/s ({N} requests): {thr:8.1f} graphs/s served, p50 {rec['p50_ms']:.1f} ms, "
                f"p99 {rec['p99_ms']:.1f} ms (p99 without the R-MAT-20 requests {rec['p99_small_ms']:.1f} ms), "
                f"drained after {last_done:.1f} s")
    finally:
        srv.stop()
    # plain: the same kind of requests one at a time through the single-graph path
    plan = list(served_sample.keys())
    tp = time.perf_counter()
    same = True
    for gid, T, eps in plan:
        o, a = graphs[gid]
        g = dsg.Graph(ctx, o, a, t_cap=T, validate=False).run(T, eps, "peel")
        dens = g.iter_densities()
        res = served_sample[(gid, T, eps)]
        same = same and g.best() == res["best"] and [(e, v) for e, v, _ in dens] == res["hist"] and \
            g.digests()[0] == res["digests"]
        g.close()
    plain_s = time.perf_counter() - tp
    plain_gps = len(plan) / plain_s
    best = max(results, key=lambda r: r["graphs_per_s"])
    log(f"plain: {len(plan)} requests in {plain_s:.2f}s = {plain_gps:.1f} graphs/s; served/plain = "
        f"{best['graphs_per_s'] / plain_gps:.1f}x; alone == served: {same}")
    line = {
        "metric": "served graphs/s under a Poisson request stream (continuous batching), p50/p99 latency",
        "value": best["graphs_per_s"],
        "unit": "graphs/s",
        "n_gpus": 1,
        "steps": len(results),
        "warmup": 0,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"Poisson stream: 98% batched-mix graphs, 2% R-MAT scale 20; T~U{{5..50}}, "
                               f"eps in {{1/20, 1/10}}; HBM budget {budget / 1e9:.0f} GB; {args.requests} measured "
                               f"requests per rate after {args.serve_warmup} warm-up ones; schedule cfg={cfg} "
                               f"blocks/CU={bpc}"},
        "rates": results,
        "plain": {"graphs_per_s": plain_gps, "requests": len(plan)},
        "served_over_plain": best["graphs_per_s"] / plain_gps,
        "check": {"alone_equals_served": bool(same)},
    }
    print(json.dumps(line), flush=True)


def bench_par(args):
    """Pruning-and-Refining (Algorithm 1) with exact k-core pruning and PEEL eps = 1/10 refinement, T iterations, on
    the R-MAT graph.  A step is one whole dsg_par_run: Coreness (a PEEL pass with zero loads and eps = 0 over the
    input), the cut to the ceil(k_max/2)-core, T refinements and the re-cuts.  The line gives the time per step
    (lower is better) beside the unpruned refinement (T PEEL iterations on the input graph) timed in the same
    process, and the CPU oracle running the same framework."""
    import numpy as np
    import torch

    import graphgen
    import paper_2311_04333_amd as dsg

    T, eps = args.T, (1, 10)
    offsets, adj = graphgen.rmat(1, args.scale, 16 << args.scale, 57, 19, 19)
    n, m = len(offsets) - 1, len(adj) // 2
    ctx = dsg.Context(0)
    o_dev = torch.from_numpy(offsets).cuda()
    a_dev = torch.from_numpy(adj).cuda()
    ws = torch.empty(dsg.par_workspace_bytes(n, len(adj), T) + 256, dtype=torch.uint8, device="cuda")
    for w in range(max(args.warmup, 1)):
        r = dsg.par_run(ctx, o_dev, a_dev, T, eps, "peel", validate=False, workspace=ws)
    log(f"par: k_max={r.kmax}, first cut {r.sizes[0] if r.sizes else None}, last {r.final_size}, best {r.best}, "
        f"prunes after the first {r.prunes}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = dsg.par_run(ctx, o_dev, a_dev, T, eps, "peel", validate=False, workspace=ws)
    torch.cuda.synchronize()
    par_ms = 1e3 * (time.perf_counter() - t0) / args.steps
    del ws
    # the unpruned refinement, and the Coreness pass alone (the dominant kernel of a par step)
    g = dsg.Graph(ctx, o_dev, a_dev, t_cap=T, validate=False)
    g.set_kernel_timing(True)
    g.reset().run(T, eps, "peel")
    g.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g.reset().run(T, eps, "peel")
    g.sync()
    plain_ms = 1e3 * (time.perf_counter() - t1)
    g.close()
    _, kmax, core_rounds, core_ms = dsg.coreness(ctx, o_dev, a_dev, validate=False, timed=True)
    alg_bytes = 16.0 * m + 16.0 * n
    achieved = alg_bytes / (core_ms / 1e3) / 1e9 if core_ms > 0 else None
    log(f"par: {par_ms:.1f} ms per step; unpruned refinement {plain_ms:.1f} ms; Coreness round loop {core_ms:.2f} ms "
        f"({core_rounds} rounds)")
    check = None
    cpu = None
    if args.cpu_iters is None or args.cpu_iters > 0:
        # the CPU-baseline leg: the oracle's run of the whole framework, whose
        # result also serves as the check (no oracle run without this leg)
        from oracle import prune

        t2 = time.perf_counter()
        ref = prune.par_run(offsets, adj, T, "peel", eps)
        cpu_s = time.perf_counter() - t2
        check = {"matches_oracle": bool(ref.best == r.best and ref.hist == r.hist and ref.sizes == r.sizes and
                                        ref.kmax == r.kmax and np.array_equal(ref.best_mask, r.best_mask))}
        cpu = {"value": cpu_s * 1e3, "unit": "ms", "cores": 1, "kind": "oracle",
               "sample": f"the whole framework on the same graph (T={T}), single thread"}
    line = {
        "metric": "PaRGreedy++ time (Coreness + k-core cuts + T refinements) vs the unpruned refinement",
        "value": par_ms,
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": max(args.warmup, 1),
        "ms_per_step": par_ms,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"R-MAT scale {args.scale} (n={n}, m={m}), PEEL eps=1/10 refinement, T={T}, exact "
                               f"k-core pruning"},
        "unpruned_ms": plain_ms,
        "speedup_vs_unpruned": plain_ms / par_ms,
        "k_max": r.kmax,
        "cuts": {"first": r.sizes[0] if r.sizes else None, "last": r.final_size, "prunes_after_first": r.prunes},
        "best": r.best,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS if achieved else None, "traffic": None,
                     "kernel": "k_peel_rounds<true> (the Coreness pass: zero loads, eps = 0, monotone thresholds, "
                               "whole input graph)",
                     "avg_launch_ms": core_ms, "rounds": core_rounds, "alg_bytes_per_launch": alg_bytes},
        "cpu_baseline": cpu,
        "check": check,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
