#!/usr/bin/env python
"""Benchmark: Greedy++ peeling (PaRGreedy++ ordering) on one MI355X.

Workload: R-MAT scale 22 with edge factor 16 and (a,b,c,d) = (.57,.19,.19,.05).
After symmetrising and deduplicating it has n = 4,194,304 vertices and
m = 64,156,259 edges.  The run is round-synchronous peeling with
eps = 1/10 for T = 20 iterations.  One step is one full run of the hot path:
reset the state, then 20 iterations.  Each iteration does init, the round
loop with its sweeps, the sort by round, Algorithm 3, and the load and best
updates.  The graph is resident in HBM before timing starts.

Metric: edge-visits/s = 2m * T * steps / wall time of the timed steps.

Also printed, on the same JSON line:
  roofline      the dominant kernel (the persistent round loop).  Its
                average launch time comes from HIP events recorded on the
                library's stream during the timed steps.  Its algorithmic
                bytes per launch are 16m + 16n: each CSR entry read once plus
                one 4-byte neighbour-state access, and four int32 arrays of
                length n.  These are divided by that time and compared with
                8 TB/s.
  cpu_baseline  the CPU oracle (single thread) timed on a bounded sample of
                the same workload: the first iterations of the same run.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--variant peel|sort]
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
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2311_04333_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(workload: str, kernel: str, launches_bytes_alg: float):
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--variant", default="peel", choices=["peel", "sort"])
    ap.add_argument("--T", type=int, default=20)
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--cpu-iters", type=int, default=2, help="oracle iterations timed for cpu_baseline (0 = skip)")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding is a design, not an implementation", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import graphgen
    import paper_2311_04333_amd as dsg

    eps = (1, 10) if args.variant == "peel" else (0, 1)
    T = args.T
    t0 = time.time()
    offsets, adj = graphgen.rmat(1, args.scale, 16 << args.scale, 57, 19, 19)
    n, m = len(offsets) - 1, len(adj) // 2
    workload = f"rmat{args.scale}_{args.variant}"
    log(f"generated R-MAT scale {args.scale}: n={n} m={m} in {time.time() - t0:.1f}s")

    if args.copy_calib_mib > 0:
        src = torch.ones(args.copy_calib_mib << 18, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    ctx = dsg.Context(0)
    g = dsg.Graph(ctx, offsets, adj, t_cap=T)
    g.set_kernel_timing(True)
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
    edge_visits = 2.0 * m * T * args.steps
    value = edge_visits / elapsed
    kernel = "k_peel_rounds" if args.variant == "peel" else "k_sweep_sort"
    # algorithmic bytes per launch of the dominant kernel
    if args.variant == "peel":
        alg_bytes = 16.0 * m + 16.0 * n
    else:
        alg_bytes = 16.0 * m + 12.0 * n
    avg_launch_s = (kern_ms / launches) / 1e3 if launches else float("nan")
    achieved = alg_bytes / avg_launch_s / 1e9
    traffic = load_traffic(workload, kernel, alg_bytes)
    log(f"timed {args.steps} steps: {ms_per_step:.2f} ms/step (last run {run_ms:.2f} ms device), "
        f"{kernel}: {kern_ms / max(launches, 1):.3f} ms/launch over {launches} launches")

    check = None
    if not args.no_check:
        loads = g.loads()
        best = g.best()
        mask = g.best_mask()
        ok = int(loads.sum()) == T * m and int(mask.sum()) == best[1]
        check = {"sum_loads_eq_Tm": bool(int(loads.sum()) == T * m), "best_set_size_ok": bool(mask.sum() == best[1])}
        golden = os.path.join(ROOT, "tests", "golden", f"config2{'' if args.variant == 'peel' else '_sort'}.json")
        if args.scale == 22 and T == 20 and os.path.exists(golden):
            with open(golden) as f:
                gd = json.load(f)
            digests, rounds = g.digests()
            dens = g.iter_densities()
            match = ([list(x[:2]) for x in dens] == gd["hist"] and [str(d) for d in digests] == gd["digests"] and
                     rounds == gd["rounds"] and list(best) == gd["best"] and
                     hashlib.sha256(loads.astype(np.int64).tobytes()).hexdigest() == gd["loads_sha256"])
            check["matches_oracle_golden"] = bool(match)
            ok = ok and match
        if not ok:
            log(f"RESULT CHECK FAILED: {check}")

    cpu = None
    if args.cpu_iters > 0:
        import oracle

        t1 = time.perf_counter()
        oracle.run(offsets, adj, args.cpu_iters, args.variant, eps)
        cpu_s = time.perf_counter() - t1
        cpu = {"value": 2.0 * m * args.cpu_iters / cpu_s, "unit": "edge-visits/s", "cores": 1, "kind": "oracle",
               "sample": f"first {args.cpu_iters} of the {T} iterations of the same run (same graph, single thread, "
                         f"{cpu_s:.1f} s)"}
        log(f"cpu oracle: {args.cpu_iters} iterations in {cpu_s:.1f}s")

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
        "config": {"workload": f"R-MAT scale {args.scale} (n={n}, m={m}), {args.variant} "
                               f"eps={eps[0]}/{eps[1]}, T={T} per step"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": kernel,
                     "avg_launch_ms": kern_ms / max(launches, 1), "alg_bytes_per_launch": alg_bytes},
        "cpu_baseline": cpu,
        "check": check,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
