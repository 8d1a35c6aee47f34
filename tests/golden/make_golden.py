"""Write the stored expected values for the full-size parity checks.

Calls only the CPU oracle (oracle/) on graphs from the seeded generators
(graphgen/); nothing here touches the GPU path.  Usage:

    python tests/golden/make_golden.py config2       # R-MAT scale 22, PEEL eps=1/10, T=20 (~2 min)
    python tests/golden/make_golden.py config3_sort  # Chung-Lu n=40M, SORT, T=50
    python tests/golden/make_golden.py config3_peel  # Chung-Lu n=40M, PEEL eps=1/20, T=50
    python tests/golden/make_golden.py mix_large     # largest graphs of the 4096-graph batched mix, PEEL eps=1/10, T=20

Each file records the workload, a hash of the generated CSR (so a generator
change is caught separately from a peeling mismatch), the per-iteration
(edges, vertices, index), order digests and round counts, the best subgraph,
and SHA-256 hashes of the final loads (int64) and of the best-set mask (uint8).
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import graphgen  # noqa: E402
import oracle  # noqa: E402


def sha(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


WORKLOADS = {
    "config2": dict(gen=lambda: graphgen.config2(1), T=20, variant="peel", eps=(1, 10),
                    desc="R-MAT scale 22, edge factor 16, (a,b,c,d)=(.57,.19,.19,.05), seed 1; PEEL eps=1/10, T=20"),
    "config2_sort": dict(gen=lambda: graphgen.config2(1), T=20, variant="sort", eps=(0, 1),
                         desc="R-MAT scale 22 as above; SORT, T=20"),
    "config3_sort": dict(gen=lambda: graphgen.config3(1), T=50, variant="sort", eps=(0, 1),
                         desc="Chung-Lu n=40M, gamma 2.1, mean weight 30, weight cap 2M, seed 1; SORT, T=50"),
    "config3_peel": dict(gen=lambda: graphgen.config3(1), T=50, variant="peel", eps=(1, 20),
                         desc="Chung-Lu n=40M as above; PEEL eps=1/20, T=50"),
}


def mix_large_indices(seed: int = 1, count: int = 4096):
    """The 8 largest graphs of the batched mix (by expected edge count: all are ER + planted block), then the two
    largest ER and the two largest R-MAT graphs, so that every kind of the mix is covered at its largest size."""
    rows = []
    for i in range(count):
        kind, n, d, _ = graphgen.mix_params(seed, i)
        block = max(2, n // 20)
        m = n * d / 2 + (0.3 * block * (block - 1) / 2 if kind == 2 else 0.0)
        rows.append((m, i, kind))
    rows.sort(reverse=True)
    top = [i for _, i, _ in rows[:8]]
    for kind in (0, 1):
        top += [i for _, i, k in rows if k == kind][:2]
    return top


def state_record(o, a, st, T, variant, eps):
    return {
        "n": len(o) - 1,
        "m": len(a) // 2,
        "csr_sha256": sha(o) + sha(a),
        "T": T,
        "variant": variant,
        "eps": list(eps),
        "hist": [list(h) for h in st.hist],
        "hist_idx": st.hist_idx,
        "digests": [str(d) for d in st.digests],
        "rounds": st.rounds,
        "best": [int(x) for x in st.best],
        "loads_sha256": sha(st.loads.astype(np.int64)),
        "loads_sum": int(st.loads.sum()),
        "best_mask_sha256": sha(st.best_mask().astype(np.uint8)),
        "last_round_sha256": sha(st.last_round.astype(np.int32)),
        "last_pos_sha256": sha(st.last_pos.astype(np.int32)),
    }


def make_mix_large():
    t0 = time.time()
    graphs = []
    for i in mix_large_indices():
        o, a = graphgen.mix_graph(1, i)
        t1 = time.time()
        st = oracle.run(o, a, 20, "peel", (1, 10))
        rec = state_record(o, a, st, 20, "peel", (1, 10))
        rec["mix_index"] = i
        rec["kind"] = graphgen.mix_params(1, i)[0]
        graphs.append(rec)
        print(f"  mix graph {i}: n={rec['n']} m={rec['m']} in {time.time() - t1:.1f}s best={rec['best']}", flush=True)
    out = {"workload": "mix_large",
           "description": "graphs of the batched mix (seed 1): the 8 largest, then the 2 largest ER and the 2 largest "
                          "R-MAT graphs; PEEL eps=1/10, T=20 each",
           "graphs": graphs, "oracle_seconds": round(time.time() - t0, 1)}
    path = os.path.join(HERE, "mix_large.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


def make(name: str):
    if name == "mix_large":
        return make_mix_large()
    w = WORKLOADS[name]
    t0 = time.time()
    o, a = w["gen"]()
    print(f"{name}: generated n={len(o) - 1} m={len(a) // 2} in {time.time() - t0:.1f}s", flush=True)
    st = None
    for t in range(w["T"]):
        t1 = time.time()
        st = oracle.run(o, a, 1, w["variant"], w["eps"], state=st)
        print(f"  iteration {t + 1}/{w['T']}: {time.time() - t1:.1f}s rounds={st.rounds[-1]} hist={st.hist[-1]}",
              flush=True)
    out = {
        "workload": name,
        "description": w["desc"],
        "n": len(o) - 1,
        "m": len(a) // 2,
        "csr_sha256": sha(o) + sha(a),
        "T": w["T"],
        "variant": w["variant"],
        "eps": list(w["eps"]),
        "hist": [list(h) for h in st.hist],
        "hist_idx": st.hist_idx,
        "digests": [str(d) for d in st.digests],
        "rounds": st.rounds,
        "best": [int(x) for x in st.best],
        "loads_sha256": sha(st.loads.astype(np.int64)),
        "loads_sum": int(st.loads.sum()),
        "best_mask_sha256": sha(st.best_mask().astype(np.uint8)),
        "last_round_sha256": sha(st.last_round.astype(np.int32)),
        "last_pos_sha256": sha(st.last_pos.astype(np.int32)),
        "oracle_seconds": round(time.time() - t0, 1),
    }
    path = os.path.join(HERE, f"{name}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    for name in sys.argv[1:] or ["config2"]:
        make(name)
