"""Planted mistakes in the oracle must be caught by its pins.

Each mutant is a copy of oracle/greedypp_oracle.c with one plausible mistake
written into it: a wrong comparison, a dropped term, a wrong index or a
transposed operand.  The copy is compiled to a temporary library, and the
full pin suite (tests/pins.py) runs against it.  The test passes when at
least one pin rejects the mutant.  The mistakes go into the oracle copy, on
the CPU, never into the GPU path.
"""
import os
import subprocess

import pytest

import oracle
from pins import ALL_PINS

SRC = os.path.join(os.path.dirname(oracle.__file__), "greedypp_oracle.c")

MUTANTS = [
    ("seq_tie_to_higher_id",
     "if (best < 0 || load[v] + deg[v] < load[best] + deg[best]) best = v;",
     "if (best < 0 || load[v] + deg[v] <= load[best] + deg[best]) best = v;"),
    ("seq_decrement_twice", "if (alive[adj[k]]) deg[adj[k]]--;", "if (alive[adj[k]]) deg[adj[k]] -= 2;"),
    ("peel_round_max_not_min", "if (p < mn) mn = p;", "if (p > mn) mn = p;"),
    ("peel_eps_factor_wrong", "i128 lim = (i128)(eps_den + eps_num) * (i128)mn;\n        if (mono) {",
     "i128 lim = (i128)(eps_den + 2 * eps_num) * (i128)mn;\n        if (mono) {"),
    ("peel_no_delayed_decrement", "if (round[adj[e]] == -1) deg[adj[e]]--;", "if (round[adj[e]] == -2) deg[adj[e]]--;"),
    ("peel_mono_bound_not_kept", "if (mono) {\n            if (dmax > lim) lim = dmax;\n            dmax = lim;",
     "if (mono) {\n            dmax = lim;"),
    ("peel_mono_bound_unscaled", "if (mono) {\n            if (dmax > lim) lim = dmax;\n            dmax = lim;",
     "if (mono) {\n            if (dmax > lim) lim = dmax;\n            dmax = mn;"),
    ("alg3_charge_later_endpoint", "A[pos[u] < pos[v] ? pos[u] : pos[v]] += 1;",
     "A[pos[u] > pos[v] ? pos[u] : pos[v]] += 1;"),
    ("alg3_suffix_off_by_one", "run += A[i];\n        B[i] = run;", "B[i] = run;\n        run += A[i];"),
    ("alg3_size_off_by_one", "i64 e = B[i], v = n - i;", "i64 e = B[i], v = n - i + 1;"),
    ("alg3_ties_to_largest_index", "if ((i128)e * bv > (i128)be * v) {", "if ((i128)e * bv >= (i128)be * v) {"),
    ("alg3_transposed_compare", "if ((i128)e * bv > (i128)be * v) {", "if ((i128)e * v > (i128)be * bv) {"),
    ("best_update_not_strict", "if ((i128)e * best[1] > (i128)best[0] * v) {",
     "if ((i128)e * best[1] >= (i128)best[0] * v) {"),
    ("load_update_wrong_index", "i64 inc = A[last_pos[u]];", "i64 inc = A[u];"),
    ("best_snapshot_dropped", "memcpy(best_pos, last_pos, sizeof(int32_t) * (size_t)n);\n        }\n    }\n    free(A);",
     "(void)0;\n        }\n    }\n    free(A);"),
    ("sort_tie_to_higher_id", "return (x->id > y->id) - (x->id < y->id);", "return (x->id < y->id) - (x->id > y->id);"),
    ("digest_mixer_missing_increment", "z += 0x9E3779B97F4A7C15ULL;", "z += 0;"),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(name, old, new, tmp_path):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique/found"
    mutated = tmp_path / "mutant.c"
    mutated.write_text(src.replace(old, new))
    so = tmp_path / "mutant.so"
    subprocess.check_call(["gcc", "-O1", "-fPIC", "-shared", "-std=gnu11", "-o", str(so), str(mutated)])
    lib = oracle.load_library(str(so))
    caught = []
    for pin in ALL_PINS:
        try:
            pin(lib)
        except AssertionError:
            caught.append(pin.__name__)
    assert caught, f"mutant {name} passed every pin"
