"""Shared helpers for the GPU parity tests: run the HIP path, run the oracle, compare."""
from __future__ import annotations

import hashlib
import sys

import numpy as np

import oracle


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def sha(arr) -> str:
    return hashlib.sha256(np.ascontiguousarray(arr).tobytes()).hexdigest()


def assert_same(g, ref: oracle.State, what: str = "", check_order: bool = True):
    """Bit-exact comparison of every output of the GPU graph with the oracle state."""
    loads = g.loads()
    assert np.array_equal(loads, ref.loads), f"{what}: loads differ at {np.flatnonzero(loads != ref.loads)[:10]}"
    dens = g.iter_densities()
    assert [(e, v) for e, v, _ in dens] == ref.hist, f"{what}: per-iteration densities differ"
    assert [i for _, _, i in dens] == ref.hist_idx, f"{what}: per-iteration indices differ"
    assert tuple(g.best()) == tuple(int(x) for x in ref.best), f"{what}: best {g.best()} vs {ref.best}"
    assert np.array_equal(g.best_mask(), ref.best_mask()), f"{what}: best mask differs"
    digests, rounds = g.digests()
    assert rounds == ref.rounds, f"{what}: rounds {rounds} vs {ref.rounds}"
    assert digests == ref.digests, f"{what}: order digests differ"
    if check_order and ref.last_round is not None:
        rnd, pos, nr = g.order()
        assert np.array_equal(rnd, ref.last_round), f"{what}: last-iteration rounds differ"
        assert np.array_equal(pos, ref.last_pos), f"{what}: last-iteration positions differ"
        assert nr == ref.rounds[-1]


def bad_csrs():
    """Broken CSRs, one per property that validation checks."""
    import graphgen

    good_o, good_a = graphgen.from_edges(4, [(0, 1), (1, 2), (2, 3)])
    # a larger graph with one entry dropped from the middle of a hub row: the
    # asymmetry sits many 4096-entry chunks in, past runs of empty rows
    o, a = graphgen.rmat(5, 14, 16 << 14)
    v = int(np.argmax(np.diff(o)))
    x = int(o[v]) + (int(o[v + 1]) - int(o[v])) // 2
    o2 = o.copy()
    o2[v + 1:] -= 1
    return {
        "asymmetric": (good_o, np.array([1, 0, 2, 1, 3, 1], np.int32)),
        "self_loop": (np.array([0, 1, 2], np.int32), np.array([0, 1], np.int32)),
        "unsorted": (np.array([0, 2, 3, 4], np.int32), np.array([2, 1, 0, 0], np.int32)),
        "out_of_range": (good_o, np.array([1, 0, 2, 1, 3, 9], np.int32)),
        "offsets_end": (np.array([0, 1, 3, 5, 5], np.int32), good_a),
        "hub_row_hole": (o2, np.delete(a, x)),
    }
