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
