"""The multi-threaded timing build (oracle/timing_omp.c) gives exactly the plain oracle's outputs.

The timing build only serves the CPU baseline's all-cores timing; these checks keep its numbers honest: every
output field (per-iteration densities, indices, digests, rounds, widths, loads, best, last order) equals the
plain oracle's on graphs with ties, hubs, isolated vertices and several thread counts.
"""
import numpy as np
import pytest

import graphgen
import oracle


def _graphs():
    return {
        "config1": graphgen.config1(3),
        "rmat10": graphgen.rmat(4, 10, 16 << 10),
        "chunglu_6k": graphgen.chunglu(9, 6_000, 2.1, 12.0, 600.0),
        "star": graphgen.from_edges(200, [(0, j) for j in range(1, 200)]),
        "K12": graphgen.complete(12),
        "isolated": (np.zeros(9, np.int32), np.zeros(0, np.int32)),
    }


@pytest.mark.parametrize("name", list(_graphs().keys()))
@pytest.mark.parametrize("variant,eps", [("peel", (1, 10)), ("peel", (0, 1)), ("peel_mono", (1, 20)),
                                         ("sort", (0, 1))])
@pytest.mark.parametrize("threads", [1, 3])
def test_timing_build_equals_oracle(name, variant, eps, threads):
    o, a = _graphs()[name]
    ref = oracle.run(o, a, 5, variant, eps)
    got = oracle.run_omp(o, a, 3, variant, eps, threads=threads)
    got = oracle.run_omp(o, a, 2, variant, eps, state=got, threads=threads)  # resume, as run does
    assert got.hist == ref.hist and got.hist_idx == ref.hist_idx
    assert got.digests == ref.digests and got.rounds == ref.rounds and got.width == ref.width
    assert np.array_equal(got.loads, ref.loads)
    assert list(got.best) == list(ref.best)
    assert np.array_equal(got.best_mask(), ref.best_mask())
    assert np.array_equal(got.last_pos, ref.last_pos) and np.array_equal(got.last_round, ref.last_round)
