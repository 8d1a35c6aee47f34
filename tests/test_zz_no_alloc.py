"""dsg_par_run_noalloc (Pruning-and-Refining on the library's static device scratch) against dsg_par_run with a
caller workspace, bit for bit, on two calls in a row: a larger graph, then a smaller one, so the second call runs on
scratch that the first one left dirty.  Also the host-side refusal of a graph that needs more scratch than there is.
"""
import ctypes

import numpy as np
import pytest

import graphgen
from gpu_helpers import log

pytestmark = pytest.mark.gpu


def assert_same(g, r, what):
    assert g.kmax == r.kmax, f"{what}: kmax {g.kmax} vs {r.kmax}"
    assert np.array_equal(g.core, r.core), f"{what}: core numbers differ"
    assert g.sizes == r.sizes, f"{what}: refined graph sizes differ"
    assert g.levels == r.levels, f"{what}: levels differ"
    assert g.hist == r.hist, f"{what}: per-iteration densities differ"
    assert g.hist_idx == r.hist_idx, f"{what}: per-iteration indices differ"
    assert g.best == r.best, f"{what}: best {g.best} vs {r.best}"
    assert np.array_equal(g.best_mask, r.best_mask), f"{what}: best set differs"
    assert (g.level, g.prunes, g.final_size) == (r.level, r.prunes, r.final_size), f"{what}: level/prunes/size"


def test_noalloc_equals_workspace_path_twice():
    import torch

    import paper_2311_04333_amd as dsg

    assert torch.cuda.is_available()
    ctx = dsg.Context(0)
    cases = [
        ("rmat16", graphgen.rmat(5, 16, 16 << 16), 8, (1, 10), "peel"),
        ("config1", graphgen.config1(2), 6, (0, 1), "sort"),
    ]
    for name, (o, a), T, eps, variant in cases:
        od = torch.from_numpy(o).cuda()
        ad = torch.from_numpy(a).cuda()
        need = dsg.par_workspace_bytes(len(o) - 1, len(a), T)
        assert need <= dsg.NOALLOC_SCRATCH_BYTES, name
        log(f"noalloc case={name} n={len(o) - 1} nnz={len(a)} T={T} variant={variant} eps={eps}")
        ref = dsg.par_run(ctx, od, ad, T, eps, variant)
        got = dsg.par_run_noalloc(ctx, od, ad, T, eps, variant)
        torch.cuda.synchronize()
        assert_same(got, ref, name)
    ctx.close()


def test_noalloc_refuses_oversized_graph():
    """A graph whose scratch would exceed the static array is refused on the host before any device work."""
    import torch

    import paper_2311_04333_amd as dsg

    assert torch.cuda.is_available()
    ctx = dsg.Context(0)
    lib = dsg.library()
    n, nnz, T = 1 << 20, 1 << 25, 50
    assert dsg.par_workspace_bytes(n, nnz, T) > dsg.NOALLOC_SCRATCH_BYTES
    res = dsg._ParResultC()
    buf = torch.zeros(2, dtype=torch.int32, device="cuda")  # never read: the size check comes first
    ptr = ctypes.c_void_p(buf.data_ptr())
    st = lib.dsg_par_run_noalloc(ctx.handle, n, nnz, ptr, ptr, T, 1, 10, dsg.VARIANTS["peel"], 0,
                                 ctypes.addressof(res), *([None] * 8))
    assert st == -2, st  # DSG_ENOMEM
    assert b"static scratch" in lib.dsg_last_error()
    ctx.close()
