"""Seeded synthetic graph generators (input side, shared by the oracle and the GPU path).

This package draws graphs only.  It holds none of the densest-subgraph
method's arithmetic, so it can be shared by the CPU oracle and the GPU path.
Every generator returns a symmetric int32 CSR ``(offsets[n+1], adj[2m])``
with strictly increasing rows and no self-loops.  Isolated vertices are kept,
because each configuration fixes n.

The workloads stand in for the paper's real graphs (the SNAP, Network
Repository, ClueWeb and WebDataCommons datasets of Section 4), which are not
available here:

* ``config1``: Erdos-Renyi n=2000, m=20000, plus a planted 50-vertex set
  whose internal pairs appear with probability 1/2.
* ``config2``: R-MAT scale 22 with edge factor 16 and (a,b,c,d) =
  (.57,.19,.19,.05), symmetrised, deduplicated and relabelled.
* ``config3``: Chung-Lu power law with n=40M, gamma=2.1, mean weight 30 and
  maximum weight 2M.
* ``mix_graph(seed, i)``: the i-th graph of the batched mix.  Its n is
  log-uniform in 100..200k, its mean degree is uniform in 4..64, and its type
  is 1/3 each ER, R-MAT, or ER with a planted block (5% of vertices, p=0.3).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB_PATH = os.path.join(_HERE, "_graphgen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile graphgen.c into _graphgen.so next to it (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    u64 = ctypes.c_uint64
    lib.gg_er_planted.restype = P
    lib.gg_er_planted.argtypes = [u64, i64, i64, i64, i64, i64]
    lib.gg_gnp.restype = P
    lib.gg_gnp.argtypes = [u64, i64, i64, i64]
    lib.gg_from_edges.restype = P
    lib.gg_from_edges.argtypes = [i64, P, P, i64]
    lib.gg_rmat.restype = P
    lib.gg_rmat.argtypes = [u64, ctypes.c_int, i64, i64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.gg_chunglu.restype = P
    lib.gg_chunglu.argtypes = [u64, i64, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int]
    lib.gg_er_block.restype = P
    lib.gg_er_block.argtypes = [u64, i64, i64, i64, i64, i64]
    lib.gg_n.restype = i64
    lib.gg_n.argtypes = [P]
    lib.gg_nnz.restype = i64
    lib.gg_nnz.argtypes = [P]
    lib.gg_error.restype = ctypes.c_char_p
    lib.gg_error.argtypes = [P]
    lib.gg_copy.restype = ctypes.c_int
    lib.gg_copy.argtypes = [P, P, P]
    lib.gg_free.restype = None
    lib.gg_free.argtypes = [P]
    lib.gg_rnd.restype = u64
    lib.gg_rnd.argtypes = [u64, u64, u64]
    _lib = lib
    return lib


def _take(handle):
    lib = _load()
    if not handle:
        raise MemoryError("graph generator returned no handle")
    try:
        n = lib.gg_n(handle)
        nnz = lib.gg_nnz(handle)
        if n <= 0 or nnz < 0:
            raise ValueError("graph generator failed: " + lib.gg_error(handle).decode())
        offsets = np.empty(n + 1, dtype=np.int32)
        adj = np.empty(max(nnz, 1), dtype=np.int32)
        if lib.gg_copy(handle, offsets.ctypes.data, adj.ctypes.data) != 0:
            raise ValueError("graph generator failed: " + lib.gg_error(handle).decode())
        return offsets, adj[:nnz]
    finally:
        lib.gg_free(handle)


def er_planted(seed: int, n: int, m: int, k: int, p_num: int, p_den: int):
    """G(n, m) with exactly m distinct pairs, plus a planted k-set with pair probability p_num/p_den."""
    return _take(_load().gg_er_planted(seed, n, m, k, p_num, p_den))


def gnp(seed: int, n: int, p_num: int, p_den: int):
    """G(n, p) over all pairs, p = p_num/p_den (small test graphs)."""
    return _take(_load().gg_gnp(seed, n, p_num, p_den))


def from_edges(n: int, edges):
    """CSR of an explicit undirected edge list; loops dropped, duplicates merged."""
    e = np.asarray(edges, dtype=np.int32).reshape(-1, 2)
    u = np.ascontiguousarray(e[:, 0])
    v = np.ascontiguousarray(e[:, 1])
    return _take(_load().gg_from_edges(n, u.ctypes.data, v.ctypes.data, len(u)))


def rmat(seed: int, scale: int, samples: int, a: int = 57, b: int = 19, c: int = 19,
         n: int | None = None, relabel: bool = True):
    """R-MAT with quadrant probabilities in hundredths (d = 100 - a - b - c)."""
    if n is None:
        n = 1 << scale
    return _take(_load().gg_rmat(seed, scale, n, samples, a, b, c, 1 if relabel else 0))


def chunglu(seed: int, n: int, gamma: float, mean_deg: float, max_deg: float, relabel: bool = True):
    """Chung-Lu with power-law weights; see graphgen.c for the weight formula."""
    return _take(_load().gg_chunglu(seed, n, gamma, mean_deg, max_deg, 1 if relabel else 0))


def er_block(seed: int, n: int, samples: int, block: int, p_num: int, p_den: int):
    """G(n, M samples, deduplicated) plus a dense block on a seeded vertex subset."""
    return _take(_load().gg_er_block(seed, n, samples, block, p_num, p_den))


# ----------------------------------------------------------------- named workloads
def complete(k: int):
    return from_edges(k, [(i, j) for i in range(k) for j in range(i + 1, k)] or [(0, 0)])


def config1(seed: int = 1):
    """ER n=2000 m=20000 plus a planted 50-vertex set, internal pair probability 1/2."""
    return er_planted(seed, 2000, 20000, 50, 1, 2)


def config2(seed: int = 1):
    """R-MAT scale 22, 16*2^22 samples, (a,b,c,d)=(.57,.19,.19,.05)."""
    return rmat(seed, 22, 16 << 22, 57, 19, 19)


def config3(seed: int = 1, n: int = 40_000_000, max_deg: float = 2_000_000.0):
    """Chung-Lu n=40M, gamma=2.1, mean weight 30, weight cap 2M."""
    return chunglu(seed, n, 2.1, 30.0, max_deg)


MIX_STREAM = 77


def mix_params(seed: int, i: int):
    """Parameters of the i-th graph of the batched mix: (kind, n, mean_degree, graph_seed)."""
    lib = _load()
    gseed = int(lib.gg_rnd(seed, MIX_STREAM, i))
    u1 = (int(lib.gg_rnd(gseed, 1, 0)) >> 11) / float(1 << 53)
    u2 = (int(lib.gg_rnd(gseed, 1, 1)) >> 11) / float(1 << 53)
    kind = int(lib.gg_rnd(gseed, 1, 2)) % 3
    n = int(math.floor(math.exp(math.log(100.0) + u1 * (math.log(200000.0) - math.log(100.0)))))
    n = max(100, min(200000, n))
    d = 4.0 + 60.0 * u2
    return kind, n, d, gseed


def mix_graph(seed: int, i: int):
    """The i-th graph of the batched mix (0 = ER, 1 = R-MAT, 2 = ER + planted block)."""
    kind, n, d, gseed = mix_params(seed, i)
    samples = int(n * d / 2)
    if kind == 0:
        return er_block(gseed, n, samples, 0, 0, 1)
    if kind == 1:
        scale = max(1, (n - 1).bit_length())
        return rmat(gseed, scale, samples, 57, 19, 19, n=n)
    block = max(2, n // 20)
    return er_block(gseed, n, samples, block, 3, 10)
