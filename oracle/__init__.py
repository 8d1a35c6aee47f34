"""CPU oracle for the Greedy++ peeling hot path (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline
leg of ``bench.py`` may import this package.  The product library never loads
it, and the two share no code.  The only code they have in common is the
seeded input generator package ``graphgen``, which holds none of the method's
arithmetic.

The arithmetic lives in ``greedypp_oracle.c``: plain loops with exact
integers, following Algorithms 2 and 3 of the paper.  This module handles
argument marshalling and result state.  ``brute`` has the exhaustive checkers
for tiny graphs.

Parity status: every function here is pinned by the ``-m "not gpu"`` tests
listed in ``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "greedypp_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_oracle.so")
_lib = None
_OMP_SRC = os.path.join(_HERE, "timing_omp.c")
_OMP_PATH = os.path.join(_HERE, "_timing_omp.so")
_omp = None

VARIANTS = {"seq": 0, "peel": 1, "sort": 2, "peel_mono": 3}


def build(force: bool = True, extra_flags=(), out: str | None = None) -> str:
    """Compile the oracle into a shared object (gcc -O2, no OpenMP: single thread)."""
    path = out or _LIB_PATH
    if force or not os.path.exists(path):
        tmp = path + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=gnu11", *extra_flags, "-o", tmp, _SRC])
        os.replace(tmp, path)
    return path


def build_omp(force: bool = True) -> str:
    """Compile the multi-threaded timing build (timing_omp.c, gcc -O2 -fopenmp)."""
    if force or not os.path.exists(_OMP_PATH):
        tmp = _OMP_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11", "-o", tmp, _OMP_SRC])
        os.replace(tmp, _OMP_PATH)
    return _OMP_PATH


def _bind(lib):
    P = ctypes.c_void_p
    i32 = ctypes.c_int32
    i64 = ctypes.c_int64
    lib.orc_run.restype = ctypes.c_int
    lib.orc_run.argtypes = [i32, P, P, i32, i32, i64, i64, P, P, P, i32, P, P, P, P, P, P, P]
    lib.orc_run_fused.restype = ctypes.c_int
    lib.orc_run_fused.argtypes = [i32, P, P, i32, i32, i64, i64, P, P, P, i32, P, P, P]
    lib.orc_order_seq.restype = i32
    lib.orc_order_seq.argtypes = [i32, P, P, P, P, P]
    lib.orc_order_peel.restype = i32
    lib.orc_order_peel.argtypes = [i32, P, P, P, i64, i64, P, P]
    lib.orc_order_peel_rule.restype = i32
    lib.orc_order_peel_rule.argtypes = [i32, P, P, P, i64, i64, i32, P, P]
    lib.orc_order_sort.restype = i32
    lib.orc_order_sort.argtypes = [i32, P, P, P]
    lib.orc_alg3.restype = None
    lib.orc_alg3.argtypes = [i32, P, P, P, P, P, P, P, P]
    lib.orc_digest.restype = ctypes.c_uint64
    lib.orc_digest.argtypes = [i32, P]
    lib.orc_coreness.restype = i32
    lib.orc_coreness.argtypes = [i32, P, P, P]
    return lib


def load_library(path: str | None = None):
    """Load the oracle library (the default one is built on first use)."""
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        _lib = _bind(ctypes.CDLL(_LIB_PATH))
    return _lib


def _ptr(a):
    return a.ctypes.data


def _csr(offsets, adj):
    off = np.ascontiguousarray(offsets, dtype=np.int32)
    a = np.ascontiguousarray(adj, dtype=np.int32)
    if a.size == 0:
        a = np.zeros(1, dtype=np.int32)
    return off, a


def parse_eps(eps) -> tuple[int, int]:
    """eps as an exact rational (num, den); a decimal string such as "0.1" is read exactly."""
    if isinstance(eps, tuple):
        num, den = int(eps[0]), int(eps[1])
    else:
        from fractions import Fraction

        f = Fraction(str(eps))
        num, den = f.numerator, f.denominator
    if num < 0 or den < 1:
        raise ValueError("eps must be a non-negative rational")
    return num, den


@dataclass
class State:
    """Algorithm state after some iterations (what carries across calls)."""

    n: int
    m: int
    loads: np.ndarray
    best: np.ndarray  # int64[4]: edges, vertices, iteration (0 = input graph), index
    best_pos: np.ndarray
    iters: int = 0
    hist: list = field(default_factory=list)  # per iteration (edges, vertices)
    hist_idx: list = field(default_factory=list)
    digests: list = field(default_factory=list)
    rounds: list = field(default_factory=list)
    width: list = field(default_factory=list)
    last_pos: np.ndarray | None = None
    last_round: np.ndarray | None = None

    @staticmethod
    def fresh(offsets) -> "State":
        n = len(offsets) - 1
        m = int(offsets[-1]) // 2
        return State(
            n=n,
            m=m,
            loads=np.zeros(n, dtype=np.int64),
            best=np.array([m, n, 0, 0], dtype=np.int64),
            best_pos=np.zeros(n, dtype=np.int32),
        )

    def best_mask(self) -> np.ndarray:
        """Membership of the best vertex set (all vertices while the input graph is best)."""
        if self.best[2] == 0:
            return np.ones(self.n, dtype=bool)
        return self.best_pos >= self.best[3]


def run(offsets, adj, T: int, variant: str, eps=(0, 1), state: State | None = None, lib=None) -> State:
    """Decoupled form: ordering, then Algorithm 3.  Appends T iterations to ``state``."""
    lib = lib or load_library()
    off, a = _csr(offsets, adj)
    n = len(off) - 1
    st = state or State.fresh(off)
    num, den = parse_eps(eps)
    hist = np.zeros(2 * max(T, 1), dtype=np.int64)
    hidx = np.zeros(max(T, 1), dtype=np.int64)
    dig = np.zeros(max(T, 1), dtype=np.uint64)
    rnd = np.zeros(max(T, 1), dtype=np.int32)
    wid = np.zeros(max(T, 1), dtype=np.int64)
    lp = np.zeros(n, dtype=np.int32) if st.last_pos is None else st.last_pos
    lr = np.zeros(n, dtype=np.int32) if st.last_round is None else st.last_round
    rc = lib.orc_run(n, _ptr(off), _ptr(a), T, VARIANTS[variant], num, den, _ptr(st.loads), _ptr(st.best),
                     _ptr(st.best_pos), st.iters, _ptr(hist), _ptr(hidx), _ptr(dig), _ptr(rnd), _ptr(wid),
                     _ptr(lp), _ptr(lr))
    if rc != 0:
        raise RuntimeError("oracle run failed")
    st.iters += T
    st.hist += [(int(hist[2 * t]), int(hist[2 * t + 1])) for t in range(T)]
    st.hist_idx += [int(x) for x in hidx[:T]]
    st.digests += [int(x) for x in dig[:T]]
    st.rounds += [int(x) for x in rnd[:T]]
    st.width += [int(x) for x in wid[:T]]
    if T > 0:
        st.last_pos, st.last_round = lp, lr
    return st


def run_omp(offsets, adj, T: int, variant: str, eps=(0, 1), state: State | None = None, threads: int = 0) -> State:
    """The multi-threaded timing build (timing_omp.c): the same outputs as ``run`` for "peel", "peel_mono" and
    "sort", computed on ``threads`` OpenMP threads (0 = OpenMP's default).  Used to time the CPU baseline on all
    host cores; the parity reference stays ``run``."""
    global _omp
    if _omp is None:
        if not os.path.exists(_OMP_PATH):
            build_omp(force=False)
        _omp = ctypes.CDLL(_OMP_PATH)
        P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        _omp.orc_run_omp.restype = ctypes.c_int
        _omp.orc_run_omp.argtypes = [i32, P, P, i32, i32, i64, i64, P, P, P, i32, P, P, P, P, P, P, P, i32]
    if variant not in ("peel", "peel_mono", "sort"):
        raise ValueError("the timing build offers peel, peel_mono and sort")
    off, a = _csr(offsets, adj)
    n = len(off) - 1
    st = state or State.fresh(off)
    num, den = parse_eps(eps)
    hist = np.zeros(2 * max(T, 1), dtype=np.int64)
    hidx = np.zeros(max(T, 1), dtype=np.int64)
    dig = np.zeros(max(T, 1), dtype=np.uint64)
    rnd = np.zeros(max(T, 1), dtype=np.int32)
    wid = np.zeros(max(T, 1), dtype=np.int64)
    lp = np.zeros(n, dtype=np.int32) if st.last_pos is None else st.last_pos
    lr = np.zeros(n, dtype=np.int32) if st.last_round is None else st.last_round
    rc = _omp.orc_run_omp(n, _ptr(off), _ptr(a), T, VARIANTS[variant], num, den, _ptr(st.loads), _ptr(st.best),
                          _ptr(st.best_pos), st.iters, _ptr(hist), _ptr(hidx), _ptr(dig), _ptr(rnd), _ptr(wid),
                          _ptr(lp), _ptr(lr), threads)
    if rc != 0:
        raise RuntimeError("timing build run failed")
    st.iters += T
    st.hist += [(int(hist[2 * t]), int(hist[2 * t + 1])) for t in range(T)]
    st.hist_idx += [int(x) for x in hidx[:T]]
    st.digests += [int(x) for x in dig[:T]]
    st.rounds += [int(x) for x in rnd[:T]]
    st.width += [int(x) for x in wid[:T]]
    if T > 0:
        st.last_pos, st.last_round = lp, lr
    return st


def run_fused(offsets, adj, T: int, variant: str, eps=(0, 1), state: State | None = None, lib=None) -> State:
    """Fused form of Algorithm 2 (density compared before each single peel)."""
    lib = lib or load_library()
    off, a = _csr(offsets, adj)
    n = len(off) - 1
    st = state or State.fresh(off)
    num, den = parse_eps(eps)
    hist = np.zeros(2 * max(T, 1), dtype=np.int64)
    hidx = np.zeros(max(T, 1), dtype=np.int64)
    lp = np.zeros(n, dtype=np.int32)
    rc = lib.orc_run_fused(n, _ptr(off), _ptr(a), T, VARIANTS[variant], num, den, _ptr(st.loads), _ptr(st.best),
                           _ptr(st.best_pos), st.iters, _ptr(hist), _ptr(hidx), _ptr(lp))
    if rc != 0:
        raise RuntimeError("oracle run failed")
    st.iters += T
    st.hist += [(int(hist[2 * t]), int(hist[2 * t + 1])) for t in range(T)]
    st.hist_idx += [int(x) for x in hidx[:T]]
    if T > 0:
        st.last_pos = lp
    return st


def order(offsets, adj, loads, variant: str, eps=(0, 1), lib=None):
    """One ordering: (pos, round, number of rounds)."""
    lib = lib or load_library()
    off, a = _csr(offsets, adj)
    n = len(off) - 1
    ld = np.ascontiguousarray(loads, dtype=np.int64)
    pos = np.zeros(n, dtype=np.int32)
    rnd = np.zeros(n, dtype=np.int32)
    if variant == "seq":
        r = lib.orc_order_seq(n, _ptr(off), _ptr(a), _ptr(ld), _ptr(pos), _ptr(rnd))
    elif variant == "peel":
        num, den = parse_eps(eps)
        r = lib.orc_order_peel(n, _ptr(off), _ptr(a), _ptr(ld), num, den, _ptr(pos), _ptr(rnd))
    elif variant == "peel_mono":
        num, den = parse_eps(eps)
        r = lib.orc_order_peel_rule(n, _ptr(off), _ptr(a), _ptr(ld), num, den, 1, _ptr(pos), _ptr(rnd))
    else:
        r = lib.orc_order_sort(n, _ptr(ld), _ptr(pos), _ptr(rnd))
    return pos, rnd, int(r)


def alg3(offsets, adj, pos, lib=None):
    """Algorithm 3 on a given order: (A, B, (edges, vertices, index))."""
    lib = lib or load_library()
    off, a = _csr(offsets, adj)
    n = len(off) - 1
    p = np.ascontiguousarray(pos, dtype=np.int32)
    A = np.zeros(n, dtype=np.int64)
    B = np.zeros(n, dtype=np.int64)
    e = ctypes.c_int64()
    v = ctypes.c_int64()
    i = ctypes.c_int64()
    lib.orc_alg3(n, _ptr(off), _ptr(a), _ptr(p), _ptr(A), _ptr(B), ctypes.addressof(e), ctypes.addressof(v),
                 ctypes.addressof(i))
    return A, B, (e.value, v.value, i.value)


def digest(round_arr, lib=None) -> int:
    lib = lib or load_library()
    r = np.ascontiguousarray(round_arr, dtype=np.int32)
    return int(lib.orc_digest(len(r), _ptr(r)))


def coreness(offsets, adj, lib=None):
    """Core numbers and k_max by Coreness (Section 2): (int32[n], k_max)."""
    lib = lib or load_library()
    o, a = _csr(offsets, adj)
    n = len(o) - 1
    core = np.zeros(max(n, 1), dtype=np.int32)
    kmax = lib.orc_coreness(n, _ptr(o), _ptr(a), _ptr(core))
    if kmax < 0:
        raise MemoryError("oracle coreness: out of memory")
    return core[:n], int(kmax)
