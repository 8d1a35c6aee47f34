"""Python binding of libdsg.so: Greedy++ peeling on one MI355X.

This module only marshals arguments.  Every step of the algorithm runs in the
library's HIP kernels (csrc/), behind the C ABI declared in include/dsg.h.
PyTorch supplies device memory (the CSR tensors and the workspace) and the
HIP stream.  When the compiled library is missing, importing this package
still works, but any call raises RuntimeError.  There is no fallback path.

    import paper_2311_04333_amd as dsg
    ctx = dsg.Context(0)
    g = dsg.Graph(ctx, offsets, adj, t_cap=64)   # numpy or torch CSR
    g.run(20, eps=(1, 10), variant="peel")
    edges, verts, it, idx = g.best()
"""
from __future__ import annotations

import ctypes
import os
import sys
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdsg.so")
_lib = None

VARIANTS = {"seq": 0, "peel": 1, "sort": 2, "peel_mono": 3}
STATUS = {0: "DSG_OK", -1: "DSG_EINVAL", -2: "DSG_ENOMEM", -3: "DSG_EDEVICE", -4: "DSG_EOVERFLOW",
          -5: "DSG_ESTATE", -6: "DSG_EBUSY"}
VALIDATE = 1
HUB_ORDER = 2
# Graph(hub_order="auto") renumbers by degree from this many vertices on
HUB_AUTO_MIN_N = 1 << 22

# every entry point declared in include/dsg.h: (name, restype, argtypes)
_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
SIGNATURES = [
    ("dsg_ctx_create", ctypes.c_int, [ctypes.c_int, _P, _P]),
    ("dsg_ctx_destroy", ctypes.c_int, [_P]),
    ("dsg_workspace_bytes", ctypes.c_int, [_I32, _I64, _I32, _P]),
    ("dsg_workspace_bytes_ex", ctypes.c_int, [_I32, _I64, _I32, _I32, _P]),
    ("dsg_graph_create", ctypes.c_int, [_P, _I32, _I64, _P, _P, _P, _I64, _I32, _I32, _P]),
    ("dsg_run", ctypes.c_int, [_P, _I32, _I32, _I32, ctypes.c_int]),
    ("dsg_run_until", ctypes.c_int, [_P, _I32, _I32, _I32, ctypes.c_int, _I32, _I32, _P, _P]),
    ("dsg_reset", ctypes.c_int, [_P]),
    ("dsg_sync", ctypes.c_int, [_P]),
    ("dsg_get_best", ctypes.c_int, [_P, _P, _P, _P, _P]),
    ("dsg_get_best_mask", ctypes.c_int, [_P, _P]),
    ("dsg_get_loads", ctypes.c_int, [_P, _P]),
    ("dsg_get_iter_densities", ctypes.c_int, [_P, _P, _P, _P, _I32, _P]),
    ("dsg_get_order", ctypes.c_int, [_P, _P, _P, _P]),
    ("dsg_get_iter_digests", ctypes.c_int, [_P, _P, _P, _I32, _P]),
    ("dsg_graph_destroy", ctypes.c_int, [_P]),
    ("dsg_last_run_ms", ctypes.c_int, [_P, _P]),
    ("dsg_coreness", ctypes.c_int, [_P, _I32, _I64, _P, _P, _P, _I64, _I32, _P, _P, _P, _P]),
    ("dsg_get_iter_bounds", ctypes.c_int, [_P, _P, _P, _I32, _P]),
    ("dsg_par_workspace_bytes", ctypes.c_int, [_I32, _I64, _I32, _P]),
    ("dsg_par_run", ctypes.c_int, [_P, _I32, _I64, _P, _P, _P, _I64, _I32, _I32, _I32, _I32, _I32, _P, _P, _P, _P, _P,
                                   _P, _P, _P, _P]),
    ("dsg_par_run_apx", ctypes.c_int, [_P, _I32, _I64, _P, _P, _P, _I64, _I32, _I32, _I32, _I32, _I32, _I32, _I32,
                                       _I32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    ("dsg_par_run_noalloc", ctypes.c_int, [_P, _I32, _I64, _P, _P, _I32, _I32, _I32, _I32, _I32, _P, _P, _P, _P, _P,
                                           _P, _P, _P, _P]),
    ("dsg_set_peel_tuning", ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int64]),
    ("dsg_set_sort_tuning", ctypes.c_int, [_P, _I32]),
    ("dsg_set_peel_select", ctypes.c_int, [_P, _I32]),
    ("dsg_set_graph_replay", ctypes.c_int, [_P, _I32]),
    ("dsg_get_graph_replay", ctypes.c_int, [_P, _P]),
    ("dsg_set_kernel_timing", ctypes.c_int, [_P, _I32]),
    ("dsg_get_kernel_timing", ctypes.c_int, [_P, _P, _P]),
    ("dsg_batch_workspace_bytes", ctypes.c_int, [_P, _I32, _I32, _P]),
    ("dsg_batch_create", ctypes.c_int, [_P, _P, _I32, _I32, _P, _I64, _I32, _P]),
    ("dsg_batch_set_config", ctypes.c_int, [_P, _I32, _I32]),
    ("dsg_batch_run", ctypes.c_int, [_P]),
    ("dsg_batch_reset", ctypes.c_int, [_P]),
    ("dsg_batch_get_best", ctypes.c_int, [_P, _I32, _P, _P, _P, _P]),
    ("dsg_batch_get_best_mask", ctypes.c_int, [_P, _I32, _P]),
    ("dsg_batch_get_loads", ctypes.c_int, [_P, _I32, _P]),
    ("dsg_batch_get_iter_densities", ctypes.c_int, [_P, _I32, _P, _P, _P, _I32, _P]),
    ("dsg_batch_get_iter_digests", ctypes.c_int, [_P, _I32, _P, _P, _I32, _P]),
    ("dsg_batch_last_run_ms", ctypes.c_int, [_P, _P]),
    ("dsg_batch_destroy", ctypes.c_int, [_P]),
    ("dsg_server_create", ctypes.c_int, [_P, _P, _I64, _I32, _P]),
    ("dsg_server_footprint", ctypes.c_int, [_I32, _I64, _I32, _P]),
    ("dsg_server_start", ctypes.c_int, [_P, _I32, _I32, ctypes.c_double, ctypes.c_double]),
    ("dsg_server_submit", ctypes.c_int, [_P, _P, _P, _I32, _I64, _I32, _I32, _I32, _P]),
    ("dsg_server_register", ctypes.c_int, [_P, _P, _P, _I32, _I64, _I32, _P]),
    ("dsg_server_submit_registered", ctypes.c_int, [_P, _I32, _I32, _I32, _I32, _P]),
    ("dsg_server_poll", ctypes.c_int, [_P, _P, _I32, _P]),
    ("dsg_server_fetch", ctypes.c_int, [_P, ctypes.c_uint64, _P, _P, _P, _P, _P, _P, _P]),
    ("dsg_server_release", ctypes.c_int, [_P, ctypes.c_uint64]),
    ("dsg_server_stop", ctypes.c_int, [_P]),
    ("dsg_server_destroy", ctypes.c_int, [_P]),
    ("dsg_last_error", ctypes.c_char_p, []),
]


class _BatchGraph(ctypes.Structure):
    """dsg_batch_graph of include/dsg.h."""

    _fields_ = [("d_offsets", ctypes.c_void_p), ("d_adj", ctypes.c_void_p), ("n", ctypes.c_int32),
                ("T", ctypes.c_int32), ("nnz", ctypes.c_int64), ("eps_num", ctypes.c_int32),
                ("eps_den", ctypes.c_int32)]


class DsgError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


def build(force: bool = True) -> str:
    """Compile libdsg.so for gfx950 (hipcc); see _build.py."""
    from . import _build

    return _build.build_library(force=force)


def library():
    """The loaded libdsg.so.  Raises RuntimeError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libdsg.so not found at {LIB_PATH}: build it first "
                           "(python -c 'import __graft_entry__ as g; g.build()')")
    # torch ships its own HIP runtime; load it first so that libdsg.so binds
    # to the same runtime (same SONAME) instead of a second copy from ROCm,
    # which would own the device separately from torch's allocations
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int):
    if status != 0:
        msg = library().dsg_last_error()
        raise DsgError(status, msg.decode() if msg else "")


def _finalize(obj, _sys=sys):
    """Garbage-collection release of a handle.  At interpreter exit the HIP
    runtime (and any profiler attached to it) may already be torn down, so no
    library call is made then: close handles explicitly before exiting.  (The
    defaults and the callers' bound references keep working while module
    globals are being cleared.)"""
    if _sys is None or _sys.is_finalizing():
        return
    try:
        obj.close()
    except Exception:
        pass


def parse_eps(eps) -> tuple[int, int]:
    """eps as an exact rational (num, den); a decimal string or float literal is read exactly."""
    if isinstance(eps, tuple):
        num, den = int(eps[0]), int(eps[1])
    else:
        f = Fraction(str(eps))
        num, den = f.numerator, f.denominator
    if num < 0 or den < 1 or num >= 2 ** 31 or den >= 2 ** 31:
        raise ValueError("eps must be a non-negative rational with 31-bit numerator and denominator")
    return num, den


def workspace_bytes(n: int, nnz: int, t_cap: int, flags: int = 0) -> int:
    out = ctypes.c_int64()
    _check(library().dsg_workspace_bytes_ex(n, nnz, t_cap, flags, ctypes.addressof(out)))
    return out.value


class Context:
    """A device and a HIP stream (torch's current stream by default)."""

    def __init__(self, device: int = 0, stream=None):
        import torch

        self.device = device
        self.torch_device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.torch_device)
        self.stream = stream
        handle = ctypes.c_void_p()
        _check(library().dsg_ctx_create(device, ctypes.c_void_p(stream.cuda_stream), ctypes.addressof(handle)))
        self._h = handle

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            library().dsg_ctx_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self, _fin=_finalize):
        _fin(self)


class Graph:
    """A CSR graph resident on the device plus its peeling state.

    ``offsets``/``adj`` may be numpy arrays (copied to the device) or int32
    device tensors (used in place).  The workspace is a torch uint8 tensor
    owned by this object.  ``hub_order``: renumber the vertices internally by
    degree (DSG_HUB_ORDER; same results, in the caller's ids); "auto" does so
    from HUB_AUTO_MIN_N vertices on.
    """

    def __init__(self, ctx: Context, offsets, adj, t_cap: int = 64, validate: bool = True, hub_order="auto"):
        import torch

        self.ctx = ctx
        dev = ctx.torch_device
        self.offsets = self._dev_i32(offsets, dev)
        self.adj = self._dev_i32(adj, dev)
        self.n = int(self.offsets.numel()) - 1
        self.nnz = int(self.adj.numel())
        self.m = self.nnz // 2
        self.t_cap = t_cap
        if hub_order == "auto":
            hub_order = self.n >= HUB_AUTO_MIN_N
        self.hub_order = bool(hub_order)
        flags = (VALIDATE if validate else 0) | (HUB_ORDER if self.hub_order else 0)
        nbytes = workspace_bytes(self.n, self.nnz, t_cap, flags)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        handle = ctypes.c_void_p()
        adj_ptr = self.adj.data_ptr() if self.nnz > 0 else 0
        _check(library().dsg_graph_create(ctx.handle, self.n, self.nnz, ctypes.c_void_p(self.offsets.data_ptr()),
                                          ctypes.c_void_p(adj_ptr), ctypes.c_void_p(aligned), nbytes, t_cap,
                                          flags, ctypes.addressof(handle)))
        self._h = handle

    @staticmethod
    def _dev_i32(x, dev):
        import torch

        if isinstance(x, torch.Tensor):
            t = x.to(device=dev, dtype=torch.int32)
        else:
            t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.int32)).to(dev)
        if t.numel() == 0:
            t = torch.zeros(1, dtype=torch.int32, device=dev)[:0]
        return t.contiguous()

    # ------------------------------------------------------------ running
    def run(self, T: int, eps=(0, 1), variant: str = "peel"):
        num, den = parse_eps(eps)
        _check(library().dsg_run(self._h, T, num, den, VARIANTS[variant]))
        return self

    def run_until(self, T_max: int, eps=(0, 1), variant: str = "peel", tol=(1, 1000)):
        """dsg_run_until: iterations until the load certificate proves the best density within a factor 1 + tol of
        the optimum, at most T_max.  Returns (iterations run, certified)."""
        num, den = parse_eps(eps)
        tn, td = parse_eps(tol)
        it = ctypes.c_int32()
        ok = ctypes.c_int32()
        _check(library().dsg_run_until(self._h, T_max, num, den, VARIANTS[variant], tn, td, ctypes.addressof(it),
                                       ctypes.addressof(ok)))
        return it.value, bool(ok.value)

    def reset(self):
        _check(library().dsg_reset(self._h))
        return self

    def sync(self):
        _check(library().dsg_sync(self._h))

    def last_run_ms(self) -> float:
        ms = ctypes.c_float()
        _check(library().dsg_last_run_ms(self._h, ctypes.addressof(ms)))
        return ms.value

    def set_peel_tuning(self, bucket_min_edges: int = -1, coarse_min_edges: int = -1):
        """PEEL round-loop tuning (results do not depend on it): frontier sizes (adjacency entries) from which a
        round applies decrements through owner buckets, and from which it sweeps coarse chunks; -1 = default."""
        _check(library().dsg_set_peel_tuning(self._h, int(bucket_min_edges), int(coarse_min_edges)))
        return self

    def set_sort_tuning(self, coarse_ranks: int = -1):
        """SORT sweep tuning (results do not depend on it): coarse position classes first; -1 = by size, 0 = off,
        1 = on."""
        _check(library().dsg_set_sort_tuning(self._h, int(coarse_ranks)))
        return self

    def set_peel_select(self, mode: int = -1):
        """dsg_set_peel_select: -1 = by size, 0 = full-list select, 1 = near-list select (same results)."""
        _check(library().dsg_set_peel_select(self._h, mode))
        return self

    def iter_bounds(self):
        """Per recorded iteration: (empirical width, largest load after it).  rho* <= largest load / iterations."""
        w = np.zeros(self.t_cap, dtype=np.int32)
        lm = np.zeros(self.t_cap, dtype=np.int64)
        cnt = ctypes.c_int32()
        _check(library().dsg_get_iter_bounds(self._h, w.ctypes.data, lm.ctypes.data, self.t_cap, ctypes.addressof(cnt)))
        k = min(cnt.value, self.t_cap)
        return [(int(w[i]), int(lm[i])) for i in range(k)]

    def set_graph_replay(self, enable: bool = True):
        """Capture a run's launches into a HIP graph and replay it for repeated runs with the same parameters."""
        _check(library().dsg_set_graph_replay(self._h, 1 if enable else 0))
        return self

    def graph_replay_state(self) -> int:
        """1 = a captured run is cached, 0 = none (or replay off), -1 = capture refused (eager runs)."""
        st = ctypes.c_int32()
        _check(library().dsg_get_graph_replay(self._h, ctypes.addressof(st)))
        return st.value

    def set_kernel_timing(self, enable: bool = True):
        _check(library().dsg_set_kernel_timing(self._h, 1 if enable else 0))
        return self

    def kernel_timing(self):
        """(total ms, launches) of the dominant kernel over the last run (timing must be enabled)."""
        ms = ctypes.c_float()
        cnt = ctypes.c_int32()
        _check(library().dsg_get_kernel_timing(self._h, ctypes.addressof(ms), ctypes.addressof(cnt)))
        return ms.value, cnt.value

    # ------------------------------------------------------------ results
    def best(self):
        """(edges, vertices, iteration, index) of the best subgraph so far."""
        e, v = ctypes.c_int64(), ctypes.c_int64()
        it, idx = ctypes.c_int32(), ctypes.c_int32()
        _check(library().dsg_get_best(self._h, ctypes.addressof(e), ctypes.addressof(v), ctypes.addressof(it),
                                      ctypes.addressof(idx)))
        return e.value, v.value, it.value, idx.value

    def best_mask(self) -> np.ndarray:
        out = np.zeros(self.n, dtype=np.uint8)
        _check(library().dsg_get_best_mask(self._h, out.ctypes.data))
        return out.astype(bool)

    def loads(self) -> np.ndarray:
        out = np.zeros(self.n, dtype=np.int64)
        _check(library().dsg_get_loads(self._h, out.ctypes.data))
        return out

    def iter_densities(self):
        """Per-iteration densest suffix: list of (edges, vertices, index)."""
        cnt = ctypes.c_int32()
        _check(library().dsg_get_iter_densities(self._h, None, None, None, 0, ctypes.addressof(cnt)))
        k = cnt.value
        e = np.zeros(max(k, 1), dtype=np.int64)
        v = np.zeros(max(k, 1), dtype=np.int64)
        i = np.zeros(max(k, 1), dtype=np.int32)
        _check(library().dsg_get_iter_densities(self._h, e.ctypes.data, v.ctypes.data, i.ctypes.data, k,
                                                ctypes.addressof(cnt)))
        return [(int(e[t]), int(v[t]), int(i[t])) for t in range(k)]

    def order(self):
        """(round[n], pos[n], number of rounds) of the last iteration."""
        rnd = np.zeros(self.n, dtype=np.int32)
        pos = np.zeros(self.n, dtype=np.int32)
        nr = ctypes.c_int32()
        _check(library().dsg_get_order(self._h, rnd.ctypes.data, pos.ctypes.data, ctypes.addressof(nr)))
        return rnd, pos, nr.value

    def digests(self):
        """(per-iteration order digests, per-iteration round counts)."""
        cnt = ctypes.c_int32()
        _check(library().dsg_get_iter_digests(self._h, None, None, 0, ctypes.addressof(cnt)))
        k = cnt.value
        d = np.zeros(max(k, 1), dtype=np.uint64)
        r = np.zeros(max(k, 1), dtype=np.int32)
        _check(library().dsg_get_iter_digests(self._h, d.ctypes.data, r.ctypes.data, k, ctypes.addressof(cnt)))
        return [int(x) for x in d[:k]], [int(x) for x in r[:k]]

    def close(self):
        if getattr(self, "_h", None):
            library().dsg_graph_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self, _fin=_finalize):
        _fin(self)


class Batch:
    """Many graphs peeled in one persistent launch (PEEL rule).

    ``graphs`` is a list of (offsets, adj) host CSRs.  They are packed into
    one offsets tensor and one adjacency tensor on the device, and each
    graph's pointers are slices of those.  ``T`` and ``eps`` may be scalars
    or per-graph lists.
    """

    def __init__(self, ctx: Context, graphs, T=20, eps=(1, 10), t_cap: int = 64, validate: bool = True):
        import torch

        self.ctx = ctx
        dev = ctx.torch_device
        count = len(graphs)
        Ts = list(T) if isinstance(T, list) else [T] * count
        epss = list(eps) if isinstance(eps, list) else [eps] * count
        sizes_o = [len(o) for o, _ in graphs]
        sizes_a = [len(a) for _, a in graphs]
        self.n = [s - 1 for s in sizes_o]
        self.nnz = sizes_a
        off_all = np.concatenate([np.asarray(o, dtype=np.int32) for o, _ in graphs])
        adj_all = np.concatenate([np.asarray(a, dtype=np.int32) for _, a in graphs] + [np.zeros(1, np.int32)])
        self.offsets = torch.from_numpy(off_all).to(dev)
        self.adj = torch.from_numpy(adj_all).to(dev)
        arr = (_BatchGraph * count)()
        po, pa = 0, 0
        base_o, base_a = self.offsets.data_ptr(), self.adj.data_ptr()
        for g in range(count):
            num, den = parse_eps(epss[g])
            arr[g].d_offsets = base_o + 4 * po
            arr[g].d_adj = base_a + 4 * pa
            arr[g].n = sizes_o[g] - 1
            arr[g].T = int(Ts[g])
            arr[g].nnz = sizes_a[g]
            arr[g].eps_num = num
            arr[g].eps_den = den
            po += sizes_o[g]
            pa += sizes_a[g]
        self._desc = arr
        self.count = count
        nbytes = ctypes.c_int64()
        _check(library().dsg_batch_workspace_bytes(ctypes.addressof(arr), count, t_cap, ctypes.addressof(nbytes)))
        self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=dev)
        aligned = (self.workspace.data_ptr() + 255) // 256 * 256
        handle = ctypes.c_void_p()
        _check(library().dsg_batch_create(ctx.handle, ctypes.addressof(arr), count, t_cap, ctypes.c_void_p(aligned),
                                          nbytes.value, VALIDATE if validate else 0, ctypes.addressof(handle)))
        self._h = handle

    def set_config(self, cfg: int, blocks_per_cu: int):
        _check(library().dsg_batch_set_config(self._h, cfg, blocks_per_cu))
        return self

    def run(self):
        _check(library().dsg_batch_run(self._h))
        return self

    def reset(self):
        _check(library().dsg_batch_reset(self._h))
        return self

    def last_run_ms(self) -> float:
        ms = ctypes.c_float()
        _check(library().dsg_batch_last_run_ms(self._h, ctypes.addressof(ms)))
        return ms.value

    def best(self, i: int):
        e, v = ctypes.c_int64(), ctypes.c_int64()
        it, idx = ctypes.c_int32(), ctypes.c_int32()
        _check(library().dsg_batch_get_best(self._h, i, ctypes.addressof(e), ctypes.addressof(v),
                                            ctypes.addressof(it), ctypes.addressof(idx)))
        return e.value, v.value, it.value, idx.value

    def best_mask(self, i: int) -> np.ndarray:
        out = np.zeros(self.n[i], dtype=np.uint8)
        _check(library().dsg_batch_get_best_mask(self._h, i, out.ctypes.data))
        return out.astype(bool)

    def loads(self, i: int) -> np.ndarray:
        out = np.zeros(self.n[i], dtype=np.int64)
        _check(library().dsg_batch_get_loads(self._h, i, out.ctypes.data))
        return out

    def iter_densities(self, i: int):
        cnt = ctypes.c_int32()
        _check(library().dsg_batch_get_iter_densities(self._h, i, None, None, None, 0, ctypes.addressof(cnt)))
        k = cnt.value
        e = np.zeros(max(k, 1), dtype=np.int64)
        v = np.zeros(max(k, 1), dtype=np.int64)
        ix = np.zeros(max(k, 1), dtype=np.int32)
        _check(library().dsg_batch_get_iter_densities(self._h, i, e.ctypes.data, v.ctypes.data, ix.ctypes.data, k,
                                                      ctypes.addressof(cnt)))
        return [(int(e[t]), int(v[t]), int(ix[t])) for t in range(k)]

    def digests(self, i: int):
        cnt = ctypes.c_int32()
        _check(library().dsg_batch_get_iter_digests(self._h, i, None, None, 0, ctypes.addressof(cnt)))
        k = cnt.value
        d = np.zeros(max(k, 1), dtype=np.uint64)
        r = np.zeros(max(k, 1), dtype=np.int32)
        _check(library().dsg_batch_get_iter_digests(self._h, i, d.ctypes.data, r.ctypes.data, k,
                                                    ctypes.addressof(cnt)))
        return [int(x) for x in d[:k]], [int(x) for x in r[:k]]

    def view(self, i: int) -> "BatchGraphView":
        return BatchGraphView(self, i)

    def close(self):
        if getattr(self, "_h", None):
            library().dsg_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self, _fin=_finalize):
        _fin(self)


class BatchGraphView:
    """Graph i of a Batch, with the result accessors of Graph."""

    def __init__(self, batch: Batch, i: int):
        self.batch, self.i = batch, i

    def loads(self):
        return self.batch.loads(self.i)

    def best(self):
        return self.batch.best(self.i)

    def best_mask(self):
        return self.batch.best_mask(self.i)

    def iter_densities(self):
        return self.batch.iter_densities(self.i)

    def digests(self):
        return self.batch.digests(self.i)


class Server:
    """Continuous-batching server (persistent kernel + pinned request ring).

    ``pool_bytes`` of device memory (a torch tensor owned here) holds the
    admitted requests.  ``submit`` returns a ticket, or None when the pool
    or the ring is full (DSG_EBUSY).
    """

    def __init__(self, ctx: Context, pool_bytes: int, ring_size: int = 8192):
        import torch

        self.ctx = ctx
        self.pool = torch.empty(pool_bytes + 256, dtype=torch.uint8, device=ctx.torch_device)
        aligned = (self.pool.data_ptr() + 255) // 256 * 256
        handle = ctypes.c_void_p()
        _check(library().dsg_server_create(ctx.handle, ctypes.c_void_p(aligned), pool_bytes, ring_size,
                                           ctypes.addressof(handle)))
        self._h = handle
        self.meta = {}

    @staticmethod
    def footprint(n: int, nnz: int, T: int) -> int:
        out = ctypes.c_int64()
        _check(library().dsg_server_footprint(n, nnz, T, ctypes.addressof(out)))
        return out.value

    def start(self, cfg: int = 1, blocks_per_cu: int = 1, idle_seconds: float = 60.0, max_seconds: float = 900.0):
        _check(library().dsg_server_start(self._h, cfg, blocks_per_cu, idle_seconds, max_seconds))
        return self

    def submit(self, offsets, adj, T: int, eps=(1, 10)):
        o = np.ascontiguousarray(offsets, dtype=np.int32)
        a = np.ascontiguousarray(adj, dtype=np.int32)
        if a.size == 0:
            a = np.zeros(1, dtype=np.int32)
        num, den = parse_eps(eps)
        t = ctypes.c_uint64()
        st = library().dsg_server_submit(self._h, o.ctypes.data, a.ctypes.data, len(o) - 1, len(adj), T, num, den,
                                         ctypes.addressof(t))
        if st == -6:
            return None
        _check(st)
        self.meta[t.value] = (len(o) - 1, T)
        return t.value

    def register(self, offsets, adj, validate: bool = True) -> int:
        """Keep a CSR resident on the device for repeated requests; returns its graph id."""
        import torch

        dev = self.ctx.torch_device
        o = torch.from_numpy(np.ascontiguousarray(offsets, dtype=np.int32)).to(dev)
        a = torch.from_numpy(np.ascontiguousarray(adj, dtype=np.int32) if len(adj) else np.zeros(1, np.int32)).to(dev)
        gid = ctypes.c_int32()
        _check(library().dsg_server_register(self._h, ctypes.c_void_p(o.data_ptr()), ctypes.c_void_p(a.data_ptr()),
                                             len(o) - 1, len(adj), VALIDATE if validate else 0,
                                             ctypes.addressof(gid)))
        self.resident = getattr(self, "resident", [])
        self.resident.append((o, a, len(o) - 1))
        return gid.value

    def submit_registered(self, graph_id: int, T: int, eps=(1, 10)):
        num, den = parse_eps(eps)
        t = ctypes.c_uint64()
        st = library().dsg_server_submit_registered(self._h, graph_id, T, num, den, ctypes.addressof(t))
        if st == -6:
            return None
        _check(st)
        self.meta[t.value] = (self.resident[graph_id][2], T)
        return t.value

    def poll(self, cap: int = 4096):
        out = np.zeros(cap, dtype=np.uint64)
        cnt = ctypes.c_int32()
        _check(library().dsg_server_poll(self._h, out.ctypes.data, cap, ctypes.addressof(cnt)))
        return [int(x) for x in out[:cnt.value]]

    def fetch(self, ticket: int, loads: bool = False):
        n, T = self.meta[ticket]
        best = np.zeros(4, dtype=np.int64)
        e = np.zeros(T, dtype=np.int64)
        v = np.zeros(T, dtype=np.int64)
        ix = np.zeros(T, dtype=np.int32)
        dg = np.zeros(T, dtype=np.uint64)
        rd = np.zeros(T, dtype=np.int32)
        ld = np.zeros(n, dtype=np.int64) if loads else None
        _check(library().dsg_server_fetch(self._h, ticket, best.ctypes.data, e.ctypes.data, v.ctypes.data,
                                          ix.ctypes.data, dg.ctypes.data, rd.ctypes.data,
                                          ld.ctypes.data if loads else None))
        return {"best": tuple(int(x) for x in best), "hist": [(int(e[t]), int(v[t])) for t in range(T)],
                "hist_idx": [int(x) for x in ix], "digests": [int(x) for x in dg], "rounds": [int(x) for x in rd],
                "loads": ld}

    def release(self, ticket: int):
        _check(library().dsg_server_release(self._h, ticket))
        self.meta.pop(ticket, None)

    def stop(self):
        _check(library().dsg_server_stop(self._h))

    def close(self):
        if getattr(self, "_h", None):
            library().dsg_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self, _fin=_finalize):
        _fin(self)


class _ParResultC(ctypes.Structure):
    _fields_ = [("best_edges", ctypes.c_int64), ("best_verts", ctypes.c_int64), ("best_iter", ctypes.c_int32),
                ("kmax", ctypes.c_int32), ("level", ctypes.c_int32), ("prunes", ctypes.c_int32),
                ("final_n", ctypes.c_int32), ("pad", ctypes.c_int32), ("final_nnz", ctypes.c_int64)]


class _ParApxC(ctypes.Structure):
    _fields_ = [("apx_kmax", ctypes.c_int32), ("apx_level", ctypes.c_int32), ("apx_n", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("apx_nnz", ctypes.c_int64)]


class ParResult:
    """Outcome of dsg_par_run (Pruning-and-Refining, Algorithm 1): best (edges, vertices, iteration), the best
    set's mask, per-iteration (edges, vertices) and index of S', the (n_i, m_i) and core level of each refined
    graph, core numbers, k_max, the final level and the number of prunes after the first."""

    def __init__(self, c, hist, hist_idx, sizes, levels, best_mask, core):
        self.best = (int(c.best_edges), int(c.best_verts), int(c.best_iter))
        self.kmax = int(c.kmax)
        self.level = int(c.level)
        self.prunes = int(c.prunes)
        self.final_size = (int(c.final_n), int(c.final_nnz) // 2)
        self.hist = hist
        self.hist_idx = hist_idx
        self.sizes = sizes
        self.levels = levels
        self.best_mask = best_mask
        self.core = core
        self.apx_core = None
        self.apx_kmax = 0
        self.apx_level = 0
        self.apx_size = None


def par_workspace_bytes(n: int, nnz: int, T: int) -> int:
    out = ctypes.c_int64()
    _check(library().dsg_par_workspace_bytes(n, nnz, T, ctypes.addressof(out)))
    return out.value


def par_run(ctx: Context, offsets, adj, T: int, eps=(0, 1), variant: str = "peel", validate: bool = True,
            workspace=None, prune: str = "exact", c=(3, 2)) -> ParResult:
    """dsg_par_run (prune="exact") or dsg_par_run_apx (prune="apx": approximate k-core pruning only; "apx_exact":
    approximate, then exact) on a CSR (numpy arrays or int32 device tensors).  `c` is the approximation ratio
    c_num / c_den.  `workspace` (a uint8 device tensor of at least par_workspace_bytes + 256 bytes) may be passed to
    reuse one allocation across calls."""
    if prune not in ("exact", "apx", "apx_exact"):
        raise ValueError(f"unknown pruning {prune!r}")
    import torch

    dev = ctx.torch_device
    o = Graph._dev_i32(offsets, dev)
    a = Graph._dev_i32(adj, dev)
    n, nnz = int(o.numel()) - 1, int(a.numel())
    nbytes = par_workspace_bytes(n, nnz, T)
    if workspace is None or workspace.numel() < nbytes + 256:
        workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    base = workspace.data_ptr()
    aligned = (base + 255) // 256 * 256
    he = np.zeros(max(T, 1), dtype=np.int64)
    hv = np.zeros(max(T, 1), dtype=np.int64)
    hi = np.zeros(max(T, 1), dtype=np.int32)
    hn = np.zeros(max(T, 1), dtype=np.int32)
    hm = np.zeros(max(T, 1), dtype=np.int64)
    hl = np.zeros(max(T, 1), dtype=np.int32)
    mask = np.zeros(n, dtype=np.uint8)
    core = np.zeros(n, dtype=np.int32)
    num, den = parse_eps(eps)
    res = _ParResultC()
    d_off = ctypes.c_void_p(o.data_ptr())
    d_adj = ctypes.c_void_p(a.data_ptr() if nnz > 0 else 0)
    outs = (he.ctypes.data, hv.ctypes.data, hi.ctypes.data, hn.ctypes.data, hm.ctypes.data, hl.ctypes.data,
            mask.ctypes.data, core.ctypes.data)
    flags = VALIDATE if validate else 0
    apx = None
    if prune == "exact":
        _check(library().dsg_par_run(ctx.handle, n, nnz, d_off, d_adj, ctypes.c_void_p(aligned), nbytes, T, num, den,
                                     VARIANTS[variant], flags, ctypes.addressof(res), *outs))
    else:
        apx = _ParApxC()
        apx_core = np.zeros(n, dtype=np.int32)
        _check(library().dsg_par_run_apx(ctx.handle, n, nnz, d_off, d_adj, ctypes.c_void_p(aligned), nbytes, T, num,
                                         den, VARIANTS[variant], flags, 1 if prune == "apx_exact" else 0, int(c[0]),
                                         int(c[1]), ctypes.addressof(res), ctypes.addressof(apx), *outs,
                                         apx_core.ctypes.data))
    hist = [(int(he[t]), int(hv[t])) for t in range(T)]
    r = ParResult(res, hist, [int(x) for x in hi[:T]], [(int(hn[t]), int(hm[t])) for t in range(T)],
                  [int(x) for x in hl[:T]], mask.astype(bool), core)
    if apx is not None:
        r.apx_core = apx_core
        r.apx_kmax = int(apx.apx_kmax)
        r.apx_level = int(apx.apx_level)
        r.apx_size = (int(apx.apx_n), int(apx.apx_nnz) // 2)
    return r


NOALLOC_SCRATCH_BYTES = 256 << 20  # DSG_NOALLOC_SCRATCH_BYTES of include/dsg.h


def par_run_noalloc(ctx: Context, offsets, adj, T: int, eps=(0, 1), variant: str = "peel",
                    validate: bool = True) -> ParResult:
    """dsg_par_run_noalloc: dsg_par_run on the library's static device scratch, for callers that cannot allocate.
    `offsets` and `adj` must already be int32 tensors on the context's device (this call copies nothing to the
    device); outputs land in host arrays."""
    import torch

    for x in (offsets, adj):
        if not (isinstance(x, torch.Tensor) and x.dtype == torch.int32 and x.device == ctx.torch_device
                and x.is_contiguous()):
            raise ValueError("par_run_noalloc takes contiguous int32 CSR tensors on the context's device")
    n, nnz = int(offsets.numel()) - 1, int(adj.numel())
    he = np.zeros(max(T, 1), dtype=np.int64)
    hv = np.zeros(max(T, 1), dtype=np.int64)
    hi = np.zeros(max(T, 1), dtype=np.int32)
    hn = np.zeros(max(T, 1), dtype=np.int32)
    hm = np.zeros(max(T, 1), dtype=np.int64)
    hl = np.zeros(max(T, 1), dtype=np.int32)
    mask = np.zeros(n, dtype=np.uint8)
    core = np.zeros(n, dtype=np.int32)
    num, den = parse_eps(eps)
    res = _ParResultC()
    _check(library().dsg_par_run_noalloc(ctx.handle, n, nnz, ctypes.c_void_p(offsets.data_ptr()),
                                         ctypes.c_void_p(adj.data_ptr() if nnz > 0 else 0), T, num, den,
                                         VARIANTS[variant], VALIDATE if validate else 0, ctypes.addressof(res),
                                         he.ctypes.data, hv.ctypes.data, hi.ctypes.data, hn.ctypes.data,
                                         hm.ctypes.data, hl.ctypes.data, mask.ctypes.data, core.ctypes.data))
    hist = [(int(he[t]), int(hv[t])) for t in range(T)]
    return ParResult(res, hist, [int(x) for x in hi[:T]], [(int(hn[t]), int(hm[t])) for t in range(T)],
                     [int(x) for x in hl[:T]], mask.astype(bool), core)


def coreness(ctx: Context, offsets, adj, validate: bool = True, timed: bool = False):
    """dsg_coreness: (core numbers int32[n], k_max, rounds of the pass, round-loop ms or None)."""
    import torch

    dev = ctx.torch_device
    o = Graph._dev_i32(offsets, dev)
    a = Graph._dev_i32(adj, dev)
    n, nnz = int(o.numel()) - 1, int(a.numel())
    nbytes = par_workspace_bytes(n, nnz, 1)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    aligned = (ws.data_ptr() + 255) // 256 * 256
    core = np.zeros(n, dtype=np.int32)
    kmax = ctypes.c_int32()
    rounds = ctypes.c_int32()
    ms = ctypes.c_float()
    _check(library().dsg_coreness(ctx.handle, n, nnz, ctypes.c_void_p(o.data_ptr()),
                                  ctypes.c_void_p(a.data_ptr() if nnz > 0 else 0), ctypes.c_void_p(aligned), nbytes,
                                  VALIDATE if validate else 0, core.ctypes.data, ctypes.addressof(kmax),
                                  ctypes.addressof(rounds), ctypes.addressof(ms) if timed else None))
    return core, int(kmax.value), int(rounds.value), (float(ms.value) if timed else None)
