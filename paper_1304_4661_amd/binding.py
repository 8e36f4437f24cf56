"""Python binding of ``libpll.so`` (the C ABI in include/pll.h).

Argument marshalling only: every step of the build and of the queries runs in
the library's HIP kernels.  If the library is missing this module raises; there
is no CPU fallback.  PyTorch is used only to hand device buffers and streams to
the library (``query_device``).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpll.so")

OK, E_INVAL, E_NOMEM, E_RANGE, E_DEVICE, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
INF = 255
WINF = 0xFFFFFFFF  # weighted distances: unreachable or 2^32 - 1 and more
MAX_TBP = 64
DEVICE_PTRS, VALIDATE, SYNC, PLAIN, PARENTS, DIRECTED = 1, 2, 4, 8, 16, 32

STAT_NAMES = [
    "n", "t_bp", "entries", "bp_used", "roots", "visited", "candidates", "windows",
    "retries", "bp_visited", "levels", "index_bytes", "build_ns", "bp_ns", "pruned_ns",
    "normal_tests", "label_scanned", "edges", "task_edges", "level_launches", "level_ns",
    "bp_direct", "bp_sets", "bp_checks", "improved", "touched", "filtered", "land_checks",
    "earlier_root", "expand_ns", "expand_direct", "expand_earlier", "expand_claims",
    "whole_graphs", "whole_ns", "whole_pairs",
]

EXPORTED = [
    "pll_build", "pll_build_batch", "pll_query", "pll_query_batch", "pll_sync",
    "pll_export_sizes", "pll_export", "pll_stats", "pll_level_trace", "pll_free", "pll_strerror",
    "pll_set_tuning", "pll_get_tuning", "pll_server_start", "pll_server_submit",
    "pll_server_done", "pll_server_stop", "pll_serve_bench", "pll_set_allocator",
    "pll_query_path", "pll_export_parents", "pll_export_in", "pll_build_weighted",
    "pll_query_weighted", "pll_export_weighted", "pll_autotune_query", "pll_export_in_parents",
    "pll_export_weighted_parents", "pll_server_submit_weighted", "pll_query_noalloc",
    "pll_query_noalloc_max_pairs", "pll_query_graph_create", "pll_query_graph_launch",
    "pll_query_graph_status", "pll_query_graph_free", "pll_autotune_build",
    "pll_build_query_batch",
]

SERVE_STATS = ["p50_us", "p99_us", "mean_us", "pairs_per_s", "requests_per_s", "seconds",
               "launches", "pairs_per_launch", "max_queue", "max_launch_us", "max_launch_at",
               "max_worker_pause_us"]


class PllError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        msg = _lib().pll_strerror(code).decode() if _LIB is not None else str(code)
        super().__init__(f"{what}: {msg} ({code})" if what else f"{msg} ({code})")
        self.code = code


_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run python -m paper_1304_4661_amd.build_lib first")
        lib = C.CDLL(LIB_PATH)
        P = C.c_void_p
        lib.pll_build.argtypes = [C.c_int32, P, P, P, C.c_int32, C.c_uint32, P, C.POINTER(C.c_void_p)]
        lib.pll_build.restype = C.c_int
        lib.pll_query.argtypes = [P, P, C.c_int64, P, C.c_uint32, P]
        lib.pll_query.restype = C.c_int
        lib.pll_build_batch.argtypes = [C.c_int32, P, P, P, P, C.c_int32, C.c_uint32, P,
                                        C.POINTER(C.c_void_p)]
        lib.pll_build_batch.restype = C.c_int
        lib.pll_build_query_batch.argtypes = [C.c_int32, P, P, P, P, C.c_int32, P, P, P,
                                              C.c_uint32, P, C.POINTER(C.c_void_p)]
        lib.pll_build_query_batch.restype = C.c_int
        lib.pll_query_batch.argtypes = [P, P, C.c_int64, P, C.c_uint32, P]
        lib.pll_query_batch.restype = C.c_int
        lib.pll_query_noalloc.argtypes = [P, P, C.c_int64, P, C.c_uint32, P]
        lib.pll_query_noalloc.restype = C.c_int
        lib.pll_autotune_build.argtypes = [C.c_int32, P, P, P, C.c_int32, C.c_uint32, P, P]
        lib.pll_autotune_build.restype = C.c_int
        lib.pll_query_graph_create.argtypes = [P, P, C.c_int64, P, C.c_uint32,
                                               C.POINTER(C.c_void_p)]
        lib.pll_query_graph_create.restype = C.c_int
        lib.pll_query_graph_launch.argtypes = [P, P]
        lib.pll_query_graph_launch.restype = C.c_int
        lib.pll_query_graph_status.argtypes = [P, P]
        lib.pll_query_graph_status.restype = C.c_int
        lib.pll_query_graph_free.argtypes = [P]
        lib.pll_query_graph_free.restype = None
        lib.pll_query_noalloc_max_pairs.argtypes = []
        lib.pll_query_noalloc_max_pairs.restype = C.c_int64
        lib.pll_sync.argtypes = [P, P]
        lib.pll_sync.restype = C.c_int
        lib.pll_export_sizes.argtypes = [P, C.c_int32, P, P, P]
        lib.pll_export_sizes.restype = C.c_int
        lib.pll_export.argtypes = [P, C.c_int32, P, P, P, P, P, P, P]
        lib.pll_export.restype = C.c_int
        lib.pll_stats.argtypes = [P, C.c_int32, P, C.c_int32]
        lib.pll_stats.restype = C.c_int
        lib.pll_query_path.argtypes = [P, P, C.c_int64, C.c_int32, P, P, C.c_uint32, P]
        lib.pll_query_path.restype = C.c_int
        lib.pll_export_parents.argtypes = [P, C.c_int32, P]
        lib.pll_export_parents.restype = C.c_int
        lib.pll_export_in_parents.argtypes = [P, C.c_int32, P]
        lib.pll_export_in_parents.restype = C.c_int
        lib.pll_export_in.argtypes = [P, C.c_int32, P, P, P, P]
        lib.pll_export_in.restype = C.c_int
        lib.pll_build_weighted.argtypes = [C.c_int32, P, P, P, P, C.c_uint32, P,
                                           C.POINTER(C.c_void_p)]
        lib.pll_build_weighted.restype = C.c_int
        lib.pll_query_weighted.argtypes = [P, P, C.c_int64, P, C.c_uint32, P]
        lib.pll_query_weighted.restype = C.c_int
        lib.pll_export_weighted.argtypes = [P, C.c_int32, P, P, P, P, P]
        lib.pll_export_weighted.restype = C.c_int
        lib.pll_export_weighted_parents.argtypes = [P, C.c_int32, P]
        lib.pll_export_weighted_parents.restype = C.c_int
        lib.pll_autotune_query.argtypes = [P, P, C.c_int64, C.c_uint32, P, P]
        lib.pll_autotune_query.restype = C.c_int
        lib.pll_level_trace.argtypes = [P, P, C.c_int64]
        lib.pll_level_trace.restype = C.c_int64
        lib.pll_free.argtypes = [P]
        lib.pll_free.restype = None
        lib.pll_strerror.argtypes = [C.c_int]
        lib.pll_strerror.restype = C.c_char_p
        lib.pll_set_allocator.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        lib.pll_set_allocator.restype = C.c_int
        lib.pll_set_tuning.argtypes = [C.c_char_p, C.c_int64]
        lib.pll_set_tuning.restype = C.c_int
        lib.pll_get_tuning.argtypes = [C.c_char_p]
        lib.pll_get_tuning.restype = C.c_int64
        lib.pll_server_start.argtypes = [P, C.c_int32, C.c_int64, C.POINTER(C.c_void_p)]
        lib.pll_server_start.restype = C.c_int
        lib.pll_server_submit.argtypes = [P, P, C.c_int64, P, C.POINTER(C.c_int64)]
        lib.pll_server_submit.restype = C.c_int
        lib.pll_server_submit_weighted.argtypes = [P, P, C.c_int64, P, C.POINTER(C.c_int64)]
        lib.pll_server_submit_weighted.restype = C.c_int
        lib.pll_server_done.argtypes = [P, C.c_int64, C.c_int32, C.POINTER(C.c_double)]
        lib.pll_server_done.restype = C.c_int
        lib.pll_server_stop.argtypes = [P, P, C.c_int32]
        lib.pll_server_stop.restype = C.c_int
        lib.pll_serve_bench.argtypes = [P, C.c_double, C.c_int64, C.c_int64, C.c_uint64,
                                        C.c_int32, C.c_int64, P, C.c_int32]
        lib.pll_serve_bench.restype = C.c_int
        _LIB = lib
    return _LIB


def library():
    """The loaded ctypes library (raises if it is not built)."""
    return _lib()


def _ptr(a):
    return None if a is None else C.c_void_p(a.ctypes.data)


def _check(rc: int, what: str):
    if rc != OK:
        raise PllError(rc, what)


def noalloc_max_pairs() -> int:
    """Largest host-pointer request of pll_query_noalloc."""
    return int(_lib().pll_query_noalloc_max_pairs())


def set_tuning(key: str, value: int):
    _check(_lib().pll_set_tuning(key.encode(), int(value)), f"set_tuning({key})")


def get_tuning(key: str) -> int:
    return int(_lib().pll_get_tuning(key.encode()))


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)
_allocator_refs = []  # keeps the installed callbacks alive


def use_torch_allocator(enable: bool = True):
    """Route the library's device allocations through torch's caching
    allocator (memory then shows in torch.cuda.memory_allocated and is
    reused by torch after pll_free), or back to hipMalloc."""
    lib = _lib()
    if not enable:
        _check(lib.pll_set_allocator(None, None, None), "set_allocator")
        _allocator_refs.clear()
        return
    import torch

    dev = torch.cuda.current_device()

    def _alloc(nbytes, stream, _ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream or 0)
        except Exception:  # out of memory: the library reports PLL_E_NOMEM
            return None

    def _free(ptr, _stream, _ctx):
        torch.cuda.caching_allocator_delete(ptr)

    a, f = ALLOC_FN(_alloc), FREE_FN(_free)
    _check(lib.pll_set_allocator(C.cast(a, C.c_void_p), C.cast(f, C.c_void_p), None),
           "set_allocator")
    _allocator_refs[:] = [a, f]


class Index:
    """A device-resident index made by :func:`build`."""

    def __init__(self, handle: C.c_void_p, weighted: bool = False):
        self._h = handle
        self.weighted = weighted  # made by build_weighted (32-bit distances)

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h is not None and self._h.value:
            _lib().pll_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def query(self, pairs, plain: bool = False) -> np.ndarray:
        """Host arrays in and out: ``pairs`` int32[q, 2] ids -> uint8[q]."""
        pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
        out = np.zeros(len(pairs), np.uint8)
        flags = PLAIN if plain else 0
        _check(_lib().pll_query(self._h, _ptr(pairs), len(pairs), _ptr(out), flags, None), "query")
        return out

    def query_device(self, pairs, out, stream=None, plain: bool = False, sync: bool = False):
        """Device tensors (torch): ``pairs`` int32 [q, 2] and ``out`` uint8 [q]
        on the GPU; runs on ``stream`` (a torch stream, default current)."""
        import torch

        assert pairs.dtype == torch.int32 and out.dtype == torch.uint8
        assert pairs.is_cuda and out.is_cuda and pairs.is_contiguous() and out.is_contiguous()
        q = out.numel()
        assert pairs.numel() == 2 * q
        if stream is None:
            stream = torch.cuda.current_stream()
        flags = DEVICE_PTRS | (PLAIN if plain else 0) | (SYNC if sync else 0)
        _check(_lib().pll_query(self._h, C.c_void_p(pairs.data_ptr()), q,
                                C.c_void_p(out.data_ptr()), flags,
                                C.c_void_p(stream.cuda_stream)), "query_device")

    def query_noalloc(self, pairs, out=None, stream=None, plain: bool = False,
                      sync: bool = True):
        """pll_query_noalloc: host arrays (``pairs`` int32[q, 2] -> new
        uint8[q]) or, with ``out`` given, torch device tensors as in
        query_device."""
        flags = PLAIN if plain else 0
        if out is None:
            pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
            res = np.zeros(len(pairs), np.uint8)
            _check(_lib().pll_query_noalloc(self._h, _ptr(pairs), len(pairs), _ptr(res), flags,
                                            None), "query_noalloc")
            return res
        import torch

        assert pairs.dtype == torch.int32 and out.dtype == torch.uint8
        assert pairs.is_cuda and out.is_cuda and pairs.is_contiguous() and out.is_contiguous()
        q = out.numel()
        assert pairs.numel() == 2 * q
        if stream is None:
            stream = torch.cuda.current_stream()
        flags |= DEVICE_PTRS | (SYNC if sync else 0)
        _check(_lib().pll_query_noalloc(self._h, C.c_void_p(pairs.data_ptr()), q,
                                        C.c_void_p(out.data_ptr()), flags,
                                        C.c_void_p(stream.cuda_stream)), "query_noalloc")
        return out

    def sync(self, stream=None):
        s = None if stream is None else C.c_void_p(stream.cuda_stream)
        _check(_lib().pll_sync(self._h, s), "sync")

    def sizes(self, graph: int = 0):
        n, e, t = C.c_int64(), C.c_int64(), C.c_int32()
        _check(_lib().pll_export_sizes(self._h, graph, C.byref(n), C.byref(e), C.byref(t)),
               "sizes")
        return n.value, e.value, t.value

    def query_path(self, pairs, max_len: int = 64):
        """Shortest paths (index built with parents=True): ``pairs``
        int32[q, 2] ids -> (paths int32[q, max_len] ids, lens int32[q]);
        lens = d+1, 0 if unreachable, -(d+1) if max_len is too small.
        Unwritten cells are -1."""
        pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
        paths = np.full((len(pairs), max_len), -1, np.int32)
        lens = np.zeros(len(pairs), np.int32)
        _check(_lib().pll_query_path(self._h, _ptr(pairs), len(pairs), int(max_len), _ptr(paths),
                                     _ptr(lens), 0, None), "query_path")
        return paths, lens

    def query_path_device(self, pairs, paths, lens, stream=None, sync: bool = False):
        """Device tensors (torch): ``pairs`` int32 [q, 2], ``paths`` int32
        [q, max_len], ``lens`` int32 [q]; runs on ``stream``."""
        import torch

        assert pairs.dtype == torch.int32 and paths.dtype == torch.int32 and lens.dtype == torch.int32
        assert pairs.is_cuda and paths.is_cuda and lens.is_cuda
        assert pairs.is_contiguous() and paths.is_contiguous() and lens.is_contiguous()
        q = lens.numel()
        assert pairs.numel() == 2 * q and paths.dim() == 2 and paths.shape[0] == q
        if stream is None:
            stream = torch.cuda.current_stream()
        flags = DEVICE_PTRS | (SYNC if sync else 0)
        _check(_lib().pll_query_path(self._h, C.c_void_p(pairs.data_ptr()), q, int(paths.shape[1]),
                                     C.c_void_p(paths.data_ptr()), C.c_void_p(lens.data_ptr()),
                                     flags, C.c_void_p(stream.cuda_stream)), "query_path_device")

    def export_in(self, graph: int = 0) -> dict:
        """L_IN of a directed index (off, hub, dist; local ranks, no
        sentinels); ``export`` gives L_OUT."""
        n, _, _ = self.sizes(graph)
        ne = C.c_int64()
        _check(_lib().pll_export_in(self._h, int(graph), C.byref(ne), None, None, None), "export_in")
        off = np.zeros(n + 1, np.int64)
        hub = np.zeros(ne.value, np.uint32)
        dist = np.zeros(ne.value, np.uint8)
        _check(_lib().pll_export_in(self._h, int(graph), None, _ptr(off), _ptr(hub), _ptr(dist)),
               "export_in")
        return {"off": off, "hub": hub, "dist": dist}

    def export_parents(self, graph: int = 0) -> np.ndarray:
        """Parents of the exported entries of one graph, as local ranks."""
        _, e, _ = self.sizes(graph)
        par = np.zeros(e, np.uint32)
        _check(_lib().pll_export_parents(self._h, int(graph), _ptr(par)), "export_parents")
        return par

    def export_in_parents(self, graph: int = 0) -> np.ndarray:
        """Parents of the L_IN entries of a directed index built with
        parents, in export_in's order, as local ranks."""
        ne = C.c_int64()
        _check(_lib().pll_export_in(self._h, int(graph), C.byref(ne), None, None, None),
               "export_in")
        par = np.zeros(ne.value, np.uint32)
        if ne.value:
            _check(_lib().pll_export_in_parents(self._h, int(graph), _ptr(par)),
                   "export_in_parents")
        return par

    def export(self, graph: int = 0) -> dict:
        """Canonical host copy of one graph: local rank order, no sentinels
        (see include/pll.h)."""
        n, e, t = self.sizes(graph)
        out = {
            "off": np.zeros(n + 1, np.int64), "hub": np.zeros(e, np.uint32),
            "dist": np.zeros(e, np.uint8), "bp_d": np.zeros((n, t), np.uint8),
            "bp_m1": np.zeros((n, t), np.uint64), "bp_0": np.zeros((n, t), np.uint64),
            "rank": np.zeros(n, np.int32),
        }
        _check(_lib().pll_export(self._h, graph, *(_ptr(out[k]) for k in
                                                ("off", "hub", "dist", "bp_d", "bp_m1", "bp_0",
                                                 "rank"))), "export")
        return out

    def label_lengths(self, graph: int = 0):
        """(rank int32[n]: id -> rank, lengths int64[n] of the normal labels
        by rank, no sentinels), without copying the labels."""
        n, _, _ = self.sizes(graph)
        off = np.zeros(n + 1, np.int64)
        rank = np.zeros(n, np.int32)
        _check(_lib().pll_export(self._h, graph, _ptr(off), None, None, None, None, None,
                                 _ptr(rank)), "export")
        return rank, np.diff(off)

    def query_weighted(self, pairs, plain: bool = False) -> np.ndarray:
        """Weighted index, host arrays: ``pairs`` int32[q, 2] ids ->
        uint32[q] (WINF: unreachable or too far)."""
        pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
        out = np.zeros(len(pairs), np.uint32)
        flags = PLAIN if plain else 0
        _check(_lib().pll_query_weighted(self._h, _ptr(pairs), len(pairs), _ptr(out), flags, None),
               "query_weighted")
        return out

    def query_weighted_device(self, pairs, out, stream=None, plain: bool = False,
                              sync: bool = False):
        """Weighted index, device tensors: ``pairs`` int32 [q, 2], ``out``
        int32 [q] (read as uint32) on the GPU; runs on ``stream``."""
        import torch

        assert pairs.dtype == torch.int32 and out.dtype == torch.int32
        assert pairs.is_cuda and out.is_cuda and pairs.is_contiguous() and out.is_contiguous()
        q = out.numel()
        assert pairs.numel() == 2 * q
        if stream is None:
            stream = torch.cuda.current_stream()
        flags = DEVICE_PTRS | (PLAIN if plain else 0) | (SYNC if sync else 0)
        _check(_lib().pll_query_weighted(self._h, C.c_void_p(pairs.data_ptr()), q,
                                         C.c_void_p(out.data_ptr()), flags,
                                         C.c_void_p(stream.cuda_stream)), "query_weighted_device")

    def export_weighted(self, side: int = 0) -> dict:
        """Labels of a weighted index in rank order, no sentinels: side 0 is
        L (L_OUT of a digraph), side 1 L_IN."""
        n, _, _ = self.sizes(0)
        ne = C.c_int64()
        _check(_lib().pll_export_weighted(self._h, int(side), C.byref(ne), None, None, None, None),
               "export_weighted")
        out = {"off": np.zeros(n + 1, np.int64), "hub": np.zeros(ne.value, np.uint32),
               "dist": np.zeros(ne.value, np.uint32), "rank": np.zeros(n, np.int32)}
        _check(_lib().pll_export_weighted(self._h, int(side), None, _ptr(out["off"]),
                                          _ptr(out["hub"]), _ptr(out["dist"]), _ptr(out["rank"])),
               "export_weighted")
        return out

    def autotune_query(self, pairs, stream=None) -> int:
        """Time the batched query kernel at 16/32/64 lanes per pair on these
        sample pairs (numpy int32[q, 2], or a torch device tensor) and keep
        the fastest as the "qgroup" knob; returns it."""
        best = C.c_int32()
        if isinstance(pairs, np.ndarray):
            pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
            _check(_lib().pll_autotune_query(self._h, _ptr(pairs), len(pairs), 0, None,
                                             C.byref(best)), "autotune_query")
        else:
            import torch

            assert pairs.dtype == torch.int32 and pairs.is_cuda and pairs.is_contiguous()
            if stream is None:
                stream = torch.cuda.current_stream()
            _check(_lib().pll_autotune_query(self._h, C.c_void_p(pairs.data_ptr()),
                                             pairs.numel() // 2, DEVICE_PTRS,
                                             C.c_void_p(stream.cuda_stream), C.byref(best)),
                   "autotune_query")
        return best.value

    def export_weighted_parents(self, side: int = 0) -> np.ndarray:
        """Parents (ranks) of export_weighted(side)'s entries (weighted
        index built with parents)."""
        ne = C.c_int64()
        _check(_lib().pll_export_weighted(self._h, int(side), C.byref(ne), None, None, None, None),
               "export_weighted")
        par = np.zeros(ne.value, np.uint32)
        if ne.value:
            _check(_lib().pll_export_weighted_parents(self._h, int(side), _ptr(par)),
                   "export_weighted_parents")
        return par

    TRACE_COLS = ["window", "first_root", "roots", "level", "entries", "candidates", "ns"]

    def level_trace(self) -> np.ndarray:
        """Per-level profile of the pruned phase (rows of TRACE_COLS); empty
        unless the "profile" knob was set during the build."""
        k = len(self.TRACE_COLS)
        nrows = int(_lib().pll_level_trace(self._h, None, 0))
        if nrows < 0:
            _check(nrows, "level_trace")
        out = np.zeros((nrows, k), np.int64)
        if nrows:
            _lib().pll_level_trace(self._h, _ptr(out), nrows)
        return out

    def stats(self) -> dict:
        c = np.zeros(len(STAT_NAMES), np.int64)
        _check(_lib().pll_stats(self._h, 0, _ptr(c), len(c)), "stats")
        return {k: int(v) for k, v in zip(STAT_NAMES, c)}


def build_device(row_ptr, col, order, t_bp: int, plain: bool = False, stream=None,
                 parents: bool = False, directed: bool = False) -> Index:
    """Build from device tensors (torch, int32, contiguous, on the GPU)."""
    import torch

    for a in (row_ptr, col, order):
        assert a.dtype == torch.int32 and a.is_cuda and a.is_contiguous()
    n = order.numel()
    if row_ptr.numel() != n + 1:
        raise PllError(E_INVAL, "build_device: row_ptr length")
    if stream is None:
        stream = torch.cuda.current_stream()
    flags = (DEVICE_PTRS | (PLAIN if plain else 0) | (PARENTS if parents else 0)
             | (DIRECTED if directed else 0))
    h = C.c_void_p()
    rc = _lib().pll_build(n, C.c_void_p(row_ptr.data_ptr()), C.c_void_p(col.data_ptr()),
                          C.c_void_p(order.data_ptr()), int(t_bp), flags,
                          C.c_void_p(stream.cuda_stream), C.byref(h))
    _check(rc, "build_device")
    return Index(h)


def autotune_build(row_ptr, col, order, t_bp: int, stream=None) -> dict:
    """pll_autotune_build on device tensors (torch, int32, on the GPU): sets
    the frontier-tile knobs to the fastest found and returns them."""
    import torch

    for a in (row_ptr, col, order):
        assert a.dtype == torch.int32 and a.is_cuda and a.is_contiguous()
    n = order.numel()
    if stream is None:
        stream = torch.cuda.current_stream()
    best = np.zeros(4, np.int64)
    _check(_lib().pll_autotune_build(n, C.c_void_p(row_ptr.data_ptr()), C.c_void_p(col.data_ptr()),
                                     C.c_void_p(order.data_ptr()), int(t_bp), DEVICE_PTRS,
                                     C.c_void_p(stream.cuda_stream), _ptr(best)),
           "autotune_build")
    return dict(zip(("xgroup", "chunk", "window_work", "sort_level"), (int(x) for x in best)))


def build_batch(vtx_off, row_ptr, col, order, t_bp: int, validate: bool = False,
                plain: bool = False, stream=None, device: bool = False,
                parents: bool = False, directed: bool = False) -> Index:
    """Build the indexes of a batch of graphs (see include/pll.h).  With
    device=True, row_ptr/col/order are torch device tensors."""
    vtx_off = np.ascontiguousarray(vtx_off, dtype=np.int64)
    G = len(vtx_off) - 1
    flags = ((VALIDATE if validate else 0) | (PLAIN if plain else 0) | (PARENTS if parents else 0)
             | (DIRECTED if directed else 0))
    h = C.c_void_p()
    if device:
        import torch

        for a in (row_ptr, col, order):
            assert a.dtype == torch.int32 and a.is_cuda and a.is_contiguous()
        if stream is None:
            stream = torch.cuda.current_stream()
        args = [C.c_void_p(a.data_ptr()) for a in (row_ptr, col, order)]
        flags |= DEVICE_PTRS
    else:
        row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
        col = np.ascontiguousarray(col, dtype=np.int32)
        order = np.ascontiguousarray(order, dtype=np.int32)
        args = [_ptr(row_ptr), _ptr(col), _ptr(order)]
    s = None if stream is None else C.c_void_p(stream.cuda_stream)
    rc = _lib().pll_build_batch(G, _ptr(vtx_off), *args, int(t_bp), flags, s, C.byref(h))
    _check(rc, "build_batch")
    return Index(h)


def build_query_batch(vtx_off, row_ptr, col, order, t_bp: int, qoff, pairs, out=None,
                      validate: bool = False, stream=None, device: bool = False):
    """Build a batch and answer each graph's pairs in the same call (see
    include/pll.h): returns (Index, answers).  qoff: int64[G+1] offsets of
    each graph's pairs.  With device=True, row_ptr/col/order/pairs (and out,
    if given) are torch device tensors and the answers are a device tensor
    complete when the call returns."""
    vtx_off = np.ascontiguousarray(vtx_off, dtype=np.int64)
    qoff = np.ascontiguousarray(qoff, dtype=np.int64)
    G = len(vtx_off) - 1
    if len(qoff) != G + 1:
        raise ValueError("qoff needs one offset per graph plus one")
    q = int(qoff[-1]) if G > 0 else 0
    if pairs is not None and (pairs.numel() if device else np.size(pairs)) < 2 * q:
        raise ValueError(f"pairs holds fewer than qoff[-1] = {q} pairs")
    if out is not None and (out.numel() if device else np.size(out)) < q:
        raise ValueError(f"out holds fewer than qoff[-1] = {q} answers")
    flags = VALIDATE if validate else 0
    h = C.c_void_p()
    if device:
        import torch

        for a in (row_ptr, col, order, pairs):
            assert a.dtype == torch.int32 and a.is_cuda and a.is_contiguous()
        if out is None:
            out = torch.empty(int(qoff[-1]) if G > 0 else 0, dtype=torch.uint8,
                              device=pairs.device)
        if stream is None:
            stream = torch.cuda.current_stream()
        args = [C.c_void_p(a.data_ptr()) for a in (row_ptr, col, order)]
        pq, po = C.c_void_p(pairs.data_ptr()), C.c_void_p(out.data_ptr())
        flags |= DEVICE_PTRS | SYNC
    else:
        row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
        col = np.ascontiguousarray(col, dtype=np.int32)
        order = np.ascontiguousarray(order, dtype=np.int32)
        pairs = np.ascontiguousarray(pairs, dtype=np.int32)
        if out is None:
            out = np.empty(int(qoff[-1]) if G > 0 else 0, np.uint8)
        args = [_ptr(row_ptr), _ptr(col), _ptr(order)]
        pq, po = _ptr(pairs), _ptr(out)
    s = None if stream is None else C.c_void_p(stream.cuda_stream)
    rc = _lib().pll_build_query_batch(G, _ptr(vtx_off), *args, int(t_bp), _ptr(qoff), pq, po,
                                      flags, s, C.byref(h))
    _check(rc, "build_query_batch")
    return Index(h), out


def build(row_ptr, col, order, t_bp: int, validate: bool = False, plain: bool = False,
          stream=None, parents: bool = False, directed: bool = False) -> Index:
    """Build the index of one graph (host CSR and order, see include/pll.h)."""
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    order = np.ascontiguousarray(order, dtype=np.int32)
    n = len(order)
    if len(row_ptr) != n + 1:
        raise PllError(E_INVAL, "build: row_ptr length")
    flags = ((VALIDATE if validate else 0) | (PLAIN if plain else 0) | (PARENTS if parents else 0)
             | (DIRECTED if directed else 0))
    h = C.c_void_p()
    s = None if stream is None else C.c_void_p(stream.cuda_stream)
    rc = _lib().pll_build(n, _ptr(row_ptr), _ptr(col), _ptr(order), int(t_bp), flags, s,
                          C.byref(h))
    _check(rc, "build")
    return Index(h)


def build_weighted(row_ptr, col, wgt, order, directed: bool = False, plain: bool = False,
                   validate: bool = False, stream=None, device: bool = False,
                   parents: bool = False) -> Index:
    """Pruned Dijkstra index of a weighted graph (Section 6; see
    include/pll.h).  Host arrays, or torch device tensors with device=True
    (wgt as int32 or uint32-valued int32 tensor)."""
    flags = ((VALIDATE if validate else 0) | (PLAIN if plain else 0)
             | (DIRECTED if directed else 0) | (PARENTS if parents else 0))
    h = C.c_void_p()
    if device:
        import torch

        for a in (row_ptr, col, order, wgt):
            assert a.dtype == torch.int32 and a.is_cuda and a.is_contiguous()
        n = order.numel()
        if row_ptr.numel() != n + 1 or wgt.numel() != col.numel():
            raise PllError(E_INVAL, "build_weighted: array lengths")
        if stream is None:
            stream = torch.cuda.current_stream()
        args = [C.c_void_p(a.data_ptr()) for a in (row_ptr, col, wgt, order)]
        flags |= DEVICE_PTRS
    else:
        row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
        col = np.ascontiguousarray(col, dtype=np.int32)
        wgt = np.ascontiguousarray(wgt, dtype=np.uint32)
        order = np.ascontiguousarray(order, dtype=np.int32)
        n = len(order)
        if len(row_ptr) != n + 1 or len(wgt) != len(col):
            raise PllError(E_INVAL, "build_weighted: array lengths")
        args = [_ptr(row_ptr), _ptr(col), _ptr(wgt), _ptr(order)]
    s = None if stream is None else C.c_void_p(stream.cuda_stream)
    _check(_lib().pll_build_weighted(n, *args, flags, s, C.byref(h)), "build_weighted")
    return Index(h, weighted=True)


class QueryGraph:
    """A batch of queries on fixed device tensors recorded as a HIP graph
    (pll_query_graph_*): launch() replays it, status() waits and reports an
    out-of-range id of the last replay."""

    def __init__(self, index: Index, pairs, out, plain: bool = False):
        import torch

        assert pairs.dtype == torch.int32 and out.dtype == torch.uint8
        assert pairs.is_cuda and out.is_cuda and pairs.is_contiguous() and out.is_contiguous()
        assert pairs.numel() == 2 * out.numel()
        self.index, self.pairs, self.out = index, pairs, out  # kept alive with the graph
        h = C.c_void_p()
        flags = DEVICE_PTRS | (PLAIN if plain else 0)
        _check(_lib().pll_query_graph_create(index.handle, C.c_void_p(pairs.data_ptr()),
                                             out.numel(), C.c_void_p(out.data_ptr()), flags,
                                             C.byref(h)), "query_graph_create")
        self._h = h

    def launch(self, stream=None):
        import torch

        stream = stream or torch.cuda.current_stream()
        _check(_lib().pll_query_graph_launch(self._h, C.c_void_p(stream.cuda_stream)),
               "query_graph_launch")

    def status(self, stream=None):
        import torch

        stream = stream or torch.cuda.current_stream()
        _check(_lib().pll_query_graph_status(self._h, C.c_void_p(stream.cuda_stream)),
               "query_graph_status")

    def close(self):
        h, self._h = getattr(self, "_h", None), None
        if h is not None:
            _lib().pll_query_graph_free(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching query server over an index (see include/pll.h).
    Submitted arrays are kept referenced until the request is answered."""

    def __init__(self, index: Index, nslots: int = 4, slot_pairs: int = 1 << 16):
        self.index = index
        h = C.c_void_p()
        _check(_lib().pll_server_start(index.handle, nslots, slot_pairs, C.byref(h)),
               "server_start")
        self._h = h
        self._keep = {}

    def submit(self, pairs) -> int:
        """Queue pairs; answers are uint8 (uint32 on a weighted index)."""
        pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
        t = C.c_int64()
        if self.index.weighted:
            out = np.zeros(len(pairs), np.uint32)
            _check(_lib().pll_server_submit_weighted(self._h, _ptr(pairs), len(pairs), _ptr(out),
                                                     C.byref(t)), "server_submit_weighted")
        else:
            out = np.zeros(len(pairs), np.uint8)
            _check(_lib().pll_server_submit(self._h, _ptr(pairs), len(pairs), _ptr(out),
                                            C.byref(t)), "server_submit")
        self._keep[t.value] = (pairs, out)
        return t.value

    def result(self, ticket: int, wait: bool = True):
        """(answers or None, latency_us or None)."""
        lat = C.c_double()
        r = _lib().pll_server_done(self._h, ticket, 1 if wait else 0, C.byref(lat))
        if r < 0:
            raise PllError(r, "server_done")
        if r == 0:
            return None, None
        # answered: the library recycles the request's record, and the
        # arrays are no longer needed here
        return self._keep.pop(ticket)[1], lat.value

    def stop(self) -> dict:
        st = np.zeros(7, np.int64)
        h, self._h = self._h, None
        if h is not None:
            _check(_lib().pll_server_stop(h, _ptr(st), 7), "server_stop")
        return {"launches": int(st[0]), "pairs": int(st[1]), "max_queue": int(st[2]),
                "records": int(st[6])}

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass


def serve_bench(index: Index, rate: float, nreq: int, max_batch: int = 4096, seed: int = 105,
                nslots: int = 4, slot_pairs: int = 1 << 16) -> dict:
    st = np.zeros(len(SERVE_STATS), np.float64)
    _check(_lib().pll_serve_bench(index.handle, float(rate), int(nreq), int(max_batch),
                                  int(seed), int(nslots), int(slot_pairs), _ptr(st), len(st)),
           "serve_bench")
    return {k: float(v) for k, v in zip(SERVE_STATS, st)}
