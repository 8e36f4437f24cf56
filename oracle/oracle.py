"""ctypes wrapper around the plain C oracle (``pll_oracle.c``).

Test infrastructure only: see the package docstring.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pll_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")

COUNTER_NAMES = [
    "n", "t_bp", "entries", "bp_used", "roots", "visited", "labeled", "edges",
    "bp_pruned", "normal_tests", "label_scanned", "root_staged", "bp_reached",
    "bp_edges", "bp_e0", "bp_e1", "max_dist",
]

_ERRORS = {-1: "invalid argument", -2: "out of memory", -3: "distance out of range"}


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle error {code}: {_ERRORS.get(code, 'unknown')}")
        self.code = code


def build_library(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _configure(lib):
    if True:
        P = C.c_void_p
        lib.orc_build.argtypes = [C.c_int32, P, P, P, C.c_int32, C.c_uint32, C.POINTER(C.c_void_p)]
        lib.orc_build.restype = C.c_int
        lib.orc_build_prefix.argtypes = [C.c_int32, P, P, P, C.c_int32, C.c_uint32, C.c_int32,
                                         C.POINTER(C.c_void_p)]
        lib.orc_build_prefix.restype = C.c_int
        lib.orc_times.argtypes = [C.c_void_p, P, P, P, P, C.c_int32]
        lib.orc_times.restype = C.c_int32
        lib.orc_query.argtypes = [C.c_void_p, P, C.c_int64, P]
        lib.orc_query.restype = C.c_int
        lib.orc_free.argtypes = [C.c_void_p]
        lib.orc_free.restype = None
        lib.orc_ncounters.argtypes = []
        lib.orc_ncounters.restype = C.c_int32
        lib.orc_counters.argtypes = [C.c_void_p, P, C.c_int32]
        lib.orc_counters.restype = C.c_int
        lib.orc_num_entries.argtypes = [C.c_void_p]
        lib.orc_num_entries.restype = C.c_int64
        lib.orc_export.argtypes = [C.c_void_p] + [P] * 10
        lib.orc_export.restype = C.c_int
        lib.orc_query_parts.argtypes = [C.c_void_p, P, C.c_int64, P, P]
        lib.orc_query_parts.restype = C.c_int
        lib.orc_root_counts.argtypes = [C.c_void_p, P, P]
        lib.orc_root_counts.restype = C.c_int
        lib.orc_paths.argtypes = [C.c_void_p, P, C.c_int64, C.c_int32, P, P]
        lib.orc_paths.restype = C.c_int
        lib.orc_export_parents.argtypes = [C.c_void_p, P]
        lib.orc_export_parents.restype = C.c_int
        lib.orc_export_in_parents.argtypes = [C.c_void_p, P]
        lib.orc_export_in_parents.restype = C.c_int
        lib.orc_build_directed.argtypes = [C.c_int32, P, P, P, C.POINTER(C.c_void_p)]
        lib.orc_build_directed.restype = C.c_int
        lib.orc_export_in.argtypes = [C.c_void_p, P, P, P, P]
        lib.orc_export_in.restype = C.c_int
        lib.orc_build_weighted.argtypes = [C.c_int32, P, P, P, P, C.c_uint32,
                                           C.POINTER(C.c_void_p)]
        lib.orc_build_weighted.restype = C.c_int
        lib.orc_wquery.argtypes = [C.c_void_p, P, C.c_int64, P]
        lib.orc_wquery.restype = C.c_int
        lib.orc_wfree.argtypes = [C.c_void_p]
        lib.orc_wfree.restype = None
        lib.orc_wncounters.argtypes = []
        lib.orc_wncounters.restype = C.c_int32
        lib.orc_wcounters.argtypes = [C.c_void_p, P, C.c_int32]
        lib.orc_wcounters.restype = C.c_int
        lib.orc_wexport.argtypes = [C.c_void_p, C.c_int32, P, P, P, P, P]
        lib.orc_wexport.restype = C.c_int
        lib.orc_wpaths.argtypes = [C.c_void_p, P, C.c_int64, C.c_int32, P, P]
        lib.orc_wpaths.restype = C.c_int
        lib.orc_wexport_parents.argtypes = [C.c_void_p, C.c_int32, P]
        lib.orc_wexport_parents.restype = C.c_int
    return lib


def _load():
    global _lib
    if _lib is None:
        _lib = _configure(C.CDLL(build_library()))
    return _lib


def load_variant(source: str, workdir: str):
    """Compile a modified copy of the oracle source (for tests that plant a
    mistake in the oracle and check that the pins catch it)."""
    import hashlib
    tag = hashlib.sha256(source.encode()).hexdigest()[:16]
    src = os.path.join(workdir, f"orc_{tag}.c")
    lib = os.path.join(workdir, f"liborc_{tag}.so")
    with open(src, "w") as f:
        f.write(source)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", lib, src])
    return _configure(C.CDLL(lib))


def source_text() -> str:
    with open(_SRC) as f:
        return f.read()


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


@dataclass
class OracleIndex:
    """Exported oracle index: vertices in rank order, no sentinels."""
    n: int
    t_bp: int
    off: np.ndarray      # int64[n+1]
    hub: np.ndarray      # uint32[entries] (ranks)
    dist: np.ndarray     # uint8[entries]
    bp_d: np.ndarray     # uint8[n, t_bp]
    bp_m1: np.ndarray    # uint64[n, t_bp]
    bp_0: np.ndarray     # uint64[n, t_bp]
    rank: np.ndarray     # int32[n]: rank of input id
    bp_root: np.ndarray  # int32[t_bp]: rank of root, -1 if empty
    bp_nsel: np.ndarray  # int32[t_bp]
    bp_sel: np.ndarray   # int32[t_bp, 64]: ranks of chosen neighbours
    par: np.ndarray | None = None  # uint32[entries]: parent (rank) of each entry's vertex
    counters: dict = field(default_factory=dict)
    root_visited: np.ndarray | None = None  # int32[n] per rank (pruned phase)
    root_labeled: np.ndarray | None = None  # int32[n] per rank
    # wall clock of the build: {"bp_s", "pruned_s", "ck_step", "ck_s"} where
    # ck_s[i] is the pruned-phase time before the root of rank i*ck_step
    times: dict = field(default_factory=dict)
    _handle: C.c_void_p | None = None

    def label(self, r: int):
        """(hubs, dists) of the vertex of rank r."""
        a, b = int(self.off[r]), int(self.off[r + 1])
        return self.hub[a:b], self.dist[a:b]

    _lib: object = None

    def close(self):
        if self._handle is not None:
            (self._lib or _load()).orc_free(self._handle)
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build(row_ptr, col, order, t_bp: int, check_symmetric: bool = True, lib=None,
          root_limit: int | None = None) -> OracleIndex:
    """Oracle index of an undirected graph.  ``root_limit``: run the pruned
    BFSs of ranks ``0..root_limit-1`` only (Theorem 4.1: the result is the
    full labels' entries whose hub ranks below ``root_limit``)."""
    lib = lib or _load()
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    order = np.ascontiguousarray(order, dtype=np.int32)
    n = len(order)
    if len(row_ptr) != n + 1:
        raise OracleError(-1)
    h = C.c_void_p()
    if root_limit is None:
        rc = lib.orc_build(n, _ptr(row_ptr), _ptr(col), _ptr(order), int(t_bp),
                           1 if check_symmetric else 0, C.byref(h))
    else:
        rc = lib.orc_build_prefix(n, _ptr(row_ptr), _ptr(col), _ptr(order), int(t_bp),
                                  1 if check_symmetric else 0, int(root_limit), C.byref(h))
    if rc != 0:
        raise OracleError(rc)
    ne = lib.orc_num_entries(h)
    tb = max(int(t_bp), 0)
    idx = OracleIndex(
        n=n, t_bp=tb,
        off=np.zeros(n + 1, np.int64), hub=np.zeros(ne, np.uint32), dist=np.zeros(ne, np.uint8),
        bp_d=np.zeros((n, tb), np.uint8), bp_m1=np.zeros((n, tb), np.uint64),
        bp_0=np.zeros((n, tb), np.uint64), rank=np.zeros(n, np.int32),
        bp_root=np.zeros(tb, np.int32), bp_nsel=np.zeros(tb, np.int32),
        bp_sel=np.zeros((tb, 64), np.int32), _handle=h)
    idx._lib = lib
    idx.par = np.zeros(ne, np.uint32)
    if ne:
        lib.orc_export_parents(h, _ptr(idx.par))
    lib.orc_export(h, _ptr(idx.off), _ptr(idx.hub), _ptr(idx.dist), _ptr(idx.bp_d),
                   _ptr(idx.bp_m1), _ptr(idx.bp_0), _ptr(idx.rank), _ptr(idx.bp_root),
                   _ptr(idx.bp_nsel), _ptr(idx.bp_sel))
    nc = lib.orc_ncounters()
    cnt = np.zeros(nc, np.int64)
    lib.orc_counters(h, _ptr(cnt), nc)
    idx.counters = {k: int(v) for k, v in zip(COUNTER_NAMES, cnt)}
    idx.root_visited = np.zeros(n, np.int32)
    idx.root_labeled = np.zeros(n, np.int32)
    lib.orc_root_counts(h, _ptr(idx.root_visited), _ptr(idx.root_labeled))
    if hasattr(lib, "orc_times"):
        bp_ns, pr_ns, step = C.c_int64(), C.c_int64(), C.c_int32()
        ck = np.zeros(1025, np.int64)
        nck = lib.orc_times(h, C.byref(bp_ns), C.byref(pr_ns), C.byref(step), _ptr(ck), 1025)
        idx.times = {"bp_s": bp_ns.value * 1e-9, "pruned_s": pr_ns.value * 1e-9,
                     "ck_step": int(step.value), "ck_s": (ck[:max(nck, 0)] * 1e-9).tolist()}
    return idx


def query(idx: OracleIndex, pairs) -> np.ndarray:
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    out = np.zeros(len(pairs), np.uint8)
    rc = (idx._lib or _load()).orc_query(idx._handle, _ptr(pairs), len(pairs), _ptr(out))
    if rc != 0:
        raise OracleError(rc)
    return out


def query_parts(idx: OracleIndex, pairs) -> tuple[np.ndarray, np.ndarray]:
    """(bit-parallel part, normal-label part) of each query, unclamped ints."""
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    a = np.zeros(len(pairs), np.int32)
    b = np.zeros(len(pairs), np.int32)
    rc = (idx._lib or _load()).orc_query_parts(idx._handle, _ptr(pairs), len(pairs), _ptr(a), _ptr(b))
    if rc != 0:
        raise OracleError(rc)
    return a, b


def paths(idx: OracleIndex, pairs, maxlen: int) -> tuple[np.ndarray, np.ndarray]:
    """Shortest paths (input ids) of each pair: (paths[q, maxlen], lens[q]);
    lens = D+1, 0 if unreachable, -(D+1) if maxlen is too small."""
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    out = np.full((len(pairs), max(maxlen, 0)), -1, np.int32)
    lens = np.zeros(len(pairs), np.int32)
    rc = (idx._lib or _load()).orc_paths(idx._handle, _ptr(pairs), len(pairs), int(maxlen),
                                        _ptr(out), _ptr(lens))
    if rc != 0:
        raise OracleError(rc)
    return out, lens


@dataclass
class DirectedIndex:
    """Exported oracle index of a directed graph (Section 6): L_OUT and L_IN
    in rank order, no sentinels."""
    n: int
    rank: np.ndarray
    out_off: np.ndarray
    out_hub: np.ndarray
    out_dist: np.ndarray
    in_off: np.ndarray
    in_hub: np.ndarray
    in_dist: np.ndarray
    out_par: np.ndarray | None = None  # uint32 parents (ranks) of the L_OUT entries
    in_par: np.ndarray | None = None   # ... of the L_IN entries
    counters: dict = field(default_factory=dict)
    _handle: C.c_void_p | None = None
    _lib: object = None

    def close(self):
        if self._handle is not None:
            (self._lib or _load()).orc_free(self._handle)
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_directed(row_ptr, col, order, lib=None) -> DirectedIndex:
    """Labels of a directed graph given by its out-edges."""
    lib = lib or _load()
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    order = np.ascontiguousarray(order, dtype=np.int32)
    n = len(order)
    if len(row_ptr) != n + 1:
        raise OracleError(-1)
    h = C.c_void_p()
    rc = lib.orc_build_directed(n, _ptr(row_ptr), _ptr(col), _ptr(order), C.byref(h))
    if rc != 0:
        raise OracleError(rc)
    out_off = np.zeros(n + 1, np.int64)
    lib.orc_export(h, _ptr(out_off), None, None, None, None, None, None, None, None, None)
    ne_out = int(out_off[-1])
    ix = DirectedIndex(n=n, rank=np.zeros(n, np.int32), out_off=out_off,
                       out_hub=np.zeros(ne_out, np.uint32), out_dist=np.zeros(ne_out, np.uint8),
                       in_off=np.zeros(n + 1, np.int64), in_hub=None, in_dist=None, _handle=h)
    ix._lib = lib
    lib.orc_export(h, None, _ptr(ix.out_hub), _ptr(ix.out_dist), None, None, None,
                   _ptr(ix.rank), None, None, None)
    ne_in = C.c_int64()
    lib.orc_export_in(h, C.byref(ne_in), _ptr(ix.in_off), None, None)
    ix.in_hub = np.zeros(ne_in.value, np.uint32)
    ix.in_dist = np.zeros(ne_in.value, np.uint8)
    lib.orc_export_in(h, None, None, _ptr(ix.in_hub), _ptr(ix.in_dist))
    ix.out_par = np.zeros(ne_out, np.uint32)
    ix.in_par = np.zeros(ne_in.value, np.uint32)
    if ne_out:
        lib.orc_export_parents(h, _ptr(ix.out_par))
    if ne_in.value:
        lib.orc_export_in_parents(h, _ptr(ix.in_par))
    nc = lib.orc_ncounters()
    cnt = np.zeros(nc, np.int64)
    lib.orc_counters(h, _ptr(cnt), nc)
    ix.counters = {k: int(v) for k, v in zip(COUNTER_NAMES, cnt)}
    return ix


def query_directed(ix: DirectedIndex, pairs) -> np.ndarray:
    """d(s, t) along edge directions, min(., 255)."""
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    out = np.zeros(len(pairs), np.uint8)
    rc = (ix._lib or _load()).orc_query(ix._handle, _ptr(pairs), len(pairs), _ptr(out))
    if rc != 0:
        raise OracleError(rc)
    return out


WCOUNTER_NAMES = ["n", "entries", "roots", "settled", "labeled", "edges", "pushes",
                  "label_scanned", "max_dist"]
WINF = 0xFFFFFFFF


@dataclass
class WeightedIndex:
    """Exported oracle index of a weighted graph (Section 6): labels in rank
    order, no sentinels, uint32 distances; ``in_*`` only for a digraph."""
    n: int
    directed: bool
    rank: np.ndarray
    off: np.ndarray
    hub: np.ndarray
    dist: np.ndarray
    in_off: np.ndarray | None = None
    in_hub: np.ndarray | None = None
    in_dist: np.ndarray | None = None
    par: np.ndarray | None = None     # uint32 parents (ranks) of the side-0 entries
    in_par: np.ndarray | None = None  # ... of the L_IN entries
    counters: dict = field(default_factory=dict)
    _handle: C.c_void_p | None = None
    _lib: object = None

    def close(self):
        if self._handle is not None:
            (self._lib or _load()).orc_wfree(self._handle)
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_weighted(row_ptr, col, wgt, order, directed: bool = False,
                   check_symmetric: bool = True, lib=None) -> WeightedIndex:
    """Pruned Dijkstra labels (weights uint32 >= 1, one per CSR entry)."""
    lib = lib or _load()
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    wgt = np.ascontiguousarray(wgt, dtype=np.uint32)
    order = np.ascontiguousarray(order, dtype=np.int32)
    n = len(order)
    if len(row_ptr) != n + 1 or len(wgt) != len(col):
        raise OracleError(-1)
    flags = (2 if directed else 0) | (1 if check_symmetric and not directed else 0)
    h = C.c_void_p()
    rc = lib.orc_build_weighted(n, _ptr(row_ptr), _ptr(col), _ptr(wgt), _ptr(order), flags,
                                C.byref(h))
    if rc != 0:
        raise OracleError(rc)

    def side(s):
        ne = C.c_int64()
        off = np.zeros(n + 1, np.int64)
        lib.orc_wexport(h, s, C.byref(ne), _ptr(off), None, None, None)
        hub = np.zeros(ne.value, np.uint32)
        dist = np.zeros(ne.value, np.uint32)
        lib.orc_wexport(h, s, None, None, _ptr(hub), _ptr(dist), None)
        return off, hub, dist

    def parents(s, ne):
        par = np.zeros(ne, np.uint32)
        if ne:
            lib.orc_wexport_parents(h, s, _ptr(par))
        return par

    rank = np.zeros(n, np.int32)
    lib.orc_wexport(h, 0, None, None, None, None, _ptr(rank))
    off, hub, dist = side(0)
    ix = WeightedIndex(n=n, directed=directed, rank=rank, off=off, hub=hub, dist=dist, _handle=h)
    ix._lib = lib
    ix.par = parents(0, len(hub))
    if directed:
        ix.in_off, ix.in_hub, ix.in_dist = side(1)
        ix.in_par = parents(1, len(ix.in_hub))
    nc = lib.orc_wncounters()
    cnt = np.zeros(nc, np.int64)
    lib.orc_wcounters(h, _ptr(cnt), nc)
    ix.counters = {k: int(v) for k, v in zip(WCOUNTER_NAMES, cnt)}
    return ix


def query_weighted(ix: WeightedIndex, pairs) -> np.ndarray:
    """d(s, t) (along the arcs for a digraph) as uint32; WINF = unreachable
    or 2^32 - 1 or more away."""
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    out = np.zeros(len(pairs), np.uint32)
    rc = (ix._lib or _load()).orc_wquery(ix._handle, _ptr(pairs), len(pairs), _ptr(out))
    if rc != 0:
        raise OracleError(rc)
    return out


def paths_weighted(ix: WeightedIndex, pairs, maxlen: int) -> tuple[np.ndarray, np.ndarray]:
    """Shortest paths (input ids) of a weighted index: (paths[q, maxlen],
    lens[q]); lens = vertices on the path, 0 if unreachable, -(vertices) if
    maxlen is too small."""
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    out = np.full((len(pairs), max(maxlen, 0)), -1, np.int32)
    lens = np.zeros(len(pairs), np.int32)
    rc = (ix._lib or _load()).orc_wpaths(ix._handle, _ptr(pairs), len(pairs), int(maxlen),
                                        _ptr(out), _ptr(lens))
    if rc != 0:
        raise OracleError(rc)
    return out, lens
