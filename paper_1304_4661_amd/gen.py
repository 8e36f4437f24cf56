"""Seeded synthetic inputs for Pruned Landmark Labeling.

This module only makes inputs: graphs in CSR form, the vertex order and query
pairs.  It holds none of the labeling or query arithmetic, so both the CPU
oracle and the GPU library can be fed from it without sharing any of the
method's code.

The paper measures on real social, web and computer networks (Section 7,
Table 3), which are not available here.  Barabasi-Albert and R-MAT graphs stand
in for them: both have power-law degrees and small-world distances, the two
traits the paper's analysis relies on (Section 7.1, degree and distance
distributions).

Conventions shared by every generator:

* the graph is undirected and unweighted (Section 3.1); each undirected edge
  appears in both rows of the CSR, rows are sorted ascending, there are no
  self-loops and no repeated edges;
* ``row_ptr`` is ``int32[n+1]`` and ``col`` is ``int32[row_ptr[n]]``;
* the vertex order is the Degree strategy (Section 4.4): degree descending,
  ties broken by ascending vertex id; ``order[i]`` is the vertex of rank ``i``;
* all randomness comes from numpy's PCG64 seeded with the given integer.
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Graph",
    "ba_edges",
    "ba_graph",
    "rmat_edges",
    "rmat_graph",
    "csr_from_edges",
    "largest_component",
    "degree_order",
    "closeness_order",
    "random_order",
    "uniform_weights",
    "random_pairs",
    "csr_sha256",
    "pack_batch",
    "batch_spec",
    "config_graph",
    "CONFIGS",
]


@dataclass
class Graph:
    n: int
    row_ptr: np.ndarray  # int32[n+1]
    col: np.ndarray      # int32[nnz]
    meta: dict = field(default_factory=dict)
    w: np.ndarray | None = None  # uint32[nnz] edge weights of a weighted graph

    @property
    def m(self) -> int:
        """Number of undirected edges."""
        return int(self.row_ptr[-1]) // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# --------------------------------------------------------------------------
# CSR construction and cleanup
# --------------------------------------------------------------------------

def csr_from_edges(n: int, u: np.ndarray, v: np.ndarray) -> Graph:
    """Symmetrize, drop self-loops, de-duplicate and build a sorted CSR."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    src = np.concatenate([u, v])
    dst = np.concatenate([v, u])
    key = np.unique(src * np.int64(n) + dst)
    src = key // n
    dst = key - src * n
    counts = np.bincount(src, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("graph too large for int32 CSR")
    return Graph(n, row_ptr.astype(np.int32), dst.astype(np.int32))


def largest_component(g: Graph) -> Graph:
    """Keep the largest connected component; ids are compacted in their
    original order.  Among equally large components the one holding the
    smallest vertex id wins."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components

    if g.n == 0:
        return g
    a = csr_matrix((np.ones(len(g.col), dtype=np.int8), g.col, g.row_ptr), shape=(g.n, g.n))
    ncomp, lab = connected_components(a, directed=False)
    sizes = np.bincount(lab, minlength=ncomp)
    # connected_components numbers components by their smallest vertex, so
    # argmax picks the one with the smallest id among ties.
    big = int(np.argmax(sizes))
    keep = lab == big
    newid = np.cumsum(keep) - 1
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    emask = keep[src]
    s2 = newid[src[emask]]
    d2 = newid[g.col[emask]]
    n2 = int(keep.sum())
    counts = np.bincount(s2, minlength=n2)
    row_ptr = np.zeros(n2 + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    # rows stay sorted: the relabel is monotone and src order is preserved
    return Graph(n2, row_ptr.astype(np.int32), d2.astype(np.int32), dict(g.meta))


# --------------------------------------------------------------------------
# Barabasi-Albert
# --------------------------------------------------------------------------

def ba_edges(n: int, m: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Preferential attachment.  Vertices ``0..m-1`` start isolated, vertex
    ``m`` joins all of them, and every later vertex ``v`` picks ``m`` distinct
    targets in ``[0, v)`` with probability proportional to degree, by drawing
    uniformly from the multiset of edge endpoints and redrawing repeats.
    Gives exactly ``m*(n-m)`` edges and a connected graph."""
    if m < 1 or n <= m:
        raise ValueError("need 1 <= m < n")
    rng = _rng(seed)
    ne = m * (n - m)
    us = np.empty(ne, dtype=np.int64)
    vs = np.empty(ne, dtype=np.int64)
    ends = np.empty(2 * ne, dtype=np.int64)
    # vertex m joins 0..m-1
    for j in range(m):
        us[j], vs[j] = m, j
        ends[2 * j], ends[2 * j + 1] = m, j
    e = m
    buf = rng.random(1 << 16)
    bi = 0
    for v in range(m + 1, n):
        nends = 2 * e
        chosen: list[int] = []
        while len(chosen) < m:
            if bi == len(buf):
                buf = rng.random(1 << 16)
                bi = 0
            t = int(ends[int(buf[bi] * nends)])
            bi += 1
            if t not in chosen:
                chosen.append(t)
        for t in chosen:
            us[e], vs[e] = v, t
            ends[2 * e], ends[2 * e + 1] = v, t
            e += 1
    return us, vs


_NATIVE = None


def _native():
    """ctypes handle of gen_native.c (compiled with gcc on first use), or None."""
    global _NATIVE
    if _NATIVE is None:
        import ctypes as C
        import os
        import subprocess

        here = os.path.dirname(os.path.abspath(__file__))
        src = os.path.join(here, "gen_native.c")
        lib = os.path.join(here, "libgen_native.so")
        try:
            if not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src):
                tmp = f"{lib}.tmp{os.getpid()}"
                subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, src])
                os.replace(tmp, lib)
            h = C.CDLL(lib)
            P = C.c_void_p
            h.ba_edges.argtypes = [C.c_int64, C.c_int32, P, C.c_int64, P, P, P]
            h.ba_edges.restype = C.c_int64
            _NATIVE = h
        except (OSError, subprocess.CalledProcessError):
            _NATIVE = False
    return _NATIVE or None


def ba_edges_fast(n: int, m: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Same edges as :func:`ba_edges` (same draws in the same order), with the
    attachment loop in C."""
    lib = _native()
    if lib is None or m > 64:
        return ba_edges(n, m, seed)
    if m < 1 or n <= m:
        raise ValueError("need 1 <= m < n")
    rng = _rng(seed)
    ne = m * (n - m)
    us = np.empty(ne, dtype=np.int64)
    vs = np.empty(ne, dtype=np.int64)
    ends = np.empty(2 * ne, dtype=np.int64)
    u = rng.random(int(ne * 1.25) + 4096)
    while True:
        used = lib.ba_edges(n, m, u.ctypes.data, len(u), us.ctypes.data, vs.ctypes.data,
                            ends.ctypes.data)
        if used >= 0:
            return us, vs
        u = np.concatenate([u, rng.random(len(u) // 2 + 4096)])


def ba_graph(n: int, m: int, seed: int) -> Graph:
    u, v = ba_edges_fast(n, m, seed)
    g = csr_from_edges(n, u, v)
    g.meta = {"kind": "ba", "n": n, "m_attach": m, "seed": seed}
    return g


# --------------------------------------------------------------------------
# R-MAT
# --------------------------------------------------------------------------

def rmat_edges(scale: int, edge_factor: int, a: float, b: float, c: float,
               seed: int, chunk: int = 1 << 22) -> tuple[np.ndarray, np.ndarray]:
    """``edge_factor * 2**scale`` R-MAT samples.  Each of the ``scale`` bits of
    source and destination is chosen by one uniform draw that picks a quadrant
    with probabilities ``(a, b, c, 1-a-b-c)``, most significant bit first.  No
    noise and no id permutation."""
    rng = _rng(seed)
    total = edge_factor << scale
    us = np.empty(total, dtype=np.int64)
    vs = np.empty(total, dtype=np.int64)
    ab, abc = a + b, a + b + c
    for lo in range(0, total, chunk):
        k = min(chunk, total - lo)
        s = np.zeros(k, dtype=np.int64)
        d = np.zeros(k, dtype=np.int64)
        for _ in range(scale):
            r = rng.random(k)
            sbit = (r >= ab).astype(np.int64)
            dbit = (((r >= a) & (r < ab)) | (r >= abc)).astype(np.int64)
            s = (s << 1) | sbit
            d = (d << 1) | dbit
        us[lo:lo + k] = s
        vs[lo:lo + k] = d
    return us, vs


def rmat_graph(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19,
               c: float = 0.19, seed: int = 0) -> Graph:
    """R-MAT, symmetrized, self-loops dropped, de-duplicated, largest connected
    component kept with ids compacted in their original order."""
    u, v = rmat_edges(scale, edge_factor, a, b, c, seed)
    g = csr_from_edges(1 << scale, u, v)
    del u, v
    g = largest_component(g)
    g.meta = {"kind": "rmat", "scale": scale, "edge_factor": edge_factor,
              "abcd": [a, b, c, round(1 - a - b - c, 6)], "seed": seed}
    return g


# --------------------------------------------------------------------------
# Directed graphs (Section 6, "Directed Graphs")
# --------------------------------------------------------------------------

def digraph_from_edges(n: int, u: np.ndarray, v: np.ndarray) -> Graph:
    """Directed edges u -> v: drop self-loops, de-duplicate, CSR of
    out-edges with sorted rows.  meta["directed"] is set; ``nnz`` is the
    number of arcs."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    keep = u != v
    key = np.unique(u[keep] * np.int64(n) + v[keep])
    src = key // n
    dst = key - src * n
    counts = np.bincount(src, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("graph too large for int32 CSR")
    return Graph(n, row_ptr.astype(np.int32), dst.astype(np.int32), {"directed": True})


def weakly_connected_part(g: Graph) -> Graph:
    """Keep the largest weakly connected component of a digraph (ids
    compacted in their original order)."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components

    if g.n == 0:
        return g
    a = csr_matrix((np.ones(len(g.col), dtype=np.int8), g.col, g.row_ptr), shape=(g.n, g.n))
    ncomp, lab = connected_components(a, directed=True, connection="weak")
    keep = lab == int(np.argmax(np.bincount(lab, minlength=ncomp)))
    newid = np.cumsum(keep) - 1
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    emask = keep[src] & keep[g.col]
    out = digraph_from_edges(int(keep.sum()), newid[src[emask]], newid[g.col[emask]])
    out.meta = dict(g.meta)
    return out


def rmat_digraph(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19,
                 c: float = 0.19, seed: int = 0) -> Graph:
    """R-MAT samples as arcs (not symmetrized), self-loops dropped,
    de-duplicated, largest weakly connected component kept."""
    u, v = rmat_edges(scale, edge_factor, a, b, c, seed)
    g = weakly_connected_part(digraph_from_edges(1 << scale, u, v))
    g.meta = {"kind": "rmat", "directed": True, "scale": scale, "edge_factor": edge_factor,
              "abcd": [a, b, c, round(1 - a - b - c, 6)], "seed": seed}
    return g


def er_digraph(n: int, p: float, seed: int) -> Graph:
    """Each of the n(n-1) arcs independently with probability p."""
    rng = _rng(seed)
    m = rng.random((n, n)) < p
    np.fill_diagonal(m, False)
    u, v = np.nonzero(m)
    return digraph_from_edges(n, u, v)


def degree_order_directed(g: Graph) -> np.ndarray:
    """Degree strategy for a digraph: in-degree plus out-degree descending,
    ties by ascending id."""
    deg = np.diff(g.row_ptr).astype(np.int64) + np.bincount(g.col, minlength=g.n)
    ids = np.arange(g.n, dtype=np.int64)
    return np.lexsort((ids, -deg)).astype(np.int32)


# --------------------------------------------------------------------------
# Orders, pairs, digests, batches
# --------------------------------------------------------------------------

def degree_order(g: Graph) -> np.ndarray:
    """Degree strategy (Section 4.4): degree descending, ties by ascending id."""
    deg = g.degrees()
    ids = np.arange(g.n, dtype=np.int64)
    return np.lexsort((ids, -deg)).astype(np.int32)


def closeness_order(g: Graph, samples: int = 16, seed: int = 0) -> np.ndarray:
    """Closeness strategy (Section 4.4): closeness centrality approximated by
    BFS distances from ``samples`` vertices drawn uniformly without
    replacement (PCG64 ``seed``); vertices in ascending order of their summed
    distance to the samples (unreachable counts as n), ties by ascending id.
    With samples >= n it is exact closeness (on a connected graph)."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import shortest_path

    n = g.n
    if n == 0:
        return np.zeros(0, np.int32)
    k = min(samples, n)
    src = np.sort(_rng(seed).choice(n, size=k, replace=False)) if k < n else np.arange(n)
    a = csr_matrix((np.ones(len(g.col), np.int8), g.col, g.row_ptr), shape=(n, n))
    d = shortest_path(a, unweighted=True, directed=False, indices=src)
    d = np.where(np.isinf(d), n, d).sum(axis=0)
    ids = np.arange(n, dtype=np.int64)
    return np.lexsort((ids, d)).astype(np.int32)


def random_order(n: int, seed: int) -> np.ndarray:
    """Random strategy (Section 4.4)."""
    return _rng(seed).permutation(n).astype(np.int32)


def uniform_weights(g: Graph, lo: int, hi: int, seed: int) -> Graph:
    """The same graph with integer edge weights drawn i.i.d. uniform in
    ``[lo, hi]`` (PCG64 ``seed``): one draw per undirected edge, stored on
    both of its CSR entries, in the order of the edges' (smaller id, larger
    id) keys; one draw per arc of a digraph, in CSR order."""
    rows = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))
    col = g.col.astype(np.int64)
    r = _rng(seed)
    if g.meta.get("directed"):
        w = r.integers(lo, hi + 1, size=len(col), dtype=np.int64)
    else:
        key = np.minimum(rows, col) * g.n + np.maximum(rows, col)
        uniq, inv = np.unique(key, return_inverse=True)
        w = r.integers(lo, hi + 1, size=len(uniq), dtype=np.int64)[inv]
    meta = dict(g.meta, weights=(lo, hi, seed))
    return Graph(g.n, g.row_ptr, g.col, meta, w.astype(np.uint32))


def random_pairs(n: int, q: int, seed: int) -> np.ndarray:
    """``q`` pairs, both ends i.i.d. uniform over ``[0, n)`` with replacement
    (``s == t`` allowed), returned as ``int32[q, 2]``."""
    return _rng(seed).integers(0, n, size=(q, 2), dtype=np.int64).astype(np.int32)


def csr_sha256(g: Graph, order: np.ndarray | None = None) -> str:
    h = hashlib.sha256()
    h.update(np.int64(g.n).tobytes())
    h.update(np.ascontiguousarray(g.row_ptr, dtype="<i4").tobytes())
    h.update(np.ascontiguousarray(g.col, dtype="<i4").tobytes())
    if order is not None:
        h.update(np.ascontiguousarray(order, dtype="<i4").tobytes())
    return h.hexdigest()


def batch_spec(count: int, seed_base: int = 4000, n_lo: float = 1e3, n_hi: float = 2e5,
               m_lo: int = 2, m_hi: int = 8) -> list[tuple[int, int, int]]:
    """(n, m, seed) for each graph of a multi-graph batch: ``n`` log-uniform in
    ``[n_lo, n_hi]``, ``m`` uniform in ``{m_lo..m_hi}``, one PCG64 stream per
    graph seeded ``seed_base + i``."""
    out = []
    for i in range(count):
        r = _rng(seed_base + i)
        n = int(round(math.exp(r.uniform(math.log(n_lo), math.log(n_hi)))))
        m = int(r.integers(m_lo, m_hi + 1))
        out.append((max(n, m + 1), m, seed_base + i))
    return out


def pack_batch(graphs: list[Graph], order_fn=None):
    """Concatenate graphs into one CSR with global ids.

    Returns ``(vtx_off int64[G+1], row_ptr int32[N+1], col int32[nnz],
    order int32[N])`` where ``order`` holds, for graph ``g``, its local order
    (``order_fn``, default Degree) in ``order[vtx_off[g]:vtx_off[g+1]]``
    (local ranks -> local ids)."""
    order_fn = order_fn or degree_order
    G = len(graphs)
    vtx_off = np.zeros(G + 1, dtype=np.int64)
    vtx_off[1:] = np.cumsum([g.n for g in graphs])
    nnz = sum(int(g.row_ptr[-1]) for g in graphs)
    if nnz >= 2**31:
        raise ValueError("batch too large for int32 CSR")
    N = int(vtx_off[-1])
    row_ptr = np.zeros(N + 1, dtype=np.int32)
    col = np.empty(nnz, dtype=np.int32)
    order = np.empty(N, dtype=np.int32)
    e = 0
    for gi, g in enumerate(graphs):
        v0 = int(vtx_off[gi])
        row_ptr[v0 + 1:v0 + g.n + 1] = g.row_ptr[1:] + e
        col[e:e + len(g.col)] = g.col + v0
        order[v0:v0 + g.n] = order_fn(g)
        e += len(g.col)
    return vtx_off, row_ptr, col, order


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

CONFIGS = {
    # name: (graph recipe, t_bp, number of query pairs, pair seed)
    "ba2000": ({"kind": "ba", "n": 2000, "m": 4, "seed": 1}, 16, 100_000, 101),
    "rmat18": ({"kind": "rmat", "scale": 18, "seed": 2}, 50, 1_000_000, 102),
    "rmat20": ({"kind": "rmat", "scale": 20, "seed": 3}, 64, 10_000_000, 103),
    # served workload; one batch of 1e7 pairs stands for a step's queries
    "rmat22": ({"kind": "rmat", "scale": 22, "seed": 5}, 64, 10_000_000, 105),
    # directed (Section 6): R-MAT arcs, no bit-parallel labels
    "rmat18d": ({"kind": "rmat", "directed": True, "scale": 18, "seed": 2}, 0, 1_000_000, 102),
    # weighted (Section 6): integer weights uniform in [1, 100], no bit-parallel labels
    "ba2000w": ({"kind": "ba", "n": 2000, "m": 4, "seed": 1, "weights": (1, 100, 7)}, 0,
                100_000, 101),
    "rmat18w": ({"kind": "rmat", "scale": 18, "seed": 2, "weights": (1, 100, 8)}, 0,
                1_000_000, 102),
}


def batch_workload(count: int = 256, t_bp: int = 16, pairs_per_graph: int = 10_000,
                   seed_base: int = 4000, pair_seed_base: int = 14000):
    """The multi-graph workload: ``count`` Barabasi-Albert graphs from
    :func:`batch_spec`, packed by :func:`pack_batch`, with ``pairs_per_graph``
    uniform pairs inside each graph (PCG64 seeded ``pair_seed_base + i``), as
    global ids.  Returns (graphs, vtx_off, row_ptr, col, order, t_bp, pairs)."""
    spec = batch_spec(count, seed_base=seed_base)
    graphs = [ba_graph(n, m, s) for n, m, s in spec]
    vtx_off, row_ptr, col, order = pack_batch(graphs)
    pairs = np.concatenate([
        random_pairs(g.n, pairs_per_graph, pair_seed_base + i) + np.int32(vtx_off[i])
        for i, g in enumerate(graphs)]).astype(np.int32)
    return graphs, vtx_off, row_ptr, col, order, t_bp, pairs


def config_graph(name: str) -> tuple[Graph, np.ndarray, int, np.ndarray]:
    """(graph, degree order, t_bp, query pairs) of a named workload."""
    recipe, t_bp, q, pseed = CONFIGS[name]
    if recipe["kind"] == "ba":
        g = ba_graph(recipe["n"], recipe["m"], recipe["seed"])
    elif recipe.get("directed"):
        g = rmat_digraph(recipe["scale"], seed=recipe["seed"])
    else:
        g = rmat_graph(recipe["scale"], seed=recipe["seed"])
    order = degree_order_directed(g) if recipe.get("directed") else degree_order(g)
    if "weights" in recipe:
        g = uniform_weights(g, *recipe["weights"])
    pairs = random_pairs(g.n, q, pseed)
    return g, order, t_bp, pairs
