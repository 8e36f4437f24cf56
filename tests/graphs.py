"""Small graph families for tests (edge lists -> CSR through the generators'
cleanup, without keeping only the largest component)."""
from __future__ import annotations

import numpy as np

from paper_1304_4661_amd import gen


def from_edges(n, edges) -> gen.Graph:
    e = np.asarray(edges, np.int64).reshape(-1, 2)
    return gen.csr_from_edges(n, e[:, 0], e[:, 1])


def path(n):
    return from_edges(n, [(i, i + 1) for i in range(n - 1)])


def cycle(n):
    return from_edges(n, [(i, (i + 1) % n) for i in range(n)])


def star(n):
    return from_edges(n, [(0, i) for i in range(1, n)])


def complete(n):
    return from_edges(n, [(i, j) for i in range(n) for j in range(i + 1, n)])


def complete_bipartite(a, b):
    return from_edges(a + b, [(i, a + j) for i in range(a) for j in range(b)])


def grid(a, b):
    e = []
    for i in range(a):
        for j in range(b):
            v = i * b + j
            if j + 1 < b:
                e.append((v, v + 1))
            if i + 1 < a:
                e.append((v, v + b))
    return from_edges(a * b, e)


def random_tree(n, seed):
    r = np.random.Generator(np.random.PCG64(seed))
    return from_edges(n, [(i, int(r.integers(0, i))) for i in range(1, n)])


def erdos_renyi(n, p, seed):
    r = np.random.Generator(np.random.PCG64(seed))
    iu = np.triu_indices(n, 1)
    keep = r.random(len(iu[0])) < p
    return from_edges(n, np.stack([iu[0][keep], iu[1][keep]], 1))


def disjoint_union(*gs):
    edges, off = [], 0
    for g in gs:
        src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
        for a, b in zip(src, g.col):
            if a < b:
                edges.append((a + off, b + off))
        off += g.n
    return from_edges(off, edges)


def empty(n):
    return from_edges(n, np.zeros((0, 2), np.int64))


def families():
    """(name, graph) pairs covering trees, cycles, grids, dense, sparse,
    disconnected and isolated-vertex cases."""
    return [
        ("path9", path(9)),
        ("cycle10", cycle(10)),
        ("star12", star(12)),
        ("k7", complete(7)),
        ("k34", complete_bipartite(3, 4)),
        ("grid4x5", grid(4, 5)),
        ("tree40", random_tree(40, 7)),
        ("er30", erdos_renyi(30, 0.12, 3)),
        ("er60", erdos_renyi(60, 0.05, 4)),
        ("union", disjoint_union(cycle(5), star(6), path(4), empty(2))),
        ("ba80", gen.ba_graph(80, 2, 11)),
        ("ba120m3", gen.ba_graph(120, 3, 12)),
        ("empty3", empty(3)),
        ("single", empty(1)),
        ("star70", star(70)),
    ]


def level_255_pruned():
    """A graph whose pruned BFS reaches a vertex at distance 255 that the
    prune test then drops, so the build must succeed (8-bit distances,
    Section 4.5.1).  Path a_0..a_254 (ids 0..254), w = 255 joined to a_254,
    x = 256 joined to a_253 and w, and three leaves 257..259 on x.  With the
    order x, a_0, a_1, ..., w, leaves: the BFS from a_0 labels a_254 at 254
    and reaches w at 255, where d(a_0, x) + d(x, w) = 254 + 1 prunes it; the
    leaves (255 away through x) are never reached because x prunes itself.
    Returns (graph, order)."""
    edges = [(i, i + 1) for i in range(254)] + [(254, 255), (256, 253), (256, 255)]
    edges += [(256, 257), (256, 258), (256, 259)]
    g = from_edges(260, edges)
    order = np.array([256] + list(range(256)) + [257, 258, 259], np.int32)
    return g, order


def directed_from_undirected(g) -> gen.Graph:
    """The symmetric digraph with both arcs of every edge (same CSR)."""
    return gen.Graph(g.n, g.row_ptr.copy(), g.col.copy(), dict(g.meta))
