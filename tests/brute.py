"""Brute-force and closed-form checkers used to pin the oracle.

Nothing here shares code with the oracle or with the GPU library.  Each
function computes a quantity the paper defines directly, by a different route
than the labeling algorithm:

* ``apsp``: all-pairs BFS distances (the corollary of Theorem 4.1 says the
  final index answers exactly these);
* ``canonical_labels``: the set of label entries the pruned labeling must
  produce, from its characterisation by shortest-path sets (the argument of
  Theorems 4.1 and 4.2): hub h is in the label of u at distance d(h, u) iff
  h was not used by the bit-parallel phase and no vertex on any shortest
  h-u path comes earlier in the order (bit-parallel vertices count as
  earliest of all);
* ``bp_closed_form``: the bit-parallel label of every vertex straight from the
  set definitions of Section 5.1 (one BFS per vertex of {r} plus S_r);
* ``label_query``: the 2-hop query of Section 3.3 as a dictionary lookup.
"""
from __future__ import annotations

import numpy as np
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import shortest_path

INF = 255


def apsp(row_ptr, col, sources=None) -> np.ndarray:
    """BFS distances as int64, unreachable = INF (255).  Rows are ``sources``
    (all vertices when None), columns are all vertices, both in input ids."""
    n = len(row_ptr) - 1
    if n == 0:
        return np.zeros((0, 0), np.int64)
    a = csr_matrix((np.ones(len(col)), np.asarray(col), np.asarray(row_ptr)), shape=(n, n))
    d = shortest_path(a, unweighted=True, directed=False, indices=sources)
    d = np.where(np.isinf(d), INF, d).astype(np.int64)
    return d


def bfs_levels(row_ptr, col, src: int) -> np.ndarray:
    """Distances from ``src`` by plain level-synchronous BFS (int64, INF=255)."""
    n = len(row_ptr) - 1
    dist = np.full(n, INF, np.int64)
    dist[src] = 0
    frontier = np.array([src], np.int64)
    lvl = 0
    while len(frontier):
        starts, ends = row_ptr[frontier], row_ptr[frontier + 1]
        nb = np.concatenate([col[a:b] for a, b in zip(starts, ends)]) if len(frontier) else np.zeros(0, np.int64)
        nb = np.unique(nb)
        nb = nb[dist[nb] == INF]
        lvl += 1
        dist[nb] = lvl
        frontier = nb
    return dist


def canonical_labels(row_ptr, col, order, bp_used_ranks) -> list[dict[int, int]]:
    """Expected normal labels, indexed by rank: ``labels[r] = {hub_rank: dist}``.

    For every vertex u, one BFS from u computes M(w), the smallest key over
    all vertices on shortest u-w paths (key = -1 for bit-parallel vertices,
    else the rank), by the recurrence M(w) = min(key(w), min over BFS parents
    p of M(p)).  Then (rank(h), d(u,h)) is in L(u) iff h is not a
    bit-parallel vertex and M(h) == rank(h)."""
    row_ptr = np.asarray(row_ptr, np.int64)
    col = np.asarray(col, np.int64)
    order = np.asarray(order, np.int64)
    n = len(order)
    rank = np.empty(n, np.int64)
    rank[order] = np.arange(n)
    key = rank.copy()
    bp = np.zeros(n, bool)
    for r in bp_used_ranks:
        bp[order[r]] = True
    key[bp] = -1
    src_of_edge = np.repeat(np.arange(n), np.diff(row_ptr))
    labels: list[dict[int, int]] = [dict() for _ in range(n)]
    for u in range(n):
        if bp[u]:
            continue
        dist = np.full(n, INF, np.int64)
        M = np.full(n, np.iinfo(np.int64).max, np.int64)
        dist[u] = 0
        M[u] = key[u]
        frontier = np.array([u], np.int64)
        lvl = 0
        while len(frontier):
            # edges leaving the frontier
            sel = np.isin(src_of_edge, frontier) if len(frontier) > 64 else None
            if sel is None:
                idx = np.concatenate([np.arange(row_ptr[f], row_ptr[f + 1]) for f in frontier])
            else:
                idx = np.nonzero(sel)[0]
            p = src_of_edge[idx]
            w = col[idx]
            fresh = (dist[w] == INF) | (dist[w] == lvl + 1)
            p, w = p[fresh], w[fresh]
            newv = np.unique(w[dist[w] == INF])
            dist[newv] = lvl + 1
            # M of the new level: min over parents, then min with own key
            np.minimum.at(M, w, M[p])
            M[newv] = np.minimum(M[newv], key[newv])
            frontier = newv
            lvl += 1
        ru = int(rank[u])
        hit = np.nonzero((dist < INF) & (~bp) & (M == key))[0]
        for h in hit:
            labels[ru][int(rank[h])] = int(dist[h])
    return labels


def bp_closed_form(D_rank: np.ndarray, roots, sels):
    """Bit-parallel labels from the definitions of Section 5.1.

    ``D_rank`` is the all-pairs distance matrix in rank space.  For slot i
    with root r and chosen neighbours S (bit j = S[j]):
    d = d(r, v), S^{-1}(v) = {w in S : d(w, v) = d(r, v) - 1} and
    S^{0}(v) = {w in S : d(w, v) = d(r, v)}.  Empty slots give (255, 0, 0).
    Returns (d uint8[n, t], m1 uint64[n, t], m0 uint64[n, t])."""
    n = D_rank.shape[0]
    t = len(roots)
    d = np.full((n, t), INF, np.uint8)
    m1 = np.zeros((n, t), np.uint64)
    m0 = np.zeros((n, t), np.uint64)
    for i, (r, S) in enumerate(zip(roots, sels)):
        if r < 0:
            continue
        dr = D_rank[r]
        d[:, i] = np.minimum(dr, INF).astype(np.uint8)
        for j, w in enumerate(S):
            dw = D_rank[w]
            bit = np.uint64(1) << np.uint64(j)
            reach = dr < INF
            m1[reach & (dw == dr - 1), i] |= bit
            m0[reach & (dw == dr), i] |= bit
    return d, m1, m0


def label_query(La: dict[int, int], Lb: dict[int, int]) -> int:
    """QUERY of Section 3.3 over normal labels only; INF when no common hub."""
    best = INF
    for h, da in La.items():
        db = Lb.get(h)
        if db is not None and da + db < best:
            best = da + db
    return best


def bp_query(d, m1, m0, a: int, b: int) -> int:
    """Bit-parallel part of the query (Section 5.3) as the explicit minimum
    over the root and each chosen neighbour (the definition, not the O(1)
    rule): uses d(a, w) = d(a, r) + {-1, 0, +1} read off the two sets."""
    best = INF
    t = d.shape[1]
    for i in range(t):
        da, db = int(d[a, i]), int(d[b, i])
        if da == INF or db == INF:
            continue
        best = min(best, da + db)  # via the root itself
        for j in range(64):
            bit = np.uint64(1) << np.uint64(j)
            # distance from a and b to the j-th neighbour
            def via(dx, mm1, mm0):
                if mm1 & bit:
                    return dx - 1
                if mm0 & bit:
                    return dx
                return dx + 1
            best = min(best, via(da, m1[a, i], m0[a, i]) + via(db, m1[b, i], m0[b, i]))
    return best


def _frontier_edges(row_ptr, frontier):
    """(source, edge index) of every adjacency entry of the frontier's rows."""
    starts = row_ptr[frontier]
    deg = row_ptr[frontier + 1] - starts
    tot = int(deg.sum())
    if tot == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    first = np.cumsum(deg) - deg
    idx = np.arange(tot, dtype=np.int64) - np.repeat(first, deg) + np.repeat(starts, deg)
    return np.repeat(frontier, deg), idx


def canonical_label_one(row_ptr, col, rank, bp, u: int) -> dict[int, int]:
    """``canonical_labels`` for one vertex ``u`` (input id) of a large graph:
    one BFS from u with the min-key recurrence, touching only the rows of
    each frontier.  ``rank`` int64[n] (id -> rank), ``bp`` bool[n] (used by
    the bit-parallel phase).  Returns {hub_rank: dist}; empty for u in B."""
    row_ptr = np.asarray(row_ptr, np.int64)
    n = len(rank)
    if bp[u]:
        return {}
    key = np.where(bp, -1, rank).astype(np.int64)
    dist = np.full(n, INF, np.int64)
    M = np.full(n, np.iinfo(np.int64).max, np.int64)
    dist[u] = 0
    M[u] = key[u]
    frontier = np.array([u], np.int64)
    lvl = 0
    while len(frontier):
        p, idx = _frontier_edges(row_ptr, frontier)
        w = np.asarray(col[idx], np.int64)
        fresh = (dist[w] == INF) | (dist[w] == lvl + 1)
        p, w = p[fresh], w[fresh]
        newv = np.unique(w[dist[w] == INF])
        dist[newv] = lvl + 1
        np.minimum.at(M, w, M[p])
        M[newv] = np.minimum(M[newv], key[newv])
        frontier = newv
        lvl += 1
    hit = np.nonzero((dist < INF) & (~bp) & (M == key))[0]
    return {int(rank[h]): int(dist[h]) for h in hit}
