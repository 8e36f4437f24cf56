"""The oracle's pins, as reusable checks.

Each check compares the oracle against something the paper or plain
mathematics fixes, computed here by a different route (see ``brute``).  They
return a list of human-readable failures, so the same checks can be pointed at
a deliberately broken copy of the oracle to show they catch it.
"""
from __future__ import annotations

import numpy as np

import brute
import oracle
from paper_1304_4661_amd import gen

INF = 255


def bp_used_ranks(ix) -> list[int]:
    used = []
    for i in range(ix.t_bp):
        if ix.bp_root[i] >= 0:
            used.append(int(ix.bp_root[i]))
            used.extend(int(x) for x in ix.bp_sel[i, : ix.bp_nsel[i]])
    return used


def labels_of(ix) -> list[dict[int, int]]:
    out = []
    for r in range(ix.n):
        h, d = ix.label(r)
        out.append({int(a): int(b) for a, b in zip(h, d)})
    return out


def check_queries_vs_apsp(ix, g, D, lib=None) -> list[str]:
    """Corollary of Theorem 4.1: the index answers exact distances."""
    n = g.n
    if n == 0:
        return []
    s, t = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    pairs = np.stack([s.ravel(), t.ravel()], 1).astype(np.int32)
    got = oracle.query(ix, pairs).astype(np.int64).reshape(n, n)
    bad = np.argwhere(got != np.minimum(D, INF))
    return [f"query({a},{b}) = {got[a, b]} != d = {D[a, b]}" for a, b in bad[:5]]


def check_bp_selection(ix, g, order) -> list[str]:
    """Greedy choice of Section 5.4: root = lowest rank not used before; S_r =
    its unused neighbours, lowest ranks first, at most 64."""
    fails = []
    n = g.n
    rank = np.empty(n, np.int64)
    rank[order] = np.arange(n)
    used = set()
    for i in range(ix.t_bp):
        free = [r for r in range(n) if r not in used]
        r = int(ix.bp_root[i])
        if not free:
            if r != -1 or ix.bp_nsel[i] != 0:
                fails.append(f"slot {i} should be empty")
            continue
        if r != free[0]:
            fails.append(f"slot {i}: root {r} != lowest unused {free[0]}")
            return fails
        used.add(r)
        v = order[r]
        nb = sorted(int(rank[w]) for w in g.col[g.row_ptr[v]:g.row_ptr[v + 1]])
        want = [w for w in nb if w not in used][:64]
        got = [int(x) for x in ix.bp_sel[i, : ix.bp_nsel[i]]]
        if got != want:
            fails.append(f"slot {i}: S_r {got} != {want}")
        used.update(want)
    return fails


def check_bp_closed_form(ix, g, order, D) -> list[str]:
    """Section 5.1 definitions of d, S^{-1} and S^{0}."""
    if ix.t_bp == 0 or g.n == 0:
        return []
    Dr = D[np.ix_(order, order)]
    roots = [int(r) for r in ix.bp_root]
    sels = [list(ix.bp_sel[i, : ix.bp_nsel[i]]) for i in range(ix.t_bp)]
    d, m1, m0 = brute.bp_closed_form(Dr, roots, sels)
    fails = []
    for name, a, b in (("bp_d", ix.bp_d, d), ("bp_m1", ix.bp_m1, m1), ("bp_0", ix.bp_0, m0)):
        if not np.array_equal(a, b):
            w = np.argwhere(a != b)[0]
            fails.append(f"{name}[{w[0]},{w[1]}] = {a[w[0], w[1]]} != {b[w[0], w[1]]}")
    return fails


def check_canonical_labels(ix, g, order) -> list[str]:
    """Normal labels equal their shortest-path-set characterisation."""
    want = brute.canonical_labels(g.row_ptr, g.col, order, bp_used_ranks(ix))
    got = labels_of(ix)
    fails = []
    for r in range(g.n):
        if got[r] != want[r]:
            fails.append(f"L(rank {r}) = {sorted(got[r].items())} != {sorted(want[r].items())}")
            if len(fails) > 3:
                break
    # sortedness: hubs strictly increasing inside each label (Section 4.5.1)
    for r in range(g.n):
        h, _ = ix.label(r)
        if len(h) > 1 and np.any(np.diff(h.astype(np.int64)) <= 0):
            fails.append(f"L(rank {r}) not sorted")
            break
    return fails


def check_hubs_not_above_vertex(ix, g, order) -> list[str]:
    """No vertex holds a hub ranked after itself: when the search from v_k
    reaches a vertex of lower rank, that vertex was a root already (or a
    bit-parallel root or neighbour), so the labels of roots < k answer its
    distance to v_k exactly and the test prunes it (Theorem 4.1's argument,
    Section 5.3 for the bit-parallel vertices).  This is what lets the GPU
    leave such neighbours unvisited without testing them."""
    fails = []
    for r in range(g.n):
        h, _ = ix.label(r)
        if len(h) and int(h.max()) > r:
            fails.append(f"L(rank {r}) holds hub {int(h.max())}")
            if len(fails) > 3:
                break
    return fails


def check_query_parts(ix, g, order, D) -> list[str]:
    """Bit-parallel part = explicit minimum over {r} and S_r (Section 5.3);
    normal part = 2-hop query over the labels (Section 3.3)."""
    n = g.n
    if n == 0:
        return []
    s, t = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    pairs = np.stack([s.ravel(), t.ravel()], 1).astype(np.int32)
    bp, nm = oracle.query_parts(ix, pairs)
    bp = bp.reshape(n, n)
    nm = nm.reshape(n, n)
    fails = []
    Dr = D[np.ix_(order, order)]
    rank = np.empty(n, np.int64)
    rank[order] = np.arange(n)
    # explicit bit-parallel minimum, per slot with both ends reached
    want = np.full((n, n), INF, np.int64)
    for i in range(ix.t_bp):
        r = int(ix.bp_root[i])
        if r < 0:
            continue
        hubs = [r] + [int(x) for x in ix.bp_sel[i, : ix.bp_nsel[i]]]
        reach = Dr[r] < INF
        H = Dr[hubs]  # rank space
        via = (H[:, :, None] + H[:, None, :]).min(0)
        via = np.where(reach[:, None] & reach[None, :], via, INF)
        want = np.minimum(want, via)
    want_id = want[np.ix_(rank, rank)]
    got_bp = np.minimum(bp, INF)
    if not np.array_equal(got_bp, np.minimum(want_id, INF)):
        a, b = np.argwhere(got_bp != np.minimum(want_id, INF))[0]
        fails.append(f"bp part ({a},{b}) = {got_bp[a, b]} != {want_id[a, b]}")
    L = labels_of(ix)
    for a in range(n):
        for b in range(n):
            w = brute.label_query(L[rank[a]], L[rank[b]])
            if min(nm[a, b], INF) != w:
                fails.append(f"normal part ({a},{b}) = {nm[a, b]} != {w}")
                return fails
    return fails


def check_visited_counter(ix, g, order) -> list[str]:
    """Visited set of root k is {v_k} plus the neighbours of the vertices it
    labels, so the visited counter is fixed by the final labels."""
    n = g.n
    rank = np.empty(n, np.int64)
    rank[order] = np.arange(n)
    used = set(bp_used_ranks(ix))
    A = [[] for _ in range(n)]
    for r in range(n):
        h, _ = ix.label(r)
        for x in h:
            A[int(x)].append(r)
    total = 0
    edges = 0
    for k in range(n):
        if k in used:
            continue
        vis = {k}
        for r in A[k]:
            v = order[r]
            nb = g.col[g.row_ptr[v]:g.row_ptr[v + 1]]
            vis.update(int(rank[w]) for w in nb)
            edges += len(nb)
        total += len(vis)
    fails = []
    if ix.counters["visited"] != total:
        fails.append(f"visited counter {ix.counters['visited']} != {total}")
    if ix.counters["edges"] != edges:
        fails.append(f"edges counter {ix.counters['edges']} != {edges}")
    if ix.counters["labeled"] != int(ix.off[-1]):
        fails.append("labeled counter != entries")
    return fails


def label_maps(off, hub, dist):
    """Per rank, its label as {hub: distance}."""
    return [dict(zip(hub[off[r]:off[r + 1]].tolist(), dist[off[r]:off[r + 1]].tolist()))
            for r in range(len(off) - 1)]


def check_parents(ix, g, order, D) -> list[str]:
    """Section 6: the parent kept with (h, d) in L(v) is v's predecessor in
    the BFS tree of h -- v itself for d = 0, else a neighbour of v whose
    plain-BFS distance to h is d - 1 and which the BFS from h labeled at
    d - 1; of those, the lowest-ranked one (ranks: positions in `order`)."""
    fails = []
    rank = np.empty(ix.n, np.int64)
    rank[np.asarray(order)] = np.arange(ix.n)
    lab = label_maps(ix.off, ix.hub, ix.dist)
    for r in range(ix.n):
        a, b = int(ix.off[r]), int(ix.off[r + 1])
        v = int(order[r])
        nb = [int(rank[w]) for w in g.col[g.row_ptr[v]:g.row_ptr[v + 1]]]
        for h, d, p in zip(ix.hub[a:b], ix.dist[a:b], ix.par[a:b]):
            h, d, p = int(h), int(d), int(p)
            if d == 0:
                if p != r:
                    fails.append(f"rank {r}: self entry has parent {p}")
            elif not (0 <= p < ix.n) or p not in nb or D[order[h], order[p]] != d - 1:
                fails.append(f"rank {r}: entry ({h},{d}) has parent {p}")
            elif p != min((q for q in nb if lab[q].get(h) == d - 1), default=None):
                fails.append(f"rank {r}: entry ({h},{d}) has parent {p}, not the lowest-ranked "
                             "labeled one")
            if len(fails) >= 5:
                return fails
    return fails


def check_paths(ix, g, order, D) -> list[str]:
    """Paths restored from the labels (Section 6) are shortest paths: from s
    to t along edges with d(s,t) edges; none for unreachable pairs; a row
    too short reports -(d+1) and s = t gives [s]."""
    n = g.n
    if n == 0:
        return []
    s, t = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    pairs = np.stack([s.ravel(), t.ravel()], 1).astype(np.int32)
    P, L = oracle.paths(ix, pairs, n + 1)
    fails = []
    for i, (a, b) in enumerate(pairs):
        d = int(D[a, b])
        if d >= INF:
            if L[i] != 0:
                fails.append(f"path({a},{b}) of an unreachable pair: {L[i]}")
        elif L[i] != d + 1:
            fails.append(f"path({a},{b}) has {L[i]} vertices, d = {d}")
        else:
            p = [int(x) for x in P[i, :d + 1]]
            if p[0] != a or p[-1] != b:
                fails.append(f"path({a},{b}) = {p} has wrong ends")
            for x, y in zip(p[:-1], p[1:]):
                if y not in g.col[g.row_ptr[x]:g.row_ptr[x + 1]]:
                    fails.append(f"path({a},{b}) = {p} uses non-edge ({x},{y})")
                    break
        if len(fails) >= 5:
            return fails
    far = np.argwhere((D >= 1) & (D < INF))
    if len(far):
        a, b = far[0]
        _, L1 = oracle.paths(ix, np.array([[a, b]], np.int32), 1)
        if L1[0] != -(int(D[a, b]) + 1):
            fails.append(f"short row for ({a},{b}) gave {L1[0]}")
    return fails


ALL = (check_queries_vs_apsp, check_bp_selection, check_bp_closed_form,
       check_canonical_labels, check_hubs_not_above_vertex, check_query_parts,
       check_visited_counter, check_parents, check_paths)


def run_all(g, order, t_bp, lib=None, checks=ALL) -> list[str]:
    ix = oracle.build(g.row_ptr, g.col, order, t_bp, lib=lib)
    D = brute.apsp(g.row_ptr, g.col)
    fails = []
    for c in checks:
        if c is check_queries_vs_apsp:
            fails += c(ix, g, D)
        elif c is check_bp_selection:
            fails += c(ix, g, order)
        elif c in (check_bp_closed_form, check_query_parts, check_parents, check_paths):
            fails += c(ix, g, order, D)
        else:
            fails += c(ix, g, order)
    return fails


def degree(g):
    return gen.degree_order(g)
