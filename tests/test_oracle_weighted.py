"""Pins of the oracle's weighted labels (Section 6, "Weighted Graphs").

The pruned Dijkstra search must give (a) query answers equal to Dijkstra
distances from scipy, (b) exactly the canonical labels: (h, d) is in L(v)
iff d = d(h, v) and h is the lowest-ranked vertex on every shortest h-v
path (for a digraph: L_IN with h->v paths, L_OUT with v->h paths), checked
by brute force over all-pairs distances, (c) the unweighted labels when
every weight is 1, (d) distances scaled by c when every weight is, and (e)
the 32-bit range rule: a distance of 2^32 - 1 or more is not stored and
reads as unreachable.  Planted mistakes in a copy of the oracle must fail
one of these."""
import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import dijkstra

import graphs
import oracle
import pins
from paper_1304_4661_amd import gen

WINF = oracle.WINF


def wapsp(g, directed=False):
    """All-pairs distances as int64 (WINF where unreachable or >= WINF)."""
    if g.n == 0:
        return np.zeros((0, 0), np.int64)
    a = csr_matrix((g.w.astype(np.float64), g.col, g.row_ptr), shape=(g.n, g.n))
    d = dijkstra(a, directed=directed)
    out = np.full(d.shape, WINF, np.int64)
    fin = np.isfinite(d)
    out[fin] = d[fin].astype(np.int64)
    return np.minimum(out, WINF)


def canonical(D, order):
    """Per rank r: {(k, D[k][r])} over ranks k that are the lowest-ranked
    vertex on every shortest k->r path (D in rank space, WINF = none)."""
    n = len(order)
    Dr = D[np.ix_(order, order)]
    out = [set() for _ in range(n)]
    for k in range(n):
        dk = Dr[k]
        for r in range(n):
            d = dk[r]
            if d >= WINF:
                continue
            on = (dk + Dr[:, r] == d) & (dk < WINF) & (Dr[:, r] < WINF)
            if np.flatnonzero(on).min() == k:
                out[r].add((k, int(d)))
    return out


def labels(off, hub, dist, n):
    return [set(zip(hub[off[r]:off[r + 1]].tolist(), dist[off[r]:off[r + 1]].tolist()))
            for r in range(n)]


def check_weighted(g, order, directed=False, lib=None):
    fails = []
    ix = oracle.build_weighted(g.row_ptr, g.col, g.w, order, directed=directed, lib=lib)
    D = wapsp(g, directed)
    n = g.n
    if n:
        s, t = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        pairs = np.stack([s.ravel(), t.ravel()], 1).astype(np.int32)
        q = oracle.query_weighted(ix, pairs).astype(np.int64).reshape(n, n)
        bad = np.argwhere(q != D)
        fails += [f"query({a},{b}) = {q[a, b]} != {D[a, b]}" for a, b in bad[:3]]
    for r in range(n):
        h = ix.hub[ix.off[r]:ix.off[r + 1]]
        if np.any(np.diff(h.astype(np.int64)) <= 0):
            fails.append(f"label of rank {r} not strictly sorted")
    if directed:
        want_in = canonical(D, order)                 # k -> r paths
        want_out = canonical(D.T.copy(), order)       # r -> k paths
        if labels(ix.in_off, ix.in_hub, ix.in_dist, n) != want_in:
            fails.append("L_IN differs from its canonical form")
        if labels(ix.off, ix.hub, ix.dist, n) != want_out:
            fails.append("L_OUT differs from its canonical form")
    elif labels(ix.off, ix.hub, ix.dist, n) != canonical(D, order):
        fails.append("labels differ from their canonical form")
    if ix.counters["entries"] != len(ix.hub) + (len(ix.in_hub) if directed else 0):
        fails.append("entry counter")
    fails += check_weighted_parents(g, order, ix, D, directed)
    fails += check_weighted_paths(g, ix, D, directed)
    return fails


def edge_weights(g):
    """Smallest weight of each arc (u, v) of the CSR."""
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    w = {}
    for u, v, x in zip(rows.tolist(), g.col.tolist(), g.w.tolist()):
        w[(u, v)] = min(x, w.get((u, v), x))
    return w


def check_weighted_parents(g, order, ix, D, directed):
    """Parent p of v for (h, d): v itself at d = 0; else an edge p -> v
    (undirected: p - v) with d(h, p) + w(p, v) = d for L (L_IN), and an arc
    v -> p with w(v, p) + d(p, h) = d for L_OUT of a digraph; of the
    vertices q with such an edge whose label on the same side holds
    (h, d - w), the lowest-ranked one."""
    fails = []
    ew = edge_weights(g)
    rank = np.empty(g.n, np.int64)
    rank[np.asarray(order)] = np.arange(g.n)
    ins = {v: [] for v in range(g.n)}
    outs = {v: [] for v in range(g.n)}
    for (a, b) in ew:
        outs[a].append(b)
        ins[b].append(a)
    sides = [("L" if not directed else "L_OUT", ix.off, ix.hub, ix.dist, ix.par)]
    if directed:
        sides.append(("L_IN", ix.in_off, ix.in_hub, ix.in_dist, ix.in_par))
    for side, off, hub, dist, par in sides:
        lab = pins.label_maps(off, hub, dist)
        for r in range(g.n):
            v = int(order[r])
            for e in range(int(off[r]), int(off[r + 1])):
                if int(par[e]) >= g.n:
                    fails.append(f"{side} parent of rank {r}: none ({int(par[e])})")
                    return fails
                h, d, p = int(order[hub[e]]), int(dist[e]), int(order[par[e]])
                if d == 0:
                    ok = p == v
                elif side == "L_OUT":
                    ok = (v, p) in ew and ew[(v, p)] + D[p, h] == d
                else:
                    ok = (p, v) in ew and D[h, p] + ew[(p, v)] == d
                if ok and d > 0:
                    if side == "L_OUT":
                        cand = [q for q in outs[v] if lab[rank[q]].get(int(hub[e])) ==
                                d - ew[(v, q)]]
                    else:
                        cand = [q for q in ins[v] if lab[rank[q]].get(int(hub[e])) ==
                                d - ew[(q, v)]]
                    ok = int(rank[p]) == min((int(rank[q]) for q in cand), default=None)
                if not ok:
                    fails.append(f"{side} parent of rank {r} for hub {h}: {p}")
                    return fails
    return fails


def check_weighted_paths(g, ix, D, directed):
    """Every restored path follows edges (arcs) from s to t and its weights
    sum to d(s, t); unreachable pairs give 0."""
    fails = []
    n = g.n
    if n == 0:
        return fails
    ew = edge_weights(g)
    s, t = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    pairs = np.stack([s.ravel(), t.ravel()], 1).astype(np.int32)
    paths, lens = oracle.paths_weighted(ix, pairs, n + 1)
    for i, (a, b) in enumerate(pairs.tolist()):
        d = D[a, b]
        if d >= WINF:
            if lens[i] != 0:
                fails.append(f"path({a},{b}) unreachable but len {lens[i]}")
            continue
        if lens[i] <= 0:
            fails.append(f"path({a},{b}) missing (len {lens[i]})")
            continue
        pth = paths[i, :lens[i]].tolist()
        hops = list(zip(pth, pth[1:]))
        if pth[0] != a or pth[-1] != b or any(x not in ew for x in hops) or \
                sum(ew[x] for x in hops) != d:
            fails.append(f"path({a},{b}) = {pth} is not a shortest path")
        if len(fails) > 3:
            break
    return fails


def weighted_families():
    out = []
    for i, (name, g) in enumerate(graphs.families()):
        if g.n > 70:
            continue
        out.append((f"{name}_w10", gen.uniform_weights(g, 1, 10, 100 + i)))
        out.append((f"{name}_w1000", gen.uniform_weights(g, 1, 1000, 200 + i)))
    out.append(("ba150_w3", gen.uniform_weights(gen.ba_graph(150, 3, 4), 1, 3, 9)))
    return out


def weighted_digraphs():
    out = []
    for i, (name, g) in enumerate([("er40", gen.er_digraph(40, 0.06, 1)),
                                   ("er60", gen.er_digraph(60, 0.05, 2)),
                                   ("rmat7", gen.rmat_digraph(7, 8, seed=4))]):
        out.append((f"{name}_w20", gen.uniform_weights(g, 1, 20, 300 + i)))
    return out


WFAM = weighted_families()
WDIG = weighted_digraphs()


@pytest.mark.parametrize("name,g", WFAM, ids=[f[0] for f in WFAM])
def test_weighted_pins_degree(name, g):
    assert not check_weighted(g, gen.degree_order(g))


@pytest.mark.parametrize("name,g", WFAM[::3], ids=[f[0] for f in WFAM[::3]])
def test_weighted_pins_random_order(name, g):
    assert not check_weighted(g, gen.random_order(g.n, 5))


@pytest.mark.parametrize("name,g", WDIG, ids=[f[0] for f in WDIG])
def test_weighted_digraph_pins(name, g):
    assert not check_weighted(g, gen.degree_order_directed(g), directed=True)
    assert not check_weighted(g, gen.random_order(g.n, 3), directed=True)


@pytest.mark.parametrize("name,g", graphs.families()[:10], ids=[f[0] for f in graphs.families()[:10]])
def test_unit_weights_are_the_unweighted_labels(name, g):
    o = gen.degree_order(g)
    w = oracle.build_weighted(g.row_ptr, g.col, np.ones(len(g.col), np.uint32), o)
    u = oracle.build(g.row_ptr, g.col, o, 0)
    assert np.array_equal(w.off, u.off) and np.array_equal(w.hub, u.hub)
    assert np.array_equal(w.dist, u.dist.astype(np.uint32))


def test_unit_weight_digraph_is_the_unweighted_digraph():
    g = gen.er_digraph(50, 0.06, 8)
    o = gen.degree_order_directed(g)
    w = oracle.build_weighted(g.row_ptr, g.col, np.ones(len(g.col), np.uint32), o, directed=True)
    u = oracle.build_directed(g.row_ptr, g.col, o)
    assert np.array_equal(w.hub, u.out_hub) and np.array_equal(w.in_hub, u.in_hub)
    assert np.array_equal(w.dist, u.out_dist.astype(np.uint32))
    assert np.array_equal(w.in_dist, u.in_dist.astype(np.uint32))


def test_scaled_weights_scale_distances():
    g = gen.uniform_weights(gen.ba_graph(120, 2, 3), 1, 50, 4)
    o = gen.degree_order(g)
    a = oracle.build_weighted(g.row_ptr, g.col, g.w, o)
    b = oracle.build_weighted(g.row_ptr, g.col, g.w * np.uint32(7), o)
    assert np.array_equal(a.off, b.off) and np.array_equal(a.hub, b.hub)
    assert np.array_equal(a.dist.astype(np.int64) * 7, b.dist.astype(np.int64))


def test_range_rule_drops_far_distances():
    # a path of 6 vertices with weights 2^30: d(0, 4) = 2^32 does not fit
    p = graphs.path(6)
    g = gen.Graph(p.n, p.row_ptr, p.col, {}, np.full(len(p.col), 1 << 30, np.uint32))
    assert not check_weighted(g, gen.degree_order(g))
    ix = oracle.build_weighted(g.row_ptr, g.col, g.w, gen.degree_order(g))
    assert int(ix.dist.max()) == 3 << 30
    q = oracle.query_weighted(ix, np.array([[0, 3], [0, 4], [1, 5], [2, 2]], np.int32))
    assert q.tolist() == [3 << 30, WINF, WINF, 0]


def test_zero_or_asymmetric_weights_rejected():
    g = gen.uniform_weights(graphs.cycle(6), 1, 9, 1)
    w = g.w.copy()
    w[0] = 0
    with pytest.raises(oracle.OracleError):
        oracle.build_weighted(g.row_ptr, g.col, w, gen.degree_order(g))
    w = g.w.copy()
    w[0] += 1
    with pytest.raises(oracle.OracleError):
        oracle.build_weighted(g.row_ptr, g.col, w, gen.degree_order(g))
    oracle.build_weighted(g.row_ptr, g.col, w, gen.degree_order(g), check_symmetric=False)


def test_weighted_generator_is_symmetric():
    g = gen.uniform_weights(gen.rmat_graph(9, seed=2), 1, 100, 3)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    fwd = dict(zip(zip(rows.tolist(), g.col.tolist()), g.w.tolist()))
    assert all(fwd[(v, u)] == w for (u, v), w in fwd.items())
    assert g.w.min() >= 1 and g.w.max() <= 100


MUTATIONS = [
    ("parent recorded as the search root",
     "uint32_t par = d == 0 ? (uint32_t)k : wtree_parent(lab, poff, padj, pw, u, k, d);",
     "uint32_t par = (uint32_t)k;"),
    ("parent of a weighted entry one edge of weight 1 closer",
     "L->dist[L->len - 1] == d - pw[j] &&", "L->dist[L->len - 1] == d - 1 &&"),
    ("path ascends the source side from the target",
     "  int64_t ct = wascend(x, tl, rt, h, NULL, 0, 1, 0);",
     "  int64_t ct = wascend(x, x->in ? x->in : x->out, rs, h, NULL, 0, 1, 0);"),
    ("prune test strict", "if (th != ORC_WINF && (uint64_t)L->dist[i] + th <= d) pruned = 1;",
     "if (th != ORC_WINF && (uint64_t)L->dist[i] + th < d) pruned = 1;"),
    ("relaxation ignores the weight", "uint64_t nd = (uint64_t)d + wgt[j];",
     "uint64_t nd = (uint64_t)d + 1;"),
    ("vertices tested when first reached, not when settled (BFS order)",
     "    uint64_t key = wheap_pop(heap);",
     "    uint64_t key = heap->a[--heap->len];"),
    ("T not reset after a root",
     "  for (int64_t i = 0; i < Lk->len; i++) T[Lk->hub[i]] = ORC_WINF;\n  return rc;", "  return rc;"),
    ("pruned vertices also relax their edges", "    if (pruned) continue;\n", ""),
    ("reverse search prunes with the wrong root labels",
     "rc = weighted_search(x, k, ioff, iadj, iaw, off, adj, aw, x->out, x->in,",
     "rc = weighted_search(x, k, ioff, iadj, iaw, off, adj, aw, x->out, x->out,"),
    ("merge join on 32-bit sums", "uint64_t v = (uint64_t)A->dist[i] + B->dist[j];",
     "uint64_t v = (uint32_t)(A->dist[i] + B->dist[j]);"),
]


@pytest.mark.parametrize("desc,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_weighted_pins_catch_planted_mistake(desc, old, new, tmp_path):
    src = oracle.source_text()
    assert src.count(old) == 1, desc
    lib = oracle.load_variant(src.replace(old, new), str(tmp_path))
    p = graphs.path(6)
    big = gen.Graph(p.n, p.row_ptr, p.col, {}, np.full(len(p.col), 3 << 29, np.uint32))
    cases = [(g, False) for _, g in WFAM[:: max(1, len(WFAM) // 8)]] + [(big, False)]
    cases += [(g, True) for _, g in WDIG]
    caught = False
    for g, directed in cases:
        order = gen.degree_order_directed(g) if directed else gen.degree_order(g)
        try:
            if check_weighted(g, order, directed=directed, lib=lib):
                caught = True
                break
        except oracle.OracleError:
            caught = True
            break
    assert caught, f"planted mistake not caught: {desc}"
