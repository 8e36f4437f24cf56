"""Pins of the oracle's directed labels (Section 6, "Directed Graphs").

L_OUT(v) holds (h, d(v,h)) and L_IN(v) holds (h, d(h,v)); the merge of
L_OUT(s) and L_IN(t) must give the directed BFS distance, and each label
must be exactly its canonical form: (h, d) is in L_IN(v) iff h is the
lowest-ranked vertex on every shortest h->v path (and the same for L_OUT
with v->h paths), checked here by brute force with scipy's BFS."""
import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import shortest_path

import graphs
import oracle
import pins
from paper_1304_4661_amd import gen

INF = 255


def dapsp(g):
    if g.n == 0:
        return np.zeros((0, 0), np.int64)
    a = csr_matrix((np.ones(len(g.col)), g.col, g.row_ptr), shape=(g.n, g.n))
    d = shortest_path(a, unweighted=True, directed=True)
    return np.where(np.isinf(d), INF, d).astype(np.int64)


def digraphs():
    out = [("er40", gen.er_digraph(40, 0.06, 1)), ("er60", gen.er_digraph(60, 0.03, 2)),
           ("er80dense", gen.er_digraph(80, 0.12, 3)), ("rmat8", gen.rmat_digraph(8, 8, seed=4))]
    n = 12
    out.append(("path", gen.digraph_from_edges(n, np.arange(n - 1), np.arange(1, n))))
    out.append(("cycle", gen.digraph_from_edges(n, np.arange(n), (np.arange(n) + 1) % n)))
    u, v = np.nonzero(np.triu(np.random.default_rng(7).random((30, 30)) < 0.15, 1))
    out.append(("dag", gen.digraph_from_edges(30, u, v)))
    out.append(("out_star", gen.digraph_from_edges(9, np.zeros(8, int), np.arange(1, 9))))
    out.append(("in_star", gen.digraph_from_edges(9, np.arange(1, 9), np.zeros(8, int))))
    out.append(("single", gen.digraph_from_edges(1, np.zeros(0, int), np.zeros(0, int))))
    return out


def labels(off, hub, dist, n):
    return [set(zip(hub[off[r]:off[r + 1]].tolist(), dist[off[r]:off[r + 1]].tolist()))
            for r in range(n)]


def check_directed(g, order, lib=None):
    fails = []
    ix = oracle.build_directed(g.row_ptr, g.col, order, lib=lib)
    D = dapsp(g)
    n = g.n
    if n:
        s, t = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        pairs = np.stack([s.ravel(), t.ravel()], 1).astype(np.int32)
        q = oracle.query_directed(ix, pairs).astype(np.int64).reshape(n, n)
        bad = np.argwhere(q != np.minimum(D, INF))
        fails += [f"query({a},{b}) = {q[a, b]} != {D[a, b]}" for a, b in bad[:3]]
    rank = np.empty(n, np.int64)
    rank[order] = np.arange(n)
    exp_in = [set() for _ in range(n)]
    exp_out = [set() for _ in range(n)]
    for h in range(n):
        for v in range(n):
            d = D[h, v]
            if d >= INF:
                continue
            on = (D[h, :] + D[:, v] == d) & (D[h, :] < INF) & (D[:, v] < INF)
            lo = rank[np.nonzero(on)[0]].min()
            if lo == rank[h]:  # (h, d(h,v)) in L_IN(v)
                exp_in[rank[v]].add((int(rank[h]), int(d)))
            if lo == rank[v]:  # (v, d(h,v)) in L_OUT(h)
                exp_out[rank[h]].add((int(rank[v]), int(d)))
    got_in = labels(ix.in_off, ix.in_hub, ix.in_dist, n)
    got_out = labels(ix.out_off, ix.out_hub, ix.out_dist, n)
    for r in range(n):
        if got_in[r] != exp_in[r]:
            fails.append(f"L_IN(rank {r}) = {sorted(got_in[r])} != {sorted(exp_in[r])}")
        if got_out[r] != exp_out[r]:
            fails.append(f"L_OUT(rank {r}) = {sorted(got_out[r])} != {sorted(exp_out[r])}")
        if len(fails) > 5:
            break
    for off, hub in ((ix.in_off, ix.in_hub), (ix.out_off, ix.out_hub)):
        for r in range(n):
            h = hub[off[r]:off[r + 1]]
            if np.any(np.diff(h.astype(np.int64)) <= 0):
                fails.append(f"label of rank {r} not sorted")
                break
    fails += check_directed_parents(g, order, ix, D)
    fails += check_directed_paths(g, ix, D, lib)
    return fails


def arcs_of(g):
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    return set(zip(rows.tolist(), g.col.tolist()))


def check_directed_parents(g, order, ix, D):
    """Parent of v for (h, d) in L_IN(v): an in-neighbour p of v with
    d(h, p) = d - 1 (v itself at d = 0); in L_OUT(v): an out-neighbour p
    with d(p, h) = d - 1.  Of those whose label on the same side holds
    (h, d - 1), the lowest-ranked one.  Parents and hubs are ranks."""
    fails = []
    arcs = arcs_of(g)
    rank = np.empty(g.n, np.int64)
    rank[np.asarray(order)] = np.arange(g.n)
    ins = {v: [] for v in range(g.n)}
    outs = {v: [] for v in range(g.n)}
    for a, b in arcs:
        outs[a].append(b)
        ins[b].append(a)
    for side, (off, hub, dist, par) in (("L_IN", (ix.in_off, ix.in_hub, ix.in_dist, ix.in_par)),
                                        ("L_OUT", (ix.out_off, ix.out_hub, ix.out_dist,
                                                   ix.out_par))):
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
                elif side == "L_IN":
                    ok = (p, v) in arcs and D[h, p] == d - 1
                else:
                    ok = (v, p) in arcs and D[p, h] == d - 1
                if ok and d > 0:
                    nb = ins[v] if side == "L_IN" else outs[v]
                    ok = int(rank[p]) == min((int(rank[q]) for q in nb
                                              if lab[rank[q]].get(int(hub[e])) == d - 1),
                                             default=None)
                if not ok:
                    fails.append(f"{side} parent of rank {r} for hub {h}: {p}")
                    return fails
    return fails


def check_directed_paths(g, ix, D, lib=None):
    """Every restored path follows arcs from s to t with d(s, t) + 1
    vertices; unreachable pairs give 0."""
    fails = []
    n = g.n
    if n == 0:
        return fails
    arcs = arcs_of(g)
    s, t = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    pairs = np.stack([s.ravel(), t.ravel()], 1).astype(np.int32)
    paths, lens = oracle.paths(ix, pairs, 64)
    for i, (a, b) in enumerate(pairs.tolist()):
        d = D[a, b]
        if d >= INF:
            if lens[i] != 0:
                fails.append(f"path({a},{b}) unreachable but len {lens[i]}")
            continue
        if lens[i] != d + 1:
            fails.append(f"path({a},{b}) len {lens[i]} != {d + 1}")
            continue
        pth = paths[i, :d + 1].tolist()
        if pth[0] != a or pth[-1] != b or any((x, y) not in arcs for x, y in zip(pth, pth[1:])):
            fails.append(f"path({a},{b}) = {pth} is not a path along the arcs")
        if len(fails) > 3:
            break
    return fails


DG = digraphs()


@pytest.mark.parametrize("name,g", DG, ids=[x[0] for x in DG])
def test_directed_pins(name, g):
    assert not check_directed(g, gen.degree_order_directed(g))
    if g.n > 1:
        assert not check_directed(g, gen.random_order(g.n, 11))


def test_symmetric_input_reduces_to_undirected():
    # both arc directions present: L_OUT = L_IN = the undirected labels
    for g in (graphs.grid(4, 5), gen.ba_graph(120, 3, 12), graphs.erdos_renyi(60, 0.05, 4)):
        order = gen.degree_order(g)
        ux = oracle.build(g.row_ptr, g.col, order, 0)
        dx = oracle.build_directed(g.row_ptr, g.col, order)
        for off, hub, dist in ((dx.out_off, dx.out_hub, dx.out_dist),
                               (dx.in_off, dx.in_hub, dx.in_dist)):
            assert np.array_equal(off, ux.off) and np.array_equal(hub, ux.hub)
            assert np.array_equal(dist, ux.dist)


MUTATIONS = [
    ("reverse search follows the arcs",
     "rc = directed_bfs(x, k, ioff, iadj, off, adj, x->lab, x->lab_in, P, T, queue);",
     "rc = directed_bfs(x, k, off, adj, ioff, iadj, x->lab, x->lab_in, P, T, queue);"),
    ("forward search prunes with the root's in-label",
     "rc = directed_bfs(x, k, off, adj, ioff, iadj, x->lab_in, x->lab, P, T, queue);",
     "rc = directed_bfs(x, k, off, adj, ioff, iadj, x->lab_in, x->lab_in, P, T, queue);"),
    ("directed parent recorded as the search root",
     "uint32_t par = d == 0 ? (uint32_t)k : tree_parent(own, poff, padj, u, k, d);",
     "uint32_t par = (uint32_t)k;"),
    ("directed parents looked up along the search's own direction",
     "rc = directed_bfs(x, k, off, adj, ioff, iadj, x->lab_in, x->lab, P, T, queue);",
     "rc = directed_bfs(x, k, off, adj, off, adj, x->lab_in, x->lab, P, T, queue);"),
    ("directed path ascends L_OUT from the target",
     "    int64_t e = find_hub(&x->lab_in[c], h);\n    if (e < 0) return ORC_E_RANGE;\n    c = (int32_t)x->lab_in[c].par[e];",
     "    int64_t e = find_hub(&x->lab[c], h);\n    if (e < 0) return ORC_E_RANGE;\n    c = (int32_t)x->lab[c].par[e];"),
    ("query merges L_OUT(s) with L_OUT(t)",
     "*B = x->lab_in ? &x->lab_in[rt] : &x->lab[rt];", "*B = &x->lab[rt];"),
    ("any directed BFS level reaching 255 is a range error",
     "    if (t_query(&own[u], T) <= d) continue;\n",
     "    if (d < (int)ORC_INF && t_query(&own[u], T) <= d) continue;\n"),
    ("transpose keeps the arcs' direction",
     "iadj[ioff[adj[j]] + fill[adj[j]]++] = r;", "iadj[ioff[adj[j]] + fill[adj[j]]++] = adj[j];"),
]


@pytest.mark.parametrize("desc,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_directed_pins_catch_planted_mistake(desc, old, new, tmp_path):
    src = oracle.source_text()
    assert src.count(old) == 1, desc
    lib = oracle.load_variant(src.replace(old, new), str(tmp_path))
    caught = False
    cases = [(g, gen.degree_order_directed(g)) for _, g in DG[:4]]
    cases.append(graphs.level_255_pruned())
    for g, order in cases:
        try:
            caught |= bool(check_directed(g, order, lib=lib))
        except oracle.OracleError:
            caught = True
    assert caught, desc
