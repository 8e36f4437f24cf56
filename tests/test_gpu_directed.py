"""GPU directed builds (Section 6) against the oracle, array for array:
L_OUT (pll_export), L_IN (pll_export_in) and every query answer.  Runs only
on an MI355X (``-m gpu``)."""
import numpy as np
import pytest

import graphs
import oracle
from paper_1304_4661_amd import binding, gen
from test_gpu_parity import Tuned, all_pairs
from test_oracle_directed import digraphs

pytestmark = pytest.mark.gpu


def _require_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"


def assert_same_directed(gx, ox, tag=""):
    o = gx.export()
    i = gx.export_in()
    assert np.array_equal(o["rank"], ox.rank), tag
    assert np.array_equal(o["off"], ox.out_off), f"{tag}: L_OUT sizes"
    assert np.array_equal(o["hub"], ox.out_hub) and np.array_equal(o["dist"], ox.out_dist), tag
    assert np.array_equal(i["off"], ox.in_off), f"{tag}: L_IN sizes"
    assert np.array_equal(i["hub"], ox.in_hub) and np.array_equal(i["dist"], ox.in_dist), tag


DG = digraphs()


@pytest.mark.parametrize("name,g", DG, ids=[x[0] for x in DG])
@pytest.mark.parametrize("knobs", [{}, dict(window=3, window_work=0), dict(window=1, window_work=0)],
                         ids=["adaptive", "w3", "w1"])
def test_directed_families(name, g, knobs):
    _require_gpu()
    order = gen.degree_order_directed(g)
    ox = oracle.build_directed(g.row_ptr, g.col, order)
    with Tuned(**knobs):
        gx = binding.build(g.row_ptr, g.col, order, 0, directed=True)
    assert_same_directed(gx, ox, name)
    if g.n:
        p = all_pairs(g.n)
        want = oracle.query_directed(ox, p)
        assert np.array_equal(gx.query(p), want)
        assert np.array_equal(gx.query(p, plain=True), want)


def test_directed_rmat_and_overflow():
    _require_gpu()
    g = gen.rmat_digraph(12, 8, seed=6)
    order = gen.degree_order_directed(g)
    ox = oracle.build_directed(g.row_ptr, g.col, order)
    pairs = gen.random_pairs(g.n, 50000, 3)
    want = oracle.query_directed(ox, pairs)
    for knobs in ({}, dict(window=256, window_work=0), dict(list_cap=1, window=128, window_work=0),
                  dict(table_cap=8)):
        with Tuned(**knobs):
            gx = binding.build(g.row_ptr, g.col, order, 0, directed=True)
        assert_same_directed(gx, ox, str(knobs))
        assert np.array_equal(gx.query(pairs), want)


def test_symmetric_directed_equals_undirected():
    _require_gpu()
    g = gen.ba_graph(500, 3, 21)
    order = gen.degree_order(g)
    u = binding.build(g.row_ptr, g.col, order, 0).export()
    dx = binding.build(g.row_ptr, g.col, order, 0, directed=True)
    for e in (dx.export(), dx.export_in()):
        assert np.array_equal(e["off"], u["off"]) and np.array_equal(e["hub"], u["hub"])
        assert np.array_equal(e["dist"], u["dist"])


def test_directed_batch_and_errors():
    _require_gpu()
    gs = [gen.er_digraph(50, 0.05, 1), gen.rmat_digraph(9, 8, seed=2), gen.er_digraph(70, 0.03, 4)]
    vtx_off, rp, col, order = gen.pack_batch(gs, order_fn=gen.degree_order_directed)
    gx = binding.build_batch(vtx_off, rp, col, order, 0, directed=True)
    for i, g in enumerate(gs):
        ox = oracle.build_directed(g.row_ptr, g.col, gen.degree_order_directed(g))
        e, ei = gx.export(i), gx.export_in(i)
        assert np.array_equal(e["hub"], ox.out_hub) and np.array_equal(ei["hub"], ox.in_hub)
        p = all_pairs(g.n)
        assert np.array_equal(gx.query(p + np.int32(vtx_off[i])), oracle.query_directed(ox, p))
    assert gx.query(np.array([[0, int(vtx_off[1])]], np.int32))[0] == 255
    g = gs[0]
    with pytest.raises(binding.PllError):
        binding.build(g.row_ptr, g.col, gen.degree_order_directed(g), 2, directed=True)
    with pytest.raises(binding.PllError):
        binding.build(g.row_ptr, g.col, gen.degree_order_directed(g), 0).export_in()
    # L_IN parents need a directed index built with parents
    with pytest.raises(binding.PllError):
        binding.build(g.row_ptr, g.col, gen.degree_order_directed(g), 0,
                      directed=True).export_in_parents()


@pytest.mark.parametrize("landmarks", [0, 1])
@pytest.mark.parametrize("window", [64, 4096])
def test_directed_landmark_rows(landmarks, window):
    # the landmark rows of the first window only skip work: labels equal
    _require_gpu()
    g = gen.rmat_digraph(12, 8, seed=11)
    order = gen.degree_order_directed(g)
    ox = oracle.build_directed(g.row_ptr, g.col, order)
    with Tuned(landmarks=landmarks, window=window, window_work=0):
        gx = binding.build(g.row_ptr, g.col, order, 0, directed=True)
    assert_same_directed(gx, ox, f"landmarks={landmarks} window={window}")
    st = gx.stats()
    if not landmarks:
        assert st["bp_direct"] == 0
    elif window < g.n:  # rows are used from the second window on
        assert st["bp_direct"] > 0


DPATH = [("er60", gen.er_digraph(60, 0.05, 2)), ("rmat9", gen.rmat_digraph(9, 8, seed=4)),
         ("rmat12", gen.rmat_digraph(12, 8, seed=5))]


@pytest.mark.parametrize("name,g", DPATH, ids=[d[0] for d in DPATH])
@pytest.mark.parametrize("window", [1, 64, 4096])
def test_directed_paths(name, g, window):
    # Section 6 paths on a digraph: labels as without parents, every path
    # follows the arcs with d(s, t) + 1 vertices, parents of both labels are
    # valid BFS-tree parents
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import shortest_path
    _require_gpu()
    order = gen.degree_order_directed(g)
    ox = oracle.build_directed(g.row_ptr, g.col, order)
    with Tuned(window=window, window_work=0):
        gx = binding.build(g.row_ptr, g.col, order, 0, directed=True, parents=True)
    assert_same_directed(gx, ox, f"{name} window={window}")
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    arcs = set(zip(rows.tolist(), g.col.tolist()))
    pairs = all_pairs(g.n) if g.n <= 600 else gen.random_pairs(g.n, 100_000, 4)
    want = oracle.query_directed(ox, pairs).astype(np.int64)
    paths, lens = gx.query_path(pairs, max_len=64)
    opaths, olens = oracle.paths(ox, pairs, 64)
    assert np.array_equal(lens, olens)
    assert np.array_equal(paths, opaths)
    reach = want < 255
    assert np.array_equal(lens[reach], want[reach] + 1) and np.all(lens[~reach] == 0)
    for i in np.flatnonzero(reach)[:20000]:
        p = paths[i, :lens[i]].tolist()
        assert p[0] == pairs[i, 0] and p[-1] == pairs[i, 1]
        assert all((a, b) in arcs for a, b in zip(p, p[1:])), (pairs[i], p)
    # parents: ranks; L_OUT parent is an out-neighbour one step closer to h,
    # L_IN parent an in-neighbour one step further from h
    a = csr_matrix((np.ones(len(g.col)), g.col, g.row_ptr), shape=(g.n, g.n))
    D = shortest_path(a, unweighted=True, directed=True)
    e = gx.export()
    po = gx.export_parents()
    ei = gx.export_in()
    pi = gx.export_in_parents()
    assert np.array_equal(po, ox.out_par) and np.array_equal(pi, ox.in_par)
    for (off, hub, dist, par, side) in ((e["off"], e["hub"], e["dist"], po, "out"),
                                        (ei["off"], ei["hub"], ei["dist"], pi, "in")):
        owner = np.repeat(np.arange(g.n), np.diff(off))
        v = order[owner]
        h = order[hub]
        p = order[par]
        d = dist.astype(np.int64)
        z = d == 0
        assert np.all(p[z] == v[z])
        nz = ~z
        if side == "out":
            assert all((x, y) in arcs for x, y in zip(v[nz].tolist(), p[nz].tolist()))
            assert np.array_equal(D[p[nz], h[nz]], d[nz] - 1)
        else:
            assert all((y, x) in arcs for x, y in zip(v[nz].tolist(), p[nz].tolist()))
            assert np.array_equal(D[h[nz], p[nz]], d[nz] - 1)


def test_directed_level_255_reached_but_pruned():
    # both searches from a_0 reach w at 255 and prune it there (the graph as
    # a digraph with both arcs of every edge); windows re-run on the range
    # flag, the plain form does not need to
    _require_gpu()
    g, order = graphs.level_255_pruned()
    ox = oracle.build_directed(g.row_ptr, g.col, order)
    p = all_pairs(g.n)
    want = oracle.query_directed(ox, p)
    for kw in ({}, {"plain": True}):
        gx = binding.build(g.row_ptr, g.col, order, 0, directed=True, **kw)
        assert_same_directed(gx, ox, f"level255 {kw}")
        assert np.array_equal(gx.query(p), want)
