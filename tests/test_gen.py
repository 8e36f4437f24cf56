"""Input generators: determinism and the CSR conventions every input obeys."""
import os

import numpy as np
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import connected_components

from paper_1304_4661_amd import gen

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _check_csr(g):
    rp, col = g.row_ptr, g.col
    assert rp.dtype == np.int32 and col.dtype == np.int32
    assert rp[0] == 0 and np.all(np.diff(rp) >= 0) and rp[-1] == len(col)
    src = np.repeat(np.arange(g.n), np.diff(rp))
    assert np.all(src != col), "self-loop"
    for v in range(0, g.n, max(1, g.n // 50)):
        row = col[rp[v]:rp[v + 1]]
        assert np.all(np.diff(row) > 0), "row not strictly sorted"
    a = csr_matrix((np.ones(len(col)), col, rp), shape=(g.n, g.n))
    assert (a != a.T).nnz == 0, "not symmetric"


def test_ba_shape_and_determinism():
    g = gen.ba_graph(500, 4, 3)
    _check_csr(g)
    assert g.m == 4 * (500 - 4)
    a = csr_matrix((np.ones(len(g.col)), g.col, g.row_ptr), shape=(g.n, g.n))
    assert connected_components(a, directed=False)[0] == 1
    g2 = gen.ba_graph(500, 4, 3)
    assert gen.csr_sha256(g) == gen.csr_sha256(g2)
    assert gen.csr_sha256(g) != gen.csr_sha256(gen.ba_graph(500, 4, 4))


def test_ba2000_named_workload():
    g, order, t_bp, pairs = gen.config_graph("ba2000")
    assert g.n == 2000 and g.m == 7984 and t_bp == 16
    assert pairs.shape == (100_000, 2) and pairs.min() >= 0 and pairs.max() < 2000


def test_rmat_cleanup():
    g = gen.rmat_graph(12, seed=9)
    _check_csr(g)
    a = csr_matrix((np.ones(len(g.col)), g.col, g.row_ptr), shape=(g.n, g.n))
    assert connected_components(a, directed=False)[0] == 1
    assert g.n <= 4096 and g.m <= 16 * 4096
    assert gen.csr_sha256(g) == gen.csr_sha256(gen.rmat_graph(12, seed=9))


def test_rmat_quadrant_probabilities():
    u, v = gen.rmat_edges(1, 1 << 16, 0.57, 0.19, 0.19, seed=1)
    q = np.bincount(u * 2 + v, minlength=4) / len(u)
    assert np.allclose(q, [0.57, 0.19, 0.19, 0.05], atol=0.01)


def test_degree_order_ties_by_id():
    from graphs import from_edges
    g = from_edges(5, [(0, 1), (2, 3), (2, 4), (1, 3)])
    # degrees: 1,2,2,2,1
    assert gen.degree_order(g).tolist() == [1, 2, 3, 0, 4]


def test_batch_spec_and_pack():
    spec = gen.batch_spec(8, n_lo=50, n_hi=400)
    assert len(spec) == 8 and all(50 <= n <= 400 and 2 <= m <= 8 for n, m, _ in spec)
    gs = [gen.ba_graph(n, m, s) for n, m, s in spec]
    vtx_off, rp, col, order = gen.pack_batch(gs)
    assert vtx_off[-1] == sum(g.n for g in gs)
    for i, g in enumerate(gs):
        a, b = vtx_off[i], vtx_off[i + 1]
        assert np.array_equal(rp[a:b + 1] - rp[a], g.row_ptr)
        assert np.array_equal(col[rp[a]:rp[b]] - a, g.col)
        assert np.array_equal(order[a:b], gen.degree_order(g))


def test_native_ba_matches_python_loop():
    for n, m, s in [(2000, 4, 1), (1500, 8, 7), (64, 2, 3)]:
        a = gen.ba_edges(n, m, s)
        b = gen.ba_edges_fast(n, m, s)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_digraph_generators():
    g = gen.digraph_from_edges(5, np.array([0, 0, 1, 2, 3, 3]), np.array([1, 1, 1, 0, 4, 2]))
    assert g.row_ptr.tolist() == [0, 1, 1, 2, 4, 4] and g.col.tolist() == [1, 0, 2, 4]
    assert g.meta["directed"]
    d = gen.rmat_digraph(10, 8, seed=3)
    a = csr_matrix((np.ones(len(d.col)), d.col, d.row_ptr), shape=(d.n, d.n))
    assert connected_components(a, directed=True, connection="weak")[0] == 1
    src = np.repeat(np.arange(d.n), np.diff(d.row_ptr))
    assert np.all(src != d.col)
    assert gen.csr_sha256(d) == gen.csr_sha256(gen.rmat_digraph(10, 8, seed=3))
    # in+out degree descending, ties by id
    g2 = gen.digraph_from_edges(4, np.array([0, 1, 2]), np.array([1, 2, 3]))
    assert gen.degree_order_directed(g2).tolist() == [1, 2, 0, 3]


def test_closeness_order():
    from graphs import from_edges
    # path 0-1-2-3-4: the middle is most central, then its neighbours (ties by id)
    p = from_edges(5, [(0, 1), (1, 2), (2, 3), (3, 4)])
    assert gen.closeness_order(p, samples=5).tolist() == [2, 1, 3, 0, 4]
    # star: the centre first whatever the sample
    st = from_edges(6, [(0, i) for i in range(1, 6)])
    assert gen.closeness_order(st, samples=2, seed=3)[0] == 0
    g = gen.ba_graph(300, 3, 5)
    o = gen.closeness_order(g, samples=16, seed=1)
    assert sorted(o.tolist()) == list(range(g.n))
    assert np.array_equal(o, gen.closeness_order(g, samples=16, seed=1))


def test_batch_workload_recipe():
    # the 256-graph batch as stated for the benchmark: sizes drawn
    # log-uniformly in [1e3, 2e5] (seeds 4000 + i), 8,888,217 vertices and
    # 41,301,184 undirected edges in all; 72 graphs have at most 4,096
    # vertices (the ones built whole by default)
    spec = gen.batch_spec(256, seed_base=4000)
    assert len(spec) == 256 and all(1000 <= n <= 200_000 and 2 <= m <= 8 for n, m, _ in spec)
    assert sum(n for n, _, _ in spec) == 8_888_217
    assert sum(1 for n, _, _ in spec if n <= 4096) == 72
    gs = [gen.ba_graph(n, m, s) for n, m, s in spec]
    assert sum(int(g.row_ptr[-1]) for g in gs) // 2 == 41_301_184


def test_generators_reproduce_the_full_size_digests():
    # the stored full-size oracle results were made from these exact CSRs
    # (tests/golden/make_full_digests.py); the GPU's full-size parity
    # tests compare against them, so the inputs must not drift
    import json
    gold = json.load(open(os.path.join(GOLDEN, "full_rmat20.json")))
    g, order, _, _ = gen.config_graph("rmat20")
    assert gen.csr_sha256(g, order) == gold["csr_sha256"]
    gold = json.load(open(os.path.join(GOLDEN, "full_ba256.json")))
    spec = gen.batch_spec(256, seed_base=4000)
    for i, (n, m, s) in enumerate(spec):
        g = gen.ba_graph(n, m, s)
        assert gen.csr_sha256(g, gen.degree_order(g)) == gold["graphs"][i]["csr_sha256"], i
