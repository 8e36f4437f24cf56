"""GPU parity of weighted graphs (Section 6): the pruned Dijkstra labels of
the library against the oracle's, bit for bit, and every query answer
against the oracle (small graphs: all pairs) or against scipy's Dijkstra
(the full-size workload: every target of sampled sources)."""
import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import dijkstra

import graphs
import oracle
from paper_1304_4661_amd import binding, gen
from test_gpu_parity import Tuned, all_pairs

pytestmark = pytest.mark.gpu
WINF = binding.WINF


def _require_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"


def assert_same_weighted(gx, ox, tag=""):
    e = gx.export_weighted(0)
    assert np.array_equal(e["rank"], ox.rank), tag
    assert np.array_equal(e["off"], ox.off), f"{tag}: label sizes differ"
    assert np.array_equal(e["hub"], ox.hub), f"{tag}: hubs differ"
    assert np.array_equal(e["dist"], ox.dist), f"{tag}: distances differ"
    if ox.directed:
        i = gx.export_weighted(1)
        assert np.array_equal(i["off"], ox.in_off), f"{tag}: L_IN sizes differ"
        assert np.array_equal(i["hub"], ox.in_hub), f"{tag}: L_IN hubs differ"
        assert np.array_equal(i["dist"], ox.in_dist), f"{tag}: L_IN distances differ"
    assert gx.stats()["entries"] == ox.counters["entries"], tag


def _families():
    out = []
    for i, (name, g) in enumerate(graphs.families()):
        out.append((f"{name}_w10", gen.uniform_weights(g, 1, 10, 100 + i)))
        out.append((f"{name}_w1000", gen.uniform_weights(g, 1, 1000, 200 + i)))
    return out


WFAM = _families()


@pytest.mark.parametrize("name,g", WFAM, ids=[f[0] for f in WFAM])
def test_weighted_families(name, g):
    _require_gpu()
    order = gen.degree_order(g)
    ox = oracle.build_weighted(g.row_ptr, g.col, g.w, order)
    gx = binding.build_weighted(g.row_ptr, g.col, g.w, order, validate=True)
    assert_same_weighted(gx, ox, name)
    if g.n:
        pairs = all_pairs(g.n)
        want = oracle.query_weighted(ox, pairs)
        assert np.array_equal(gx.query_weighted(pairs), want)
        assert np.array_equal(gx.query_weighted(pairs, plain=True), want)


@pytest.mark.parametrize("window,wgroup,work", [
    (1, 16, 0), (3, 4, 0), (64, 64, 0), (700, 16, 0), (4096, 8, 0), (4096, 16, 1000),
    (4096, 32, 200000), (4096, 64, 30000)])
def test_weighted_windows_and_groups(window, wgroup, work):
    _require_gpu()
    g = gen.uniform_weights(gen.rmat_graph(11, seed=4), 1, 100, 6)
    order = gen.degree_order(g)
    ox = oracle.build_weighted(g.row_ptr, g.col, g.w, order)
    with Tuned(window=window, wgroup=wgroup, wwork=work):
        gx = binding.build_weighted(g.row_ptr, g.col, g.w, order)
    assert_same_weighted(gx, ox, f"window={window} wgroup={wgroup} work={work}")


@pytest.mark.parametrize("lo,hi", [(1, 100000), (20000, 60000), (60000, 70000), (1, 3)])
def test_weighted_landmark_saturation(lo, hi):
    # distances beyond 16 bits weaken the landmark bound of later windows
    # (saturated landmark distances are left out); labels must not change
    _require_gpu()
    g = gen.uniform_weights(gen.rmat_graph(11, seed=8), lo, hi, 10)
    order = gen.degree_order(g)
    ox = oracle.build_weighted(g.row_ptr, g.col, g.w, order)
    with Tuned(window=4096, wwork=4000):
        gx = binding.build_weighted(g.row_ptr, g.col, g.w, order)
    assert_same_weighted(gx, ox, f"weights [{lo}, {hi}]")
    pairs = gen.random_pairs(g.n, 50_000, 2)
    assert np.array_equal(gx.query_weighted(pairs), oracle.query_weighted(ox, pairs))


def test_weighted_plain_build():
    _require_gpu()
    g = gen.uniform_weights(gen.ba_graph(600, 3, 2), 1, 50, 3)
    order = gen.random_order(g.n, 4)
    ox = oracle.build_weighted(g.row_ptr, g.col, g.w, order)
    assert_same_weighted(binding.build_weighted(g.row_ptr, g.col, g.w, order, plain=True), ox,
                         "plain")


@pytest.mark.parametrize("knobs", [dict(list_cap=1, window=256, wwork=0),
                                   dict(table_cap=1, window=128, wwork=0),
                                   dict(list_cap=5000, table_cap=64, window=1024, wwork=0)])
def test_weighted_overflow_retries(knobs):
    # lists or root tables too small: windows are re-run (fewer roots, or
    # bigger tables) until they fit; the result must not change
    _require_gpu()
    g = gen.uniform_weights(gen.rmat_graph(10, seed=5), 1, 20, 2)
    order = gen.degree_order(g)
    ox = oracle.build_weighted(g.row_ptr, g.col, g.w, order)
    with Tuned(**knobs):
        gx = binding.build_weighted(g.row_ptr, g.col, g.w, order)
    assert gx.stats()["retries"] > 0
    assert_same_weighted(gx, ox, str(knobs))


def test_weighted_small_workload():
    # BA n=2000, m=4, weights uniform in [1, 100], 1e5 pairs
    _require_gpu()
    g, order, t_bp, pairs = gen.config_graph("ba2000w")
    ox = oracle.build_weighted(g.row_ptr, g.col, g.w, order)
    gx = binding.build_weighted(g.row_ptr, g.col, g.w, order)
    assert_same_weighted(gx, ox, "ba2000w")
    want = oracle.query_weighted(ox, pairs)
    assert np.array_equal(gx.query_weighted(pairs), want)
    assert np.array_equal(gx.query_weighted(pairs, plain=True), want)


def test_unit_weights_match_the_unweighted_build():
    _require_gpu()
    g = gen.rmat_graph(11, seed=6)
    order = gen.degree_order(g)
    gw = binding.build_weighted(g.row_ptr, g.col, np.ones(len(g.col), np.uint32), order)
    gu = binding.build(g.row_ptr, g.col, order, 0)
    a, b = gw.export_weighted(0), gu.export()
    assert np.array_equal(a["off"], b["off"]) and np.array_equal(a["hub"], b["hub"])
    assert np.array_equal(a["dist"], b["dist"].astype(np.uint32))


def test_weighted_range_rule():
    # weights 2^30 on a path: distances of 2^32 or more are not stored and
    # read as WINF; large weights near the limit still sum exactly in 64 bits
    _require_gpu()
    p = graphs.path(7)
    for w in (1 << 30, (1 << 31) + 5, 0xFFFFFFF0):
        g = gen.Graph(p.n, p.row_ptr, p.col, {}, np.full(len(p.col), w, np.uint32))
        order = gen.degree_order(g)
        ox = oracle.build_weighted(g.row_ptr, g.col, g.w, order)
        gx = binding.build_weighted(g.row_ptr, g.col, g.w, order)
        assert_same_weighted(gx, ox, f"w={w}")
        pairs = all_pairs(g.n)
        got = gx.query_weighted(pairs)
        assert np.array_equal(got, oracle.query_weighted(ox, pairs))
        d = np.abs(pairs[:, 0] - pairs[:, 1]).astype(np.int64) * w
        assert np.array_equal(got.astype(np.int64), np.where(d >= WINF, WINF, d))


DIG = [("er60", gen.er_digraph(60, 0.05, 2)), ("er150", gen.er_digraph(150, 0.03, 5)),
       ("rmat9", gen.rmat_digraph(9, 8, seed=4)), ("rmat11", gen.rmat_digraph(11, 8, seed=7))]


@pytest.mark.parametrize("name,g", DIG, ids=[d[0] for d in DIG])
@pytest.mark.parametrize("window", [1, 64, 4096])
def test_weighted_digraphs(name, g, window):
    _require_gpu()
    g = gen.uniform_weights(g, 1, 30, 9)
    order = gen.degree_order_directed(g)
    ox = oracle.build_weighted(g.row_ptr, g.col, g.w, order, directed=True)
    with Tuned(window=window, wwork=0):
        gx = binding.build_weighted(g.row_ptr, g.col, g.w, order, directed=True)
    assert_same_weighted(gx, ox, f"{name} window={window}")
    pairs = all_pairs(g.n) if g.n <= 400 else gen.random_pairs(g.n, 200_000, 3)
    want = oracle.query_weighted(ox, pairs)
    assert np.array_equal(gx.query_weighted(pairs), want)
    assert np.array_equal(gx.query_weighted(pairs, plain=True), want)


def test_weighted_device_pointers_and_errors():
    import torch
    _require_gpu()
    g = gen.uniform_weights(gen.rmat_graph(10, seed=3), 1, 100, 4)
    order = gen.degree_order(g)
    ox = oracle.build_weighted(g.row_ptr, g.col, g.w, order)
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).to(dev)  # noqa: E731
    gx = binding.build_weighted(t(g.row_ptr), t(g.col), t(g.w), t(order), device=True)
    assert_same_weighted(gx, ox, "device")
    pairs = gen.random_pairs(g.n, 20_000, 8)
    dp = torch.from_numpy(pairs).to(dev)
    out = torch.empty(len(pairs), dtype=torch.int32, device=dev)
    gx.query_weighted_device(dp, out, sync=True)
    assert np.array_equal(out.cpu().numpy().view(np.uint32), oracle.query_weighted(ox, pairs))
    bad = dp.clone()
    bad[3, 0] = g.n
    with pytest.raises(binding.PllError):
        gx.query_weighted_device(bad, out, sync=True)
    # a zero weight is rejected by the device-side check
    w0 = g.w.copy()
    w0[5] = 0
    with pytest.raises(binding.PllError):
        binding.build_weighted(t(g.row_ptr), t(g.col), t(w0), t(order), device=True)
    # the unweighted calls refuse a weighted index and vice versa
    with pytest.raises(binding.PllError):
        gx.query(pairs)
    with pytest.raises(binding.PllError):
        gx.export()
    gu = binding.build(g.row_ptr, g.col, order, 0)
    with pytest.raises(binding.PllError):
        gu.query_weighted(pairs)


def test_weighted_deterministic_rebuild():
    _require_gpu()
    g = gen.uniform_weights(gen.rmat_graph(12, seed=2), 1, 100, 5)
    order = gen.degree_order(g)
    a = binding.build_weighted(g.row_ptr, g.col, g.w, order).export_weighted(0)
    b = binding.build_weighted(g.row_ptr, g.col, g.w, order).export_weighted(0)
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_weighted_rmat18_workload_sampled():
    # the benchmark workload (R-MAT 18, weights in [1, 100]) in the launch
    # configuration the benchmark times: every target of 24 sampled sources
    # against scipy's Dijkstra, the benchmark pairs against the same
    # distances where their source was sampled, and label invariants
    _require_gpu()
    g, order, _, pairs = gen.config_graph("rmat18w")
    gx = binding.build_weighted(g.row_ptr, g.col, g.w, order)
    rng = np.random.default_rng(12)
    src = rng.choice(g.n, 24, replace=False)
    a = csr_matrix((g.w.astype(np.float64), g.col, g.row_ptr), shape=(g.n, g.n))
    D = dijkstra(a, directed=False, indices=src)
    want = np.where(np.isfinite(D), D, WINF).astype(np.uint64)
    for i, s in enumerate(src):
        q = np.stack([np.full(g.n, s, np.int32), np.arange(g.n, dtype=np.int32)], 1)
        got = gx.query_weighted(q)
        assert np.array_equal(got.astype(np.uint64), want[i]), f"source {s}"
    e = gx.export_weighted(0)
    rank = e["rank"]
    # every label holds its own vertex at distance 0 as its last entry, hubs
    # strictly ascending, and each stored distance is the exact one for the
    # sampled hubs
    lens = np.diff(e["off"])
    assert np.all(lens >= 1)
    last = e["off"][1:] - 1
    assert np.array_equal(e["hub"][last], np.arange(g.n)) and np.all(e["dist"][last] == 0)
    inv = np.empty(g.n, np.int64)
    inv[rank] = np.arange(g.n)
    srank = rank[src]
    for i, s in enumerate(src):
        hits = np.flatnonzero(e["hub"] == srank[i])
        owners = np.searchsorted(e["off"], hits, side="right") - 1
        assert np.array_equal(e["dist"][hits].astype(np.uint64), want[i][inv[owners]])


def test_weighted_query_autotune():
    _require_gpu()
    g, order, _, pairs = gen.config_graph("ba2000w")
    ox = oracle.build_weighted(g.row_ptr, g.col, g.w, order)
    gx = binding.build_weighted(g.row_ptr, g.col, g.w, order)
    with Tuned(qgroup=64):
        assert gx.autotune_query(pairs[:20000]) in (16, 32, 64)
        assert np.array_equal(gx.query_weighted(pairs), oracle.query_weighted(ox, pairs))


def test_weighted_without_landmarks():
    _require_gpu()
    g = gen.uniform_weights(gen.rmat_graph(11, seed=12), 1, 50, 13)
    order = gen.degree_order(g)
    ox = oracle.build_weighted(g.row_ptr, g.col, g.w, order)
    with Tuned(landmarks=0, wwork=20000):
        gx = binding.build_weighted(g.row_ptr, g.col, g.w, order)
    assert_same_weighted(gx, ox, "no landmarks")
    assert gx.stats()["land_checks"] == 0


WPATH = [("rmat10_w50", gen.uniform_weights(gen.rmat_graph(10, seed=21), 1, 50, 22), False),
         ("ba600_w9", gen.uniform_weights(gen.ba_graph(600, 3, 5), 1, 9, 23), False),
         ("grid_w3", gen.uniform_weights(graphs.grid(12, 15), 1, 3, 24), False),
         ("er150d_w20", gen.uniform_weights(gen.er_digraph(150, 0.03, 25), 1, 20, 26), True),
         ("rmat9d_w30", gen.uniform_weights(gen.rmat_digraph(9, 8, seed=27), 1, 30, 28), True)]


@pytest.mark.parametrize("name,g,directed", WPATH, ids=[w[0] for w in WPATH])
@pytest.mark.parametrize("window", [1, 64, 4096])
def test_weighted_paths(name, g, directed, window):
    # Section 6 paths on weighted graphs: labels as without parents; every
    # restored path follows edges (arcs) from s to t with weights summing to
    # the distance; parents are tight predecessors in the hub's search tree
    from test_oracle_weighted import edge_weights
    _require_gpu()
    order = gen.degree_order_directed(g) if directed else gen.degree_order(g)
    ox = oracle.build_weighted(g.row_ptr, g.col, g.w, order, directed=directed)
    with Tuned(window=window, wwork=0):
        gx = binding.build_weighted(g.row_ptr, g.col, g.w, order, directed=directed,
                                    parents=True)
    assert_same_weighted(gx, ox, f"{name} window={window}")
    ew = edge_weights(g)
    pairs = all_pairs(g.n) if g.n <= 200 else gen.random_pairs(g.n, 40_000, 5)
    want = oracle.query_weighted(ox, pairs).astype(np.int64)
    paths, lens = gx.query_path(pairs, max_len=g.n + 1)
    opaths, olens = oracle.paths_weighted(ox, pairs, g.n + 1)
    assert np.array_equal(lens, olens) and np.array_equal(paths, opaths)
    reach = want < WINF
    assert np.all(lens[~reach] == 0) and np.all(lens[reach] > 0)
    for i in np.flatnonzero(reach):
        p = paths[i, :lens[i]].tolist()
        hops = list(zip(p, p[1:]))
        assert p[0] == pairs[i, 0] and p[-1] == pairs[i, 1]
        assert all(x in ew for x in hops) and sum(ew[x] for x in hops) == want[i], (pairs[i], p)
    # too little room: nothing written, -(vertices) reported
    short = gx.query_path(pairs[:2000], max_len=1)[1]
    long_ = lens[:2000]
    assert np.all(short[long_ > 1] == -long_[long_ > 1])
    # parents: tight predecessors (L / L_IN) or successors (L_OUT)
    a = csr_matrix((g.w.astype(np.float64), g.col, g.row_ptr), shape=(g.n, g.n))
    D = dijkstra(a, directed=directed)
    sides = [(0, "out" if directed else "in")] + ([(1, "in")] if directed else [])
    for side, kind in sides:
        e = gx.export_weighted(side)
        par = gx.export_weighted_parents(side)
        # both sides keep the lowest-ranked tight predecessor (successor)
        assert np.array_equal(par, ox.par if side == 0 else ox.in_par), (name, side)
        owner = np.repeat(np.arange(g.n), np.diff(e["off"]))
        v, h, pp = order[owner], order[e["hub"]], order[par]
        d = e["dist"].astype(np.float64)
        z = d == 0
        assert np.all(pp[z] == v[z])
        for vv, hh, p_, dd in zip(v[~z].tolist(), h[~z].tolist(), pp[~z].tolist(), d[~z].tolist()):
            if kind == "out":
                assert (vv, p_) in ew and ew[(vv, p_)] + D[p_, hh] == dd
            else:
                assert (p_, vv) in ew and D[hh, p_] + ew[(p_, vv)] == dd


def test_weighted_rmat18_workload_equals_the_oracle():
    # the benchmark's weighted workload array for array against oracle O8
    # (pruned Dijkstra searches, about half a minute on one host core), and
    # the benchmark's 1e6 pairs
    _require_gpu()
    g, order, _, pairs = gen.config_graph("rmat18w")
    ox = oracle.build_weighted(g.row_ptr, g.col, g.w, order)
    gx = binding.build_weighted(g.row_ptr, g.col, g.w, order)
    assert_same_weighted(gx, ox, "rmat18w")
    assert np.array_equal(gx.query_weighted(pairs), oracle.query_weighted(ox, pairs))
