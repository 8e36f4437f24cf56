"""GPU shortest-path queries (Section 6) against the graph and the oracle.

Both sides keep, with each label entry (h, d) of v, the lowest-ranked
neighbour of v that the BFS from h labeled at d - 1, and both take the
first best hub of the merge and the same bit-parallel walk rule, so the
exported parents and every restored path must equal the oracle's; the paths
are also checked against the graph (BFS length, a walk along edges from s
to t).  Runs only on an MI355X (``-m gpu``)."""
import numpy as np
import pytest

import brute
import graphs
import oracle
from paper_1304_4661_amd import binding, gen
from test_gpu_parity import Tuned, all_pairs, assert_same_index

pytestmark = pytest.mark.gpu
INF = 255


def _require_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"


def check_paths(g, pairs, P, L, D):
    for i, (s, t) in enumerate(pairs):
        d = int(D[s, t])
        if d >= INF:
            assert L[i] == 0, (s, t, L[i])
            continue
        assert L[i] == d + 1, (s, t, d, L[i])
        p = P[i, :L[i]]
        assert p[0] == s and p[-1] == t, (s, t, p)
        for x, y in zip(p[:-1], p[1:]):
            assert y in g.col[g.row_ptr[x]:g.row_ptr[x + 1]], (s, t, p)


def check_parents(g, order, gx, D, ox=None):
    """Every exported parent is the vertex itself (distance 0) or a
    neighbour one step closer to the hub; with the oracle, every parent
    equals its own."""
    e = gx.export()
    par = gx.export_parents()
    if ox is not None:
        assert np.array_equal(par, ox.par)
    for r in range(g.n):
        v = int(order[r])
        nb = g.col[g.row_ptr[v]:g.row_ptr[v + 1]]
        for k in range(int(e["off"][r]), int(e["off"][r + 1])):
            h, d, p = int(e["hub"][k]), int(e["dist"][k]), int(par[k])
            if d == 0:
                assert p == r
            else:
                assert int(order[p]) in nb and D[order[h], order[p]] == d - 1


FAMILIES = graphs.families()


@pytest.mark.parametrize("name,g", FAMILIES, ids=[f[0] for f in FAMILIES])
@pytest.mark.parametrize("t_bp", [0, 2, 64])
def test_paths_small_families(name, g, t_bp):
    _require_gpu()
    if g.n == 0:
        return
    order = gen.degree_order(g)
    ox = oracle.build(g.row_ptr, g.col, order, t_bp)
    gx = binding.build(g.row_ptr, g.col, order, t_bp, parents=True)
    assert_same_index(gx, ox, name)  # parents change nothing else
    D = brute.apsp(g.row_ptr, g.col)
    check_parents(g, order, gx, D, ox)
    p = all_pairs(g.n)
    P, L = gx.query_path(p, g.n + 1)
    check_paths(g, p, P, L, D)
    OP, OL = oracle.paths(ox, p, g.n + 1)
    assert np.array_equal(L, OL)
    assert np.array_equal(P, OP)


def test_paths_concurrent_windows_and_rmat():
    _require_gpu()
    g = gen.rmat_graph(12, seed=4)
    order = gen.degree_order(g)
    ox = oracle.build(g.row_ptr, g.col, order, 8)
    D = brute.apsp(g.row_ptr, g.col, sources=np.arange(0, g.n, 37))
    rng = np.random.default_rng(5)
    src = np.arange(0, g.n, 37)
    pairs = np.stack([np.repeat(src, 40), rng.integers(0, g.n, len(src) * 40)], 1).astype(np.int32)
    Dp = np.empty((g.n, g.n), np.int64)  # only the sampled rows are filled
    Dp[src] = D
    for knobs in (dict(window=64, window_work=0), dict(window=16384)):
        with Tuned(**knobs):
            gx = binding.build(g.row_ptr, g.col, order, 8, parents=True)
        assert_same_index(gx, ox, str(knobs))
        # the same parents whatever the window (no first-claimer choice)
        assert np.array_equal(gx.export_parents(), ox.par), str(knobs)
        P, L = gx.query_path(pairs, 64)
        check_paths(g, pairs, P, L, Dp)
        OP, OL = oracle.paths(ox, pairs, 64)
        assert np.array_equal(L, OL)
        assert np.array_equal(P, OP)


def test_paths_ba2000_workload():
    _require_gpu()
    g, order, t_bp, pairs = gen.config_graph("ba2000")
    ox = oracle.build(g.row_ptr, g.col, order, t_bp)
    gx = binding.build(g.row_ptr, g.col, order, t_bp, parents=True)
    D = brute.apsp(g.row_ptr, g.col)
    check_parents(g, order, gx, D, ox)
    P, L = gx.query_path(pairs, 16)
    check_paths(g, pairs, P, L, D)
    OP, OL = oracle.paths(ox, pairs, 16)
    assert np.array_equal(L, OL)
    assert np.array_equal(P, OP)


def test_path_row_too_short_and_unsupported():
    _require_gpu()
    g = graphs.path(9)
    order = gen.degree_order(g)
    gx = binding.build(g.row_ptr, g.col, order, 0, parents=True)
    P, L = gx.query_path(np.array([[0, 8], [3, 3], [2, 5]], np.int32), 4)
    assert L.tolist() == [-9, 1, 4]
    assert np.all(P[0] == -1) and P[1, 0] == 3 and P[2].tolist() == [2, 3, 4, 5]
    plain = binding.build(g.row_ptr, g.col, order, 0)
    with pytest.raises(binding.PllError):
        plain.query_path(np.array([[0, 1]], np.int32))
    with pytest.raises(binding.PllError):
        plain.export_parents()


def test_paths_in_a_batch():
    _require_gpu()
    gs = [gen.ba_graph(300, 2, 3), graphs.grid(5, 6), gen.ba_graph(150, 4, 8)]
    vtx_off, rp, col, order = gen.pack_batch(gs)
    gx = binding.build_batch(vtx_off, rp, col, order, 3, parents=True)
    rng = np.random.default_rng(2)
    for i, g in enumerate(gs):
        a = int(vtx_off[i])
        D = brute.apsp(g.row_ptr, g.col)
        loc = rng.integers(0, g.n, (400, 2)).astype(np.int32)
        P, L = gx.query_path(loc + a, 64)
        d = D[loc[:, 0], loc[:, 1]]
        assert np.array_equal(L, d + 1)
        for k in range(len(loc)):
            p = P[k, :L[k]] - a
            assert p[0] == loc[k, 0] and p[-1] == loc[k, 1]
            for x, y in zip(p[:-1], p[1:]):
                assert y in g.col[g.row_ptr[x]:g.row_ptr[x + 1]]
        ox = oracle.build(g.row_ptr, g.col, gen.degree_order(g), 3)
        par = gx.export_parents(i)
        e = gx.export(i)
        assert len(par) == len(e["hub"]) == len(ox.hub)
        assert np.array_equal(par, ox.par)
    # a pair across graphs has no path
    _, L = gx.query_path(np.array([[0, int(vtx_off[1])]], np.int32), 8)
    assert L[0] == 0


def test_paths_device_pointers():
    # the same answers through device buffers, and a bad id reported by
    # the call under PLL_SYNC without touching the outputs
    import torch

    _require_gpu()
    g, order, t_bp, pairs = gen.config_graph("ba2000")
    gx = binding.build(g.row_ptr, g.col, order, t_bp, parents=True)
    P, L = gx.query_path(pairs[:5000], 16)
    dp = torch.from_numpy(pairs[:5000]).cuda()
    paths = torch.full((5000, 16), -1, dtype=torch.int32, device="cuda")
    lens = torch.zeros(5000, dtype=torch.int32, device="cuda")
    gx.query_path_device(dp, paths, lens, sync=True)
    assert np.array_equal(lens.cpu().numpy(), L)
    # parents of a build are fixed: the same index gives the same paths
    assert np.array_equal(paths.cpu().numpy(), P)
    bad = dp.clone()
    bad[7, 1] = g.n
    lens.fill_(-5)
    with pytest.raises(binding.PllError):
        gx.query_path_device(bad, paths, lens, sync=True)
    assert int(lens.min()) == -5 and int(lens.max()) == -5
