"""GPU parity of batched builds: every graph of a batch must equal the
oracle's index of that graph alone, bit for bit, and queries must answer each
graph's distances (255 across graphs)."""
import numpy as np
import pytest

import graphs
import oracle
from paper_1304_4661_amd import binding, gen
from test_gpu_parity import Tuned, assert_same_index

pytestmark = pytest.mark.gpu


def _require_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"


def _check_batch(gs, t_bp, seed=0, device=False, **tune):
    vtx_off, rp, col, order = gen.pack_batch(gs)
    with Tuned(**tune):
        if device:
            import torch
            d = [torch.from_numpy(a).cuda() for a in (rp, col, order)]
            bx = binding.build_batch(vtx_off, *d, t_bp, device=True)
        else:
            bx = binding.build_batch(vtx_off, rp, col, order, t_bp, validate=True)
    oxs = []
    for i, g in enumerate(gs):
        ox = oracle.build(g.row_ptr, g.col, gen.degree_order(g), t_bp)
        assert_same_index(_GraphView(bx, i), ox, f"graph {i}")
        oxs.append(ox)
    # queries: within graphs against each oracle, across graphs 255
    rng = np.random.Generator(np.random.PCG64(seed))
    N = int(vtx_off[-1])
    p = rng.integers(0, N, (20000, 2)).astype(np.int32)
    got = bx.query(p)
    gof = np.searchsorted(vtx_off, p, side="right") - 1
    same = gof[:, 0] == gof[:, 1]
    assert np.all(got[~same] == 255)
    for i in range(len(gs)):
        sel = same & (gof[:, 0] == i)
        if sel.any():
            loc = (p[sel] - vtx_off[i]).astype(np.int32)
            assert np.array_equal(got[sel], oracle.query(oxs[i], loc)), f"graph {i} queries"
    assert np.array_equal(bx.query(p, plain=True), got)
    return bx


class _GraphView:
    """Adapter so assert_same_index can export one graph of a batch."""

    def __init__(self, ix, g):
        self.ix, self.g = ix, g

    def export(self):
        return self.ix.export(self.g)


def test_batch_of_families():
    _require_gpu()
    gs = [g for _, g in graphs.families() if g.n > 0]
    for t_bp in (0, 3, 16):
        _check_batch(gs, t_bp, seed=t_bp)


def test_batch_of_ba_graphs_small_windows():
    # every graph is small enough to be built whole by one workgroup; with
    # whole_n = 0 the same batch goes through the shared windows
    _require_gpu()
    spec = gen.batch_spec(24, seed_base=500, n_lo=50, n_hi=1500)
    gs = [gen.ba_graph(n, m, s) for n, m, s in spec]
    bx = _check_batch(gs, 16, seed=3)
    assert bx.stats()["whole_graphs"] == 24 and bx.stats()["windows"] == 0
    bx = _check_batch(gs, 16, seed=4, window=7, group=8, whole_n=0)
    assert bx.stats()["whole_graphs"] == 0 and bx.stats()["windows"] > 0


def test_batch_whole_and_windowed_graphs_mixed():
    # graphs of at most whole_n vertices are built whole (one workgroup per
    # graph, ranks after the interleaved ones), the others share windows;
    # each equals its oracle, and queries across the two kinds answer 255
    _require_gpu()
    gs = [gen.ba_graph(n, m, 40 + i) for i, (n, m) in
          enumerate([(1800, 3), (300, 2), (2500, 5), (64, 1), (900, 4), (4000, 2)])]
    gs.insert(3, graphs.disjoint_union(graphs.cycle(9), graphs.star(12), graphs.empty(3)))
    gs.insert(6, graphs.empty(1))
    gs.append(gen.rmat_graph(11, seed=8))
    for t_bp, lim in ((16, 1000), (0, 1000), (64, 2048), (5, 16384)):
        bx = _check_batch(gs, t_bp, seed=t_bp, whole_n=lim)
        want = sum(1 for g in gs if g.n <= lim)
        assert bx.stats()["whole_graphs"] == want, (t_bp, lim)
        assert (bx.stats()["windows"] > 0) == (want < len(gs)), (t_bp, lim)


def test_batch_whole_pool_runs_out():
    # a pool of one entry per vertex cannot hold the labels: the launch is
    # redone with twice the pool until it fits, and the labels are the same
    _require_gpu()
    gs = [gen.ba_graph(n, 3, 70 + n) for n in (700, 1500, 250)]
    bx = _check_batch(gs, 8, seed=9, whole_pool=1)
    assert bx.stats()["retries"] >= 2 and bx.stats()["whole_graphs"] == 3


def test_batch_whole_graph_distance_255():
    # Section 4.5.1's 8-bit distances inside one workgroup: the BFS from a_0
    # reaches w at 255 and prunes it there (the build succeeds, as the
    # oracle's does); a path of 257 vertices has a pair 256 apart and fails
    # with PLL_E_RANGE
    _require_gpu()
    g255, o255 = graphs.level_255_pruned()
    gs = [gen.ba_graph(500, 3, 11), g255, graphs.path(40)]
    orders = [gen.degree_order(gs[0]), o255, gen.degree_order(gs[2])]
    vtx_off = np.zeros(len(gs) + 1, np.int64)
    vtx_off[1:] = np.cumsum([g.n for g in gs])
    _, rp, col, _ = gen.pack_batch(gs)
    order = np.concatenate(orders).astype(np.int32)
    for t_bp in (0, 1):
        bx = binding.build_batch(vtx_off, rp, col, order, t_bp, validate=True)
        assert bx.stats()["whole_graphs"] == 3
        for i, (g, o) in enumerate(zip(gs, orders)):
            ox = oracle.build(g.row_ptr, g.col, o, t_bp)
            assert_same_index(_GraphView(bx, i), ox, f"graph {i} t_bp={t_bp}")
        p = np.stack(np.meshgrid(np.arange(260), np.arange(260)), -1).reshape(-1, 2)
        p = (p + vtx_off[1]).astype(np.int32)
        want = oracle.query(oracle.build(g255.row_ptr, g255.col, o255, t_bp),
                             (p - vtx_off[1]).astype(np.int32))
        assert np.array_equal(bx.query(p), want)
    bad = [gen.ba_graph(300, 2, 12), graphs.path(257)]
    vtx_off, rp, col, order = gen.pack_batch(bad)
    for t_bp in (0, 1):
        with pytest.raises(binding.PllError) as e:
            binding.build_batch(vtx_off, rp, col, order, t_bp)
        assert e.value.code == binding.E_RANGE


def test_batch_device_pointers_and_single_graph_batch():
    _require_gpu()
    g = gen.ba_graph(900, 3, 8)
    _check_batch([g], 8, device=True)
    _check_batch([graphs.star(70), gen.ba_graph(300, 2, 9), graphs.path(40)], 1, device=True)


def test_batch_solo_equivalence():
    # each graph of a batch equals its own pll_build export
    _require_gpu()
    gs = [gen.rmat_graph(10, seed=s) for s in (1, 2, 3)] + [gen.ba_graph(700, 4, 5)]
    vtx_off, rp, col, order = gen.pack_batch(gs)
    bx = binding.build_batch(vtx_off, rp, col, order, 16)
    for i, g in enumerate(gs):
        solo = binding.build(g.row_ptr, g.col, gen.degree_order(g), 16).export()
        part = bx.export(i)
        for k in solo:
            assert np.array_equal(solo[k], part[k]), (i, k)


def test_persistent_queries_and_recorded_batches():
    # the persistent batched form (groups take chunks of pairs from a shared
    # cursor) and a query batch recorded as a HIP graph answer exactly as the
    # static form, for a batch index (cross-graph pairs 255) and a single
    # graph; every replay is checked after eager work on the same stream,
    # with the pairs changed in place between replays
    import torch
    _require_gpu()
    gs = [gen.ba_graph(n, m, 900 + n) for n, m in ((300, 2), (1200, 3), (2500, 4))]
    vtx_off, rp, col, order = gen.pack_batch(gs)
    bx = binding.build_batch(vtx_off, rp, col, order, 8)
    N = int(vtx_off[-1])
    rng = np.random.Generator(np.random.PCG64(17))
    for q in (1, 777, 200_000):
        p = rng.integers(0, N, (q, 2)).astype(np.int32)
        want = bx.query(p)
        for persist in (0, 1):
            with Tuned(qpersist=persist):
                assert np.array_equal(bx.query(p), want), (q, persist)
                dp = torch.from_numpy(p).cuda()
                out = torch.full((q,), 7, dtype=torch.uint8, device="cuda")
                bx.query_device(dp, out, sync=True)
                assert np.array_equal(out.cpu().numpy(), want)
                assert np.array_equal(bx.query_noalloc(p), want)
                qg = binding.QueryGraph(bx, dp, out)
            for r in range(3):
                p2 = rng.integers(0, N, (q, 2)).astype(np.int32)
                dp.copy_(torch.from_numpy(p2))
                out.fill_(7)
                bx.query(p2[: max(1, q // 3)])  # eager work between replays
                qg.launch()
                qg.status()
                assert np.array_equal(out.cpu().numpy(), bx.query(p2)), (q, persist, r)
            # an out-of-range id: the replay writes nothing and reports it
            bad = p2.copy()
            bad[-1, 0] = N
            dp.copy_(torch.from_numpy(bad))
            out.fill_(9)
            qg.launch()
            with pytest.raises(binding.PllError):
                qg.status()
            assert int((out != 9).sum()) == 0
            qg.close()


def test_query_autotune_chooses_a_form():
    _require_gpu()
    g = gen.ba_graph(3000, 4, 5)
    gx = binding.build(g.row_ptr, g.col, gen.degree_order(g), 16)
    p = gen.random_pairs(g.n, 50_000, 6)
    want = gx.query(p)
    old = binding.get_tuning("qpersist"), binding.get_tuning("qgroup")
    try:
        assert gx.autotune_query(p) in (16, 32, 64)
        assert binding.get_tuning("qpersist") in (0, 1)
        assert np.array_equal(gx.query(p), want)
    finally:
        binding.set_tuning("qpersist", old[0])
        binding.set_tuning("qgroup", old[1])


def test_build_autotune():
    # the frontier-tile autotuner settles on values from its candidate sets
    # and the build it leaves behind still gives the oracle's labels
    import torch
    _require_gpu()
    g = gen.rmat_graph(13, seed=9)
    order = gen.degree_order(g)
    keys = ("xgroup", "chunk", "window_work", "sort_level")
    old = {k: binding.get_tuning(k) for k in keys}
    try:
        d = [torch.from_numpy(a).cuda() for a in (g.row_ptr, g.col, order)]
        best = binding.autotune_build(*d, 16)
        assert best["xgroup"] in (8, 16, 32) and best["chunk"] in (128, 256, 512)
        assert best["window_work"] in (64000000, 128000000, 256000000)
        assert best["sort_level"] in (1 << 18, 1 << 20, 1 << 22)
        assert all(binding.get_tuning(k) == best[k] for k in keys)
        ox = oracle.build(g.row_ptr, g.col, order, 16)
        assert_same_index(binding.build_device(*d, 16), ox, "after build autotune")
    finally:
        for k, v in old.items():
            binding.set_tuning(k, v)


def test_build_and_query_in_one_call():
    # pll_build_query_batch: a graph built whole answers its own pairs inside
    # the whole-graph launch, the others are answered after the build; every
    # answer equals the graph's oracle and pll_query on the returned index,
    # with host and device pointers, with and without whole graphs, and a
    # graph without pairs in the middle
    import torch
    _require_gpu()
    gs = [gen.ba_graph(n, m, 80 + i) for i, (n, m) in
          enumerate([(6000, 3), (300, 2), (1500, 4), (5000, 2), (64, 1), (900, 3)])]
    gs.insert(2, graphs.disjoint_union(graphs.cycle(9), graphs.star(12), graphs.empty(3)))
    vtx_off, rp, col, order = gen.pack_batch(gs)
    rng = np.random.Generator(np.random.PCG64(31))
    counts = [0 if i == 4 else 700 + 150 * i for i in range(len(gs))]
    qoff = np.zeros(len(gs) + 1, np.int64)
    qoff[1:] = np.cumsum(counts)
    pairs = np.concatenate([rng.integers(vtx_off[i], vtx_off[i + 1], (c, 2))
                            for i, c in enumerate(counts)]).astype(np.int32)
    want = np.concatenate([oracle.query(oracle.build(g.row_ptr, g.col, gen.degree_order(g), 16),
                                        (pairs[qoff[i]:qoff[i + 1]] - vtx_off[i]).astype(np.int32))
                           for i, g in enumerate(gs)])
    for lim in (4096, 0):
        with Tuned(whole_n=lim):
            ix, got = binding.build_query_batch(vtx_off, rp, col, order, 16, qoff, pairs,
                                                validate=True)
            st = ix.stats()
            assert np.array_equal(got, want), lim
            assert np.array_equal(ix.query(pairs), want), lim
            whole = [i for i, g in enumerate(gs) if g.n <= lim]
            assert st["whole_graphs"] == len(whole)
            assert st["whole_pairs"] == sum(counts[i] for i in whole)
            ix.close()
            d = [torch.from_numpy(a).cuda() for a in (rp, col, order, pairs)]
            out = torch.full((len(pairs),), 7, dtype=torch.uint8, device="cuda")
            ix, got = binding.build_query_batch(vtx_off, *d[:3], 16, qoff, d[3], out=out,
                                                device=True)
            assert np.array_equal(got.cpu().numpy(), want), lim
            ix.close()
    with pytest.raises(binding.PllError):  # an id past the batch (device pointers)
        bad = torch.from_numpy(pairs).cuda()
        bad[5, 1] = int(vtx_off[-1])
        binding.build_query_batch(vtx_off, *d[:3], 16, qoff, bad, device=True)
