"""GPU parity: the HIP library against the CPU oracle, bit for bit.

Every index array (labels, bit-parallel labels, ranks) and every query answer
must equal the oracle's.  Runs only on an MI355X (``-m gpu``)."""
import os

import numpy as np
import pytest

import graphs
import oracle
from paper_1304_4661_amd import binding, gen

pytestmark = pytest.mark.gpu


def _require_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"


def assert_same_index(gx, ox, tag=""):
    e = gx.export()
    assert np.array_equal(e["rank"], ox.rank), tag
    assert np.array_equal(e["off"], ox.off), f"{tag}: label sizes differ"
    assert np.array_equal(e["hub"], ox.hub), f"{tag}: hubs differ"
    assert np.array_equal(e["dist"], ox.dist), f"{tag}: distances differ"
    assert np.array_equal(e["bp_d"], ox.bp_d), f"{tag}: bit-parallel distances differ"
    assert np.array_equal(e["bp_m1"], ox.bp_m1), f"{tag}: S^-1 differ"
    assert np.array_equal(e["bp_0"], ox.bp_0), f"{tag}: S^0 differ"


def all_pairs(n):
    s, t = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return np.stack([s.ravel(), t.ravel()], 1).astype(np.int32)


class Tuned:
    """Temporarily set library tuning knobs."""

    def __init__(self, **kv):
        self.kv = kv
        self.old = {}

    def __enter__(self):
        for k, v in self.kv.items():
            self.old[k] = binding.get_tuning(k)
            binding.set_tuning(k, v)

    def __exit__(self, *a):
        for k, v in self.old.items():
            binding.set_tuning(k, v)


FAMILIES = graphs.families()


@pytest.mark.parametrize("name,g", FAMILIES, ids=[f[0] for f in FAMILIES])
@pytest.mark.parametrize("t_bp", [0, 2, 64])
def test_small_families(name, g, t_bp):
    _require_gpu()
    order = gen.degree_order(g)
    ox = oracle.build(g.row_ptr, g.col, order, t_bp)
    gx = binding.build(g.row_ptr, g.col, order, t_bp, validate=True)
    assert_same_index(gx, ox, name)
    if g.n:
        p = all_pairs(g.n)
        want = oracle.query(ox, p)
        assert np.array_equal(gx.query(p), want)
        assert np.array_equal(gx.query(p, plain=True), want)


@pytest.mark.parametrize("root_sort", [0, 1])
@pytest.mark.parametrize("name,g", FAMILIES[::2], ids=[f[0] for f in FAMILIES[::2]])
def test_prune_test_paths(name, g, root_sort):
    # both prune-test kernels, straight from the frontier (0) and grouped by
    # root with the root's data in LDS (1), at every group size, give the
    # oracle's labels
    _require_gpu()
    order = gen.degree_order(g)
    for t_bp in (0, 5):
        ox = oracle.build(g.row_ptr, g.col, order, t_bp)
        for group in (4, 16, 64):
            with Tuned(root_sort=root_sort, group=group, window=7, window_work=0):
                gx = binding.build(g.row_ptr, g.col, order, t_bp)
            assert_same_index(gx, ox, f"{name} t_bp={t_bp} sort={root_sort} group={group}")


def test_root_grouped_tests_with_long_root_labels():
    # roots whose labels do not fit the LDS table (more than 1024 entries)
    # are tested through the window's global table: under a Random order
    # (Section 4.4) R-MAT 12 gives 164 vertices labels of 1025-1386 entries
    _require_gpu()
    g = gen.rmat_graph(12, seed=3)
    order = gen.random_order(g.n, 1)
    ox = oracle.build(g.row_ptr, g.col, order, 0)
    assert int(np.diff(ox.off).max()) > 1024
    with Tuned(root_sort=1):
        assert_same_index(binding.build(g.row_ptr, g.col, order, 0), ox, "long root labels")


@pytest.mark.parametrize("window,group,xgroup,work", [
    (1, 16, 16, 0), (3, 4, 4, 0), (17, 8, 64, 0), (64, 64, 8, 0), (1024, 32, 16, 0),
    (16384, 4, 16, 300), (4096, 4, 32, 5000), (700, 8, 4, 0)])
def test_windows_and_groups(window, group, xgroup, work):
    # concurrent roots + cleaning must give the sequential labels exactly,
    # for fixed windows (work 0) and windows resized after every window
    _require_gpu()
    g = gen.ba_graph(700, 3, 31)
    order = gen.degree_order(g)
    ox = oracle.build(g.row_ptr, g.col, order, 4)
    with Tuned(window=window, group=group, xgroup=xgroup, window_work=work, chunk=64):
        gx = binding.build(g.row_ptr, g.col, order, 4)
    assert_same_index(gx, ox, f"w{window} g{group} x{xgroup} work{work}")


@pytest.mark.parametrize("knobs", [dict(list_cap=1, window=256, window_work=0),
                                   dict(list_cap=1, window=16384, window_work=100000),
                                   dict(table_cap=8, window=64, window_work=0)],
                         ids=["lists-fixed", "lists-adaptive", "tables"])
def test_overflow_retries(knobs):
    # lists and root tables far too small: windows overflow and are re-run
    # (fewer roots, or a grown table area) and the labels stay exact
    _require_gpu()
    g = gen.ba_graph(900, 3, 77)
    order = gen.degree_order(g)
    ox = oracle.build(g.row_ptr, g.col, order, 2)
    with Tuned(**knobs):
        gx = binding.build(g.row_ptr, g.col, order, 2)
    assert_same_index(gx, ox, str(knobs))
    if "list_cap" in knobs:
        assert gx.stats()["retries"] > 0


def test_torch_allocator_hook():
    # builds through torch's caching allocator: same index, memory visible
    # to torch while the index lives and handed back by pll_free
    import torch

    _require_gpu()
    g, order, t_bp, pairs = gen.config_graph("ba2000")
    ox = oracle.build(g.row_ptr, g.col, order, t_bp)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    binding.use_torch_allocator(True)
    try:
        gx = binding.build(g.row_ptr, g.col, order, t_bp)
        held = torch.cuda.memory_allocated() - base
        assert held >= gx.stats()["index_bytes"] > 0
        assert_same_index(gx, ox, "torch allocator")
        assert np.array_equal(gx.query(pairs), oracle.query(ox, pairs))
        gx.close()
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == base
    finally:
        binding.use_torch_allocator(False)


def test_level_trace():
    # the per-level profile accounts for every visit and candidate
    _require_gpu()
    g, order, t_bp, _ = gen.config_graph("ba2000")
    with Tuned(profile=0):
        gx = binding.build(g.row_ptr, g.col, order, t_bp)
    assert gx.level_trace().shape == (0, 7)
    with Tuned(profile=1, window_work=2000):
        gx = binding.build(g.row_ptr, g.col, order, t_bp)
    tr, st = gx.level_trace(), gx.stats()
    assert tr.shape[1] == len(binding.Index.TRACE_COLS) and len(tr) == st["level_launches"]
    assert tr[:, 4].sum() == st["visited"] and tr[:, 5].sum() == st["candidates"]
    assert len(np.unique(tr[:, 0])) == st["windows"] and np.all(tr[:, 6] >= 0)
    for wi in np.unique(tr[:, 0]):
        rows = tr[tr[:, 0] == wi]
        assert np.array_equal(rows[:, 3], np.arange(len(rows)))  # levels 0, 1, ...
        assert len(np.unique(rows[:, 1])) == 1 and len(np.unique(rows[:, 2])) == 1
    firsts = tr[tr[:, 3] == 0][:, 1:3]
    assert firsts[0, 0] == 0 and np.array_equal(firsts[1:, 0], firsts[:-1].sum(1))
    assert firsts[-1].sum() == g.n


def test_random_order_and_plain_build():
    _require_gpu()
    g = graphs.erdos_renyi(150, 0.04, 8)
    order = gen.random_order(g.n, 5)
    ox = oracle.build(g.row_ptr, g.col, order, 3)
    assert_same_index(binding.build(g.row_ptr, g.col, order, 3, plain=True), ox, "plain")
    assert_same_index(binding.build(g.row_ptr, g.col, order, 3), ox, "windowed")


def test_ba2000_workload():
    # the small named workload: BA n=2000, m=4, t_bp=16, 1e5 pairs
    _require_gpu()
    g, order, t_bp, pairs = gen.config_graph("ba2000")
    ox = oracle.build(g.row_ptr, g.col, order, t_bp)
    gx = binding.build(g.row_ptr, g.col, order, t_bp)
    assert_same_index(gx, ox, "ba2000")
    want = oracle.query(ox, pairs)
    assert np.array_equal(gx.query(pairs), want)
    assert np.array_equal(gx.query(pairs, plain=True), want)
    st = gx.stats()
    assert st["entries"] == ox.counters["entries"]
    assert st["roots"] == ox.counters["roots"]


def test_device_pointer_queries():
    import torch
    _require_gpu()
    g, order, t_bp, pairs = gen.config_graph("ba2000")
    ox = oracle.build(g.row_ptr, g.col, order, t_bp)
    gx = binding.build(g.row_ptr, g.col, order, t_bp)
    dp = torch.from_numpy(pairs).cuda()
    out = torch.empty(len(pairs), dtype=torch.uint8, device="cuda")
    gx.query_device(dp, out, sync=True)
    assert np.array_equal(out.cpu().numpy(), oracle.query(ox, pairs))
    out2 = torch.empty_like(out)
    gx.query_device(dp, out2, plain=True)
    gx.sync()
    assert torch.equal(out, out2)
    # an out-of-range id: nothing written, error reported
    bad = dp.clone()
    bad[5, 1] = g.n
    out3 = torch.full_like(out, 7)
    with pytest.raises(binding.PllError):
        gx.query_device(bad, out3, sync=True)
    assert int((out3 != 7).sum()) == 0
    gx.query_device(bad, out3)
    with pytest.raises(binding.PllError):
        gx.sync()
    gx.sync()  # cleared


def test_range_error_and_clamped_answers():
    _require_gpu()
    g = graphs.path(256)
    order = gen.degree_order(g)
    gx = binding.build(g.row_ptr, g.col, order, 1)
    ox = oracle.build(g.row_ptr, g.col, order, 1)
    assert_same_index(gx, ox, "path256")
    q = np.array([[1, 255], [0, 255], [0, 254]], np.int32)
    assert gx.query(q).tolist() == [254, 255, 254]
    g2 = graphs.path(257)
    for t in (0, 1):
        with pytest.raises(binding.PllError) as e:
            binding.build(g2.row_ptr, g2.col, gen.degree_order(g2), t)
        assert e.value.code == binding.E_RANGE


def test_deterministic_rebuild():
    _require_gpu()
    g = gen.rmat_graph(12, seed=4)
    order = gen.degree_order(g)
    a = binding.build(g.row_ptr, g.col, order, 8).export()
    b = binding.build(g.row_ptr, g.col, order, 8).export()
    for k in a:
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.slow
def test_rmat14_and_tiny_windows():
    _require_gpu()
    g = gen.rmat_graph(14, seed=7)
    order = gen.degree_order(g)
    ox = oracle.build(g.row_ptr, g.col, order, 16)
    assert_same_index(binding.build(g.row_ptr, g.col, order, 16), ox, "rmat14")
    with Tuned(window=5, chunk=64, group=4):
        assert_same_index(binding.build(g.row_ptr, g.col, order, 16), ox, "rmat14 w5")
    p = gen.random_pairs(g.n, 200_000, 9)
    assert np.array_equal(binding.build(g.row_ptr, g.col, order, 16).query(p), oracle.query(ox, p))


def test_rmat18_benchmark_workload():
    # the benchmark's workload itself: R-MAT 18, t_bp = 50, 1e6 pairs, built
    # from device pointers in the launch configuration bench.py times
    import torch
    _require_gpu()
    g, order, t_bp, pairs = gen.config_graph("rmat18")
    ox = oracle.build(g.row_ptr, g.col, order, t_bp)
    d = [torch.from_numpy(a).cuda() for a in (g.row_ptr, g.col, order)]
    gx = binding.build_device(*d, t_bp)
    assert_same_index(gx, ox, "rmat18")
    dp = torch.from_numpy(pairs).cuda()
    out = torch.empty(len(pairs), dtype=torch.uint8, device="cuda")
    gx.query_device(dp, out, sync=True)
    assert np.array_equal(out.cpu().numpy(), oracle.query(ox, pairs))


def test_query_autotune():
    # the autotuner picks one of the group sizes and answers do not change
    import torch
    _require_gpu()
    g, order, t_bp, pairs = gen.config_graph("ba2000")
    ox = oracle.build(g.row_ptr, g.col, order, t_bp)
    gx = binding.build(g.row_ptr, g.col, order, t_bp)
    want = oracle.query(ox, pairs)
    with Tuned(qgroup=64):
        best = gx.autotune_query(pairs[:20000])
        assert best in (16, 32, 64) and binding.get_tuning("qgroup") == best
        assert np.array_equal(gx.query(pairs), want)
        best2 = gx.autotune_query(torch.from_numpy(pairs[:20000]).cuda())
        assert best2 in (16, 32, 64)
        assert np.array_equal(gx.query(pairs), want)
        bad = pairs[:10].copy()
        bad[2, 1] = g.n
        with pytest.raises(binding.PllError):
            gx.autotune_query(bad)
        with pytest.raises(binding.PllError):
            gx.autotune_query(torch.from_numpy(bad).cuda())


def test_block_cache_across_streams():
    # freed build memory is reused by later builds, also on other streams
    # (event-ordered); with the cache off every block is freed; results equal
    import torch
    _require_gpu()
    g, order, t_bp, pairs = gen.config_graph("ba2000")
    ox = oracle.build(g.row_ptr, g.col, order, t_bp)
    want = oracle.query(ox, pairs)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    dev = torch.device("cuda:0")
    d = [torch.from_numpy(a).to(dev) for a in (g.row_ptr, g.col, order)]
    dp = torch.from_numpy(pairs).to(dev)
    torch.cuda.synchronize()
    for keep in (16384, 0, 16384):
        with Tuned(pool_keep_mb=keep):
            for s in (s1, s2, s1):
                with torch.cuda.stream(s):
                    gx = binding.build_device(*d, t_bp, stream=s)
                    out = torch.empty(len(pairs), dtype=torch.uint8, device=dev)
                    gx.query_device(dp, out, stream=s, sync=True)
                assert np.array_equal(out.cpu().numpy(), want), (keep, s)
                assert_same_index(gx, ox, f"keep={keep}")
                gx.close()


@pytest.mark.parametrize("landmarks", [0, 1])
@pytest.mark.parametrize("name,order_fn", [("degree", gen.degree_order),
                                           ("random", lambda g: gen.random_order(g.n, 3))])
def test_landmark_rows_without_bit_parallel(landmarks, name, order_fn):
    # t_bp = 0: the first window's 16 exact BFS rows prune expansions; the
    # labels must be the oracle's either way
    _require_gpu()
    g = gen.rmat_graph(11 if name == "random" else 13, seed=9)
    order = order_fn(g)
    ox = oracle.build(g.row_ptr, g.col, order, 0)
    with Tuned(landmarks=landmarks, window_work=200000):
        gx = binding.build(g.row_ptr, g.col, order, 0)
    assert_same_index(gx, ox, f"{name} landmarks={landmarks}")
    if not landmarks:
        assert gx.stats()["bp_direct"] == 0
    elif name == "degree":
        assert gx.stats()["bp_direct"] > 0


def test_adaptive_test_group_on_long_labels():
    # t_bp = 0 under a random order gives labels long enough (hundreds of
    # entries) that the per-window choice of lanes per prune test moves
    # past 4; labels stay the oracle's
    _require_gpu()
    g = gen.rmat_graph(11, seed=6)
    order = gen.random_order(g.n, 5)
    ox = oracle.build(g.row_ptr, g.col, order, 0)
    with Tuned(group=0, window_work=100000, landmarks=0):
        gx = binding.build(g.row_ptr, g.col, order, 0)
    st = gx.stats()
    assert st["windows"] > 4 and st["label_scanned"] > 32 * st["normal_tests"]
    assert_same_index(gx, ox, "adaptive group")


@pytest.mark.parametrize("t_bp", [0, 16])
def test_earlier_roots_skipped_at_expansion(t_bp):
    # neighbours ranked before the window are left unvisited (their labels
    # already answer exactly); later windows see many such edges, and the
    # labels stay the oracle's
    _require_gpu()
    g = gen.rmat_graph(12, seed=8)
    order = gen.degree_order(g)
    ox = oracle.build(g.row_ptr, g.col, order, t_bp)
    with Tuned(window_work=50000):
        gx = binding.build(g.row_ptr, g.col, order, t_bp)
    st = gx.stats()
    assert st["windows"] > 3 and st["earlier_root"] > 0
    assert_same_index(gx, ox, f"t_bp={t_bp}")
    gx.close()


@pytest.mark.parametrize("t_bp", [17, 32, 50, 64])
def test_packed_distance_rows(t_bp):
    # the expansion's distance-row prune reads 4-bit copies of the rows
    # (tpad 32 or 64) or the 8-bit rows (knob off, or tpad 48): the same
    # labels either way (a saturated 4-bit distance prunes nothing, so a
    # neighbour the 4-bit row cannot rule out is left to the tests)
    _require_gpu()
    g = gen.rmat_graph(13, seed=12)
    order = gen.degree_order(g)
    ox = oracle.build(g.row_ptr, g.col, order, t_bp)
    st = {}
    for packed in (1, 0):
        with Tuned(packed_rows=packed):
            gx = binding.build(g.row_ptr, g.col, order, t_bp)
        assert_same_index(gx, ox, f"t_bp={t_bp} packed={packed}")
        st[packed] = gx.stats()
        gx.close()
    assert st[1]["bp_direct"] > 0 and st[0]["bp_direct"] > 0  # both forms prune by rows


@pytest.mark.parametrize("live", [0, 1])
@pytest.mark.parametrize("t_bp", [0, 32])
def test_live_adjacency(live, t_bp):
    # the expansion's adjacency is rebuilt without earlier-ranked neighbours
    # as the windows advance (knob 1) or kept whole (0): same labels, and
    # the compacted runs expand fewer entries
    _require_gpu()
    g = gen.rmat_graph(13, seed=11)
    order = gen.degree_order(g)
    ox = oracle.build(g.row_ptr, g.col, order, t_bp)
    # fixed windows of 1024 roots: rebuilt at s = 1024, 2048, 4096
    with Tuned(live_adjacency=live, window=1024, window_work=0):
        gx = binding.build(g.row_ptr, g.col, order, t_bp)
    assert_same_index(gx, ox, f"t_bp={t_bp} live={live}")
    st = gx.stats()
    gx.close()
    with Tuned(live_adjacency=1 - live, window=1024, window_work=0):
        gy = binding.build(g.row_ptr, g.col, order, t_bp)
    sy = gy.stats()
    gy.close()
    assert st["windows"] == sy["windows"] and st["windows"] > 4 and g.n > 4096
    on, off = (st, sy) if live else (sy, st)
    assert on["edges"] + on["task_edges"] < off["edges"] + off["task_edges"]


@pytest.mark.parametrize("t_bp", [0, 1])
def test_level_255_reached_but_pruned(t_bp):
    # Section 4.5.1's 8-bit distances: the BFS from a_0 reaches w at 255 and
    # must prune it there.  With the default windows x and a_0 share the first
    # window, where a_0 cannot yet prune with x's labels: the window's test at
    # 255 flags a range error and the window is run again with fewer roots
    # until a_0 runs after x is committed.  The plain form runs one root at a
    # time from the start.
    _require_gpu()
    g, order = graphs.level_255_pruned()
    ox = oracle.build(g.row_ptr, g.col, order, t_bp)
    assert ox.counters["max_dist"] == 254
    p = all_pairs(g.n)
    want = oracle.query(ox, p)
    for tag, kw, knobs in (("windows", {}, {}), ("plain", {"plain": True}, {}),
                           ("window 2", {}, {"window": 2, "window_work": 0})):
        with Tuned(**knobs):
            gx = binding.build(g.row_ptr, g.col, order, t_bp, **kw)
        assert_same_index(gx, ox, f"level255 t_bp={t_bp} {tag}")
        assert np.array_equal(gx.query(p), want), tag
        if tag == "windows" and t_bp == 0:
            assert gx.stats()["retries"] > 0  # the range flag re-ran the window


P9_CASES = [("ba2000", gen.ba_graph(2000, 4, 1), 16), ("rmat11", gen.rmat_graph(11, seed=5), 8),
            ("rmat11t0", gen.rmat_graph(11, seed=5), 0), ("grid", graphs.grid(9, 11), 2),
            ("union", graphs.disjoint_union(graphs.cycle(7), graphs.star(9), graphs.empty(2)), 1)]


@pytest.mark.parametrize("name,g,t_bp", P9_CASES, ids=[c[0] for c in P9_CASES])
def test_plain_counters_equal_the_oracle(name, g, t_bp):
    # Work counters are canonical (the visited set of root k is {v_k} plus the
    # neighbours of what k labels), so the plain GPU form, with the
    # expansion-time shortcuts off, does exactly the sequential algorithm's
    # work.  Offsets: the GPU labels a root at distance 0 without its test
    # (the oracle tests it and always keeps it), so its normal tests and
    # scanned entries lack one test and |L(v_k)| entries per root.
    _require_gpu()
    order = gen.degree_order(g)
    ox = oracle.build(g.row_ptr, g.col, order, t_bp)
    c = ox.counters
    with Tuned(expand_prune=0):
        gx = binding.build(g.row_ptr, g.col, order, t_bp, plain=True)
    assert_same_index(gx, ox, name)
    s = gx.stats()
    assert s["roots"] == c["roots"]
    assert s["visited"] == c["visited"]
    assert s["candidates"] == c["labeled"] == c["entries"]
    assert s["edges"] + s["task_edges"] == c["edges"]
    assert s["normal_tests"] + c["roots"] == c["normal_tests"]
    assert s["label_scanned"] + c["root_staged"] == c["label_scanned"]
    assert s["earlier_root"] == 0 and s["bp_direct"] == 0
    # the same knob on the windowed form changes the work, not the labels
    with Tuned(expand_prune=0):
        assert_same_index(binding.build(g.row_ptr, g.col, order, t_bp), ox, name + " windows")
