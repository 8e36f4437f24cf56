"""Serving: continuous batching must not change any answer.  Each request's
answers in a busy mix equal the same pairs answered alone (and the oracle)."""
import threading

import numpy as np
import pytest

import oracle
from paper_1304_4661_amd import binding, gen

pytestmark = pytest.mark.gpu


def test_alone_vs_mix():
    import torch
    assert torch.cuda.is_available()
    g, order, t_bp, _ = gen.config_graph("ba2000")
    gx = binding.build(g.row_ptr, g.col, order, t_bp)
    ox = oracle.build(g.row_ptr, g.col, order, t_bp)
    rng = np.random.Generator(np.random.PCG64(42))
    reqs = []
    for _ in range(600):
        q = int(np.exp(rng.uniform(0, np.log(3000))))
        reqs.append(rng.integers(0, g.n, (q, 2)).astype(np.int32))
    # small slots so that batches mix requests and several are in flight
    srv = binding.Server(gx, nslots=3, slot_pairs=4096)
    tickets = [None] * len(reqs)

    def worker(k0):
        for k in range(k0, len(reqs), 4):
            tickets[k] = srv.submit(reqs[k])

    th = [threading.Thread(target=worker, args=(i,)) for i in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    lat = []
    for k, p in enumerate(reqs):
        ans, us = srv.result(tickets[k])
        lat.append(us)
        alone = gx.query(p)
        assert np.array_equal(ans, alone), f"request {k} differs from its answer alone"
        assert np.array_equal(ans, oracle.query(ox, p)), f"request {k} differs from the oracle"
    st = srv.stop()
    assert st["pairs"] == sum(len(p) for p in reqs)
    assert st["launches"] < len(reqs)  # requests were coalesced
    assert min(lat) > 0


def test_request_larger_than_a_slot():
    # a request of more pairs than a slot holds is served in slot-sized
    # parts; its answers equal the same pairs answered alone, also when
    # other requests queue around it
    import torch
    assert torch.cuda.is_available()
    g, order, t_bp, _ = gen.config_graph("ba2000")
    gx = binding.build(g.row_ptr, g.col, order, t_bp)
    rng = np.random.Generator(np.random.PCG64(44))
    big = rng.integers(0, g.n, (10_000, 2)).astype(np.int32)
    small = [rng.integers(0, g.n, (q, 2)).astype(np.int32) for q in (5, 700, 1024, 1)]
    srv = binding.Server(gx, nslots=2, slot_pairs=1024)
    tickets = [srv.submit(small[0]), srv.submit(big)] + [srv.submit(p) for p in small[1:]]
    for t, p in zip(tickets, [small[0], big] + small[1:]):
        ans, us = srv.result(t)
        assert us > 0 and np.array_equal(ans, gx.query(p))
    st = srv.stop()
    assert st["pairs"] == len(big) + sum(len(p) for p in small)
    assert st["launches"] >= 10  # the big request took at least 10 slot loads


def test_request_records_are_recycled():
    # a server keeps no record of answered requests: 3000 requests in turn
    # use a handful of records, and an answered ticket is no longer valid
    import torch
    assert torch.cuda.is_available()
    g, order, t_bp, _ = gen.config_graph("ba2000")
    gx = binding.build(g.row_ptr, g.col, order, t_bp)
    rng = np.random.Generator(np.random.PCG64(45))
    srv = binding.Server(gx, nslots=2, slot_pairs=256)
    last = None
    for k in range(3000):
        p = rng.integers(0, g.n, (1 + k % 600, 2)).astype(np.int32)  # some split in parts
        t = srv.submit(p)
        ans, _ = srv.result(t)
        assert np.array_equal(ans, gx.query(p))
        last = t
    with pytest.raises(binding.PllError):
        srv.result(last)
    st = srv.stop()
    assert st["records"] <= 8, st


def test_serve_bench_runs():
    import torch
    assert torch.cuda.is_available()
    g, order, t_bp, _ = gen.config_graph("ba2000")
    gx = binding.build(g.row_ptr, g.col, order, t_bp)
    sat = binding.serve_bench(gx, 0.0, 3000, max_batch=4096, seed=7)
    assert sat["pairs_per_s"] > 0 and sat["launches"] >= 1
    # the longest launch (its number and time) and the worker's longest pause
    assert 0 <= sat["max_launch_at"] < sat["launches"] and sat["max_launch_us"] > 0
    assert sat["max_worker_pause_us"] >= 0
    low = binding.serve_bench(gx, sat["requests_per_s"] * 0.25, 3000, max_batch=4096, seed=8)
    assert low["p50_us"] > 0 and low["p99_us"] >= low["p50_us"]


@pytest.mark.parametrize("name", ["ba2000w", "digraph"])
def test_weighted_alone_vs_mix(name):
    # a server of a weighted index answers with 32-bit distances, each
    # request the same in a busy mix as alone and as the oracle
    import ctypes as C

    import torch
    assert torch.cuda.is_available()
    directed = name == "digraph"
    if directed:
        g = gen.uniform_weights(gen.rmat_digraph(10, 8, seed=5), 1, 50, 6)
        order = gen.degree_order_directed(g)
    else:
        g, order, _, _ = gen.config_graph(name)
    gx = binding.build_weighted(g.row_ptr, g.col, g.w, order, directed=directed)
    ox = oracle.build_weighted(g.row_ptr, g.col, g.w, order, directed=directed)
    rng = np.random.Generator(np.random.PCG64(43))
    reqs = [rng.integers(0, g.n, (int(np.exp(rng.uniform(0, np.log(2000)))), 2)).astype(np.int32)
            for _ in range(200)]
    srv = binding.Server(gx, nslots=3, slot_pairs=2048)
    tickets = [srv.submit(p) for p in reqs]
    for k, p in enumerate(reqs):
        ans, us = srv.result(tickets[k])
        assert ans.dtype == np.uint32 and us > 0
        assert np.array_equal(ans, gx.query_weighted(p)), f"request {k} differs from alone"
        assert np.array_equal(ans, oracle.query_weighted(ox, p)), f"request {k} differs from oracle"
    # the 8-bit submission refuses a weighted server, the 32-bit one an
    # unweighted server
    lib = binding.library()
    one = np.zeros(2, np.int32)
    o8 = np.zeros(1, np.uint8)
    t = C.c_int64()
    assert lib.pll_server_submit(srv._h, one.ctypes.data, 1, o8.ctypes.data,
                                 C.byref(t)) == binding.E_UNSUPPORTED
    st = srv.stop()
    assert st["pairs"] == sum(len(p) for p in reqs)
    gb = gen.ba_graph(300, 3, 1)
    gu = binding.build(gb.row_ptr, gb.col, gen.degree_order(gb), 4)
    su = binding.Server(gu, nslots=1, slot_pairs=16)
    o32 = np.zeros(1, np.uint32)
    assert lib.pll_server_submit_weighted(su._h, one.ctypes.data, 1, o32.ctypes.data,
                                          C.byref(t)) == binding.E_UNSUPPORTED
    su.stop()


def test_weighted_serve_bench_runs():
    import torch
    assert torch.cuda.is_available()
    g, order, _, _ = gen.config_graph("ba2000w")
    gx = binding.build_weighted(g.row_ptr, g.col, g.w, order)
    sat = binding.serve_bench(gx, 0.0, 2000, max_batch=4096, seed=9)
    assert sat["pairs_per_s"] > 0 and sat["launches"] >= 1
