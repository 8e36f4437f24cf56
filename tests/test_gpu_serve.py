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


def test_serve_bench_runs():
    import torch
    assert torch.cuda.is_available()
    g, order, t_bp, _ = gen.config_graph("ba2000")
    gx = binding.build(g.row_ptr, g.col, order, t_bp)
    sat = binding.serve_bench(gx, 0.0, 3000, max_batch=4096, seed=7)
    assert sat["pairs_per_s"] > 0 and sat["launches"] >= 1
    low = binding.serve_bench(gx, sat["requests_per_s"] * 0.25, 3000, max_batch=4096, seed=8)
    assert low["p50_us"] > 0 and low["p99_us"] >= low["p50_us"]
