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
    _require_gpu()
    spec = gen.batch_spec(24, seed_base=500, n_lo=50, n_hi=1500)
    gs = [gen.ba_graph(n, m, s) for n, m, s in spec]
    _check_batch(gs, 16, seed=3)
    _check_batch(gs, 16, seed=4, window=7, group=8)


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
