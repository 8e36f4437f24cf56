"""pll_query_noalloc (through the C ABI) answers exactly as pll_query, on two
calls in a row with the second one smaller, for host and device pointers,
with its staging and error flag in the library's static device array."""
import numpy as np
import pytest

from paper_1304_4661_amd import binding, gen

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.fixture(scope="module")
def indexes():
    _gpu()
    out = []
    for g, t in ((gen.ba_graph(2000, 4, 1), 16), (gen.rmat_graph(12, seed=4), 8)):
        order = gen.degree_order(g)
        out.append((g, binding.build(g.row_ptr, g.col, order, t)))
    yield out
    for _, ix in out:
        ix.close()


def test_host_pointers_two_calls_second_smaller(indexes):
    for k, (g, ix) in enumerate(indexes):
        for plain in (False, True):
            big = gen.random_pairs(g.n, 60_000, 10 + k)
            small = gen.random_pairs(g.n, 777, 20 + k)
            a = ix.query_noalloc(big, plain=plain)
            b = ix.query_noalloc(small, plain=plain)
            assert np.array_equal(a, ix.query(big, plain=plain))
            assert np.array_equal(b, ix.query(small, plain=plain))


def test_device_pointers_two_calls_second_smaller(indexes):
    torch = _gpu()
    for k, (g, ix) in enumerate(indexes):
        for q in (200_000, 1_001):
            p = torch.from_numpy(gen.random_pairs(g.n, q, 30 + q + k)).cuda()
            want = torch.full((q,), 7, dtype=torch.uint8, device="cuda")
            got = torch.full((q,), 7, dtype=torch.uint8, device="cuda")
            ix.query_device(p, want, sync=True)
            ix.query_noalloc(p, got, sync=True)
            assert torch.equal(got, want)
            # asynchronous form, then the index's sticky error stays clear
            got2 = torch.zeros_like(got)
            ix.query_noalloc(p, got2, sync=False)
            ix.sync()
            assert torch.equal(got2, want)


def test_alternating_indexes_reuse_the_array(indexes):
    # the array keeps the last call's contents: answers never leak between
    # calls on different indexes
    (g1, a), (g2, b) = indexes
    p1 = gen.random_pairs(g1.n, 5000, 41)
    p2 = gen.random_pairs(min(g1.n, g2.n), 300, 42)
    for _ in range(3):
        assert np.array_equal(a.query_noalloc(p1), a.query(p1))
        assert np.array_equal(b.query_noalloc(p2), b.query(p2))


def test_errors_and_limits(indexes):
    torch = _gpu()
    g, ix = indexes[0]
    mx = binding.noalloc_max_pairs()
    assert mx == 1 << 21
    with pytest.raises(binding.PllError) as e:
        ix.query_noalloc(np.zeros((mx + 1, 2), np.int32))
    assert e.value.code == binding.E_INVAL
    ix.query_noalloc(np.zeros((mx, 2), np.int32))  # the limit itself fits
    bad = np.array([[0, 1], [g.n, 0]], np.int32)
    with pytest.raises(binding.PllError):
        ix.query_noalloc(bad)
    # device pointers: an out-of-range id writes nothing; the next valid call
    # starts from a cleared flag
    dbad = torch.from_numpy(bad).cuda()
    out = torch.full((2,), 9, dtype=torch.uint8, device="cuda")
    with pytest.raises(binding.PllError):
        ix.query_noalloc(dbad, out, sync=True)
    assert int((out != 9).sum()) == 0
    ok = torch.from_numpy(gen.random_pairs(g.n, 64, 43)).cuda()
    o2 = torch.zeros(64, dtype=torch.uint8, device="cuda")
    ix.query_noalloc(ok, o2, sync=True)
    assert np.array_equal(o2.cpu().numpy(), ix.query(ok.cpu().numpy()))
    # asynchronous error goes to the index's sticky error, reported once
    ix.query_noalloc(dbad, out, sync=False)
    with pytest.raises(binding.PllError):
        ix.sync()
    ix.sync()
    assert ix.query_noalloc(np.zeros((0, 2), np.int32)).size == 0
