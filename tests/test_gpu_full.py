"""GPU parity at full size: R-MAT 20, the 256-graph batch and R-MAT 22.

Each index is built as the benchmark builds it (inputs resident on the
device, default tuning) and compared with the oracle's index of the same
input through the SHA-256 digests that ``tests/golden/make_full_digests.py``
stored (whole arrays, and blocks of 16,384 ranks so that a mismatch names
its place), answers included.  Checks that need no oracle sit beside them:
BFS from sampled sources against every target (the corollary of Theorem
4.1: the index answers exact distances) and the min-key characterisation of
the labels of sampled vertices (the canonical-label lemma derived from the
proofs of Theorems 4.1 and 4.2)."""
import json
import os

import numpy as np
import pytest

import brute
import digest
from paper_1304_4661_amd import binding, gen

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name):
    path = os.path.join(GOLDEN, f"full_{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not written (tests/golden/make_full_digests.py {name})")
    with open(path) as f:
        return json.load(f)


def _device(*arrays):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrays]


def _answers(ix, d_pairs, plain=False):
    import torch
    out = torch.empty(d_pairs.shape[0], dtype=torch.uint8, device=d_pairs.device)
    ix.query_device(d_pairs, out, plain=plain, sync=True)
    return out.cpu().numpy()


def _index_digests(ix, graph=0):
    e = ix.export(graph)
    d = digest.index_digests(e["off"], e["hub"], e["dist"], e["bp_d"], e["bp_m1"], e["bp_0"])
    return d, e


def _bfs_sources(g, ix, order, sources):
    """Every target's distance from each source equals the query answer."""
    D = np.minimum(brute.apsp(g.row_ptr, g.col, sources=np.asarray(sources)), 255)
    for i, s in enumerate(sources):
        p = np.stack([np.full(g.n, s, np.int32), np.arange(g.n, dtype=np.int32)], 1)
        got = ix.query(p)
        bad = np.nonzero(got != D[i])[0]
        assert len(bad) == 0, f"source {s}: query != BFS at {bad[:5]}"


def _canonical_rows(g, e, order, bp_ranks, vertices):
    rank = np.empty(g.n, np.int64)
    rank[order] = np.arange(g.n)
    bp = np.zeros(g.n, bool)
    bp[np.asarray(order)[np.asarray(bp_ranks, np.int64)]] = True
    for u in vertices:
        want = brute.canonical_label_one(g.row_ptr, g.col, rank, bp, int(u))
        r = int(rank[u])
        a, b = int(e["off"][r]), int(e["off"][r + 1])
        got = dict(zip(e["hub"][a:b].tolist(), e["dist"][a:b].tolist()))
        assert got == want, f"vertex {u} (rank {r}): label differs from its characterisation"


def _bp_ranks(e):
    """Ranks used by the bit-parallel phase (Section 5.1 sets): a slot's root
    has distance 0 in it; a chosen neighbour w has distance 1 and holds itself
    in S^{-1}(w), which no other neighbour of the root holds anything in."""
    d, m1 = e["bp_d"], e["bp_m1"]
    if not d.size:
        return np.zeros(0, int)
    return np.nonzero(((d == 0) | ((d == 1) & (m1 != 0))).any(axis=1))[0]


def _single(name):
    gold = golden(name)
    g, order, t_bp, _ = gen.config_graph(name)
    assert gen.csr_sha256(g, order) == gold["csr_sha256"], "generator output changed"
    pairs = gen.random_pairs(g.n, gold["pairs"], gold["pair_seed"])
    d_row, d_col, d_order, d_pairs = _device(g.row_ptr, g.col, order, pairs)
    ix = binding.build_device(d_row, d_col, d_order, t_bp)
    got, e = _index_digests(ix)
    return {"gold": gold, "g": g, "order": order, "ix": ix, "digests": got, "export": e,
            "d_pairs": d_pairs, "pairs": pairs}


@pytest.fixture(scope="module")
def rmat20():
    w = _single("rmat20")
    yield w
    w["ix"].close()


@pytest.fixture(scope="module")
def rmat22():
    w = _single("rmat22")
    yield w
    w["ix"].close()


@pytest.mark.parametrize("name", ["rmat20", "rmat22"])
def test_full_index_equals_the_oracle(name, request):
    w = request.getfixturevalue(name)
    bad = digest.compare(w["digests"], w["gold"]["index"])
    assert not bad, f"{name}: " + "; ".join(bad)
    assert w["ix"].stats()["entries"] == w["gold"]["counters"]["entries"]


@pytest.mark.parametrize("name", ["rmat20", "rmat22"])
def test_full_answers_equal_the_oracle(name, request):
    # the workload's 1e7 pairs, batched (one launch) and plain
    w = request.getfixturevalue(name)
    want = w["gold"]["answers"]
    for plain in (False, True):
        a = _answers(w["ix"], w["d_pairs"], plain=plain)
        got = digest.answers_digest(a)
        assert got["sha256"] == want["sha256"], (plain, got["hist"], want["hist"])


@pytest.mark.parametrize("name,nsrc", [("rmat20", 16), ("rmat22", 6)])
def test_full_bfs_from_sampled_sources(name, nsrc, request):
    w = request.getfixturevalue(name)
    g, order = w["g"], w["order"]
    rng = np.random.Generator(np.random.PCG64(7))
    sources = [int(order[0]), int(order[-1])] + rng.integers(0, g.n, nsrc - 2).tolist()
    _bfs_sources(g, w["ix"], order, sources)


@pytest.mark.parametrize("name", ["rmat20", "rmat22"])
def test_full_labels_of_sampled_vertices(name, request):
    # top-ranked non-bit-parallel vertex, a bit-parallel vertex, random ones
    w = request.getfixturevalue(name)
    g, order, e = w["g"], w["order"], w["export"]
    used = _bp_ranks(e)
    free = np.setdiff1d(np.arange(min(g.n, 100_000)), used)
    rng = np.random.Generator(np.random.PCG64(8))
    ranks = [int(free[0]), int(used[0]) if len(used) else 0, g.n - 1] + \
        rng.integers(0, g.n, 2).tolist()
    _canonical_rows(g, e, order, used, [int(order[r]) for r in ranks])


def test_rmat22_serving_alone_vs_mix(rmat22):
    # continuous batching on the R-MAT 22 index: requests of log-uniform
    # size in [1, 4096] submitted together (mixed into shared launches) get
    # the answers they get alone
    ix, g = rmat22["ix"], rmat22["g"]
    rng = np.random.Generator(np.random.PCG64(105))
    reqs = [rng.integers(0, g.n, (int(np.exp(rng.uniform(0, np.log(4096)))), 2)).astype(np.int32)
            for _ in range(400)]
    srv = binding.Server(ix, nslots=4, slot_pairs=1 << 14)
    tickets = [srv.submit(p) for p in reqs]
    for k, p in enumerate(reqs):
        ans, _ = srv.result(tickets[k])
        assert np.array_equal(ans, ix.query(p)), f"request {k}"
    st = srv.stop()
    assert st["launches"] < len(reqs)


@pytest.fixture(scope="module")
def ba256():
    gold = golden("ba256")
    gs, vtx_off, row_ptr, col, order, t_bp, pairs = gen.batch_workload()
    d_row, d_col, d_order, d_pairs = _device(row_ptr, col, order, pairs)
    ix = binding.build_batch(vtx_off, d_row, d_col, d_order, t_bp, device=True)
    yield {"gold": gold, "gs": gs, "vtx_off": vtx_off, "ix": ix, "pairs": pairs,
           "d_pairs": d_pairs, "t_bp": t_bp}
    ix.close()


def test_ba256_every_graph_equals_its_oracle_build(ba256):
    gold, gs, ix = ba256["gold"], ba256["gs"], ba256["ix"]
    assert len(gold["graphs"]) == len(gs) == 256
    bad = []
    for i, g in enumerate(gs):
        rec = gold["graphs"][i]
        assert gen.csr_sha256(g, gen.degree_order(g)) == rec["csr_sha256"], i
        got, _ = _index_digests(ix, i)
        got.pop("blocks")
        diff = digest.compare(got, rec["index"])
        if diff:
            bad.append((i, diff[0]))
    assert not bad, f"{len(bad)} graphs differ, first {bad[:3]}"


def test_ba256_answers(ba256):
    # 1e4 pairs inside each graph (one launch for all 2.56e6), each graph's
    # answers equal its oracle's; pairs across graphs answer 255
    gold, ix, vtx_off = ba256["gold"], ba256["ix"], ba256["vtx_off"]
    a = _answers(ix, ba256["d_pairs"])
    per = len(a) // 256
    for i in range(256):
        got = digest.answers_digest(a[i * per:(i + 1) * per])
        assert got["sha256"] == gold["graphs"][i]["answers"]["sha256"], f"graph {i}"
    assert np.array_equal(_answers(ix, ba256["d_pairs"], plain=True), a)
    rng = np.random.Generator(np.random.PCG64(4))
    N = int(vtx_off[-1])
    p = rng.integers(0, N, (200_000, 2)).astype(np.int32)
    gof = np.searchsorted(vtx_off, p, side="right") - 1
    cross = gof[:, 0] != gof[:, 1]
    assert np.all(ix.query(p[cross]) == 255)


def test_ba256_build_and_query_in_one_call(ba256):
    # pll_build_query_batch on the full batch: the graphs built whole answer
    # their pairs inside the whole-graph launch, the rest after the build;
    # every graph's answers equal its oracle's
    gold, gs, vtx_off = ba256["gold"], ba256["gs"], ba256["vtx_off"]
    _, row_ptr, col, order = gen.pack_batch(gs)
    d_row, d_col, d_order = _device(row_ptr, col, order)
    per = len(ba256["pairs"]) // 256
    qoff = np.arange(257, dtype=np.int64) * per
    ix, out = binding.build_query_batch(vtx_off, d_row, d_col, d_order, ba256["t_bp"], qoff,
                                        ba256["d_pairs"], device=True)
    st = ix.stats()
    ix.close()
    whole = [i for i, g in enumerate(gs) if g.n <= binding.get_tuning("whole_n")]
    assert st["whole_graphs"] == len(whole) > 0 and st["whole_pairs"] == per * len(whole)
    a = out.cpu().numpy()
    for i in range(256):
        got = digest.answers_digest(a[i * per:(i + 1) * per])
        assert got["sha256"] == gold["graphs"][i]["answers"]["sha256"], f"graph {i}"
