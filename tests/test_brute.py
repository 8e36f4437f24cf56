"""The brute-force helpers agree with each other (CPU only)."""
import numpy as np

import brute
import graphs
import oracle
import pins
from paper_1304_4661_amd import gen


def test_canonical_label_one_matches_the_all_vertex_form():
    for g, t in ((gen.ba_graph(300, 3, 9), 4), (graphs.grid(6, 7), 1),
                 (graphs.disjoint_union(graphs.cycle(6), graphs.star(5)), 0)):
        order = gen.degree_order(g)
        ix = oracle.build(g.row_ptr, g.col, order, t)
        used = pins.bp_used_ranks(ix)
        want = brute.canonical_labels(g.row_ptr, g.col, order, used)
        rank = np.empty(g.n, np.int64)
        rank[order] = np.arange(g.n)
        bp = np.zeros(g.n, bool)
        bp[order[used]] = True
        for u in range(g.n):
            assert brute.canonical_label_one(g.row_ptr, g.col, rank, bp, u) == want[rank[u]]
