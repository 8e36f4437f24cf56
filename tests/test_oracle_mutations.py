"""Plant plausible mistakes in a copy of the oracle and check the pins see them.

Each mutation edits the oracle's C source (a private copy compiled into a
temporary library; the real oracle is untouched) in a way a careless
implementation of the paper might, and the pin suite must report at least one
failure on a handful of small graphs.
"""
import pytest

import graphs
import oracle
import pins
from paper_1304_4661_amd import gen

MUTATIONS = [
    ("E1 before E0 (Algorithm 3 order)",
     "    for (int64_t i = 0; i < ne0; i++) s0[e0[2 * i + 1]] |= s1[e0[2 * i]];\n"
     "    for (int64_t i = 0; i < ne1; i++) {\n"
     "      s1[e1[2 * i + 1]] |= s1[e1[2 * i]];\n"
     "      s0[e1[2 * i + 1]] |= s0[e1[2 * i]];\n"
     "    }\n",
     "    for (int64_t i = 0; i < ne1; i++) {\n"
     "      s1[e1[2 * i + 1]] |= s1[e1[2 * i]];\n"
     "      s0[e1[2 * i + 1]] |= s0[e1[2 * i]];\n"
     "    }\n"
     "    for (int64_t i = 0; i < ne0; i++) s0[e0[2 * i + 1]] |= s1[e0[2 * i]];\n"),
    ("S^0 not carried along E1 edges",
     "      s0[e1[2 * i + 1]] |= s0[e1[2 * i]];\n", ""),
    ("bit-parallel query subtracts 1 instead of 2",
     "    td -= 2;\n", "    td -= 1;\n"),
    ("normal prune test strict",
     "  return best <= d;\n", "  return best < d;\n"),
    ("bit-parallel prune test strict",
     "m0u[i]) <= d) {", "m0u[i]) < d) {"),
    ("literal Algorithm 1 append: distance of the root",
     "rc = label_push(&x->lab[u], (uint32_t)k, (uint8_t)d, par);",
     "rc = label_push(&x->lab[u], (uint32_t)k, (uint8_t)0, par);"),
    ("literal Algorithm 1 expansion: neighbours of the root",
     "      for (int64_t j = off[u]; j < off[u + 1]; j++) {\n        int32_t w = adj[j];\n        x->cnt[C_EDGES]++;",
     "      for (int64_t j = off[k]; j < off[k + 1]; j++) {\n        int32_t w = adj[j];\n        x->cnt[C_EDGES]++;"),
    ("bit-parallel neighbours taken highest rank first",
     "for (int64_t j = off[r]; j < off[r + 1] && x->bp_nsel[i] < ORC_BPW; j++) {",
     "for (int64_t j = off[r + 1] - 1; j >= off[r] && x->bp_nsel[i] < ORC_BPW; j--) {"),
    ("merge join stops at the first common hub",
     "      if (v < best) best = v;\n      i++;\n      j++;\n",
     "      if (v < best) best = v;\n      break;\n"),
    ("T not reset after a root",
     "    for (int64_t i = 0; i < Lk->len; i++) T[Lk->hub[i]] = (uint8_t)ORC_INF;\n    x->root_visited",
     "    x->root_visited"),
    ("P not reset after a root",
     "    /* reset only what this BFS touched (Section 4.5.1, \"Initialization\") */\n    for (int64_t i = 0; i < qt; i++) P[queue[i]] = 0xFFFF;\n", ""),
    ("next level one too far",
     "        P[w] = (uint16_t)(d + 1);\n        queue[qt++] = w;\n      }\n    }\n    /* reset",
     "        P[w] = (uint16_t)(d + 2);\n        queue[qt++] = w;\n      }\n    }\n    /* reset"),
    ("S^0 left as the raw dynamic programme",
     "x->bp_0[(int64_t)v * t + slot] = s0[v] & ~s1[v];",
     "x->bp_0[(int64_t)v * t + slot] = s0[v];"),
    ("path parent recorded as the BFS root",
     "uint32_t par = d == 0 ? (uint32_t)k : tree_parent(x->lab, off, adj, u, k, d);",
     "uint32_t par = (uint32_t)k;"),
    ("path parent: the highest-ranked labeled neighbour",
     "L->dist[L->len - 1] == d - 1 &&\n        (uint32_t)padj[j] < best)",
     "L->dist[L->len - 1] == d - 1 &&\n        (best == ORC_SENTINEL || (uint32_t)padj[j] > best))"),
    ("path parent: any neighbour the BFS labeled, at any level",
     "if (L->len > 0 && L->hub[L->len - 1] == (uint32_t)k && L->dist[L->len - 1] == d - 1 &&",
     "if (L->len > 0 && L->hub[L->len - 1] == (uint32_t)k &&"),
    ("walk towards a neighbour follows S^0 instead of S^-1",
     "      c = bp_step(x, c, i, -1, bit, 1);\n", "      c = bp_step(x, c, i, -1, bit, 0);\n"),
    ("bit-parallel path ignores the -1/-2 witnesses",
     "      kind = (int)ds + (int)dt - v;\n", "      kind = 0;\n"),
    ("any BFS level reaching 255 is a range error",
     "      if (pruned_at(x, k, u, d, T)) continue;\n      if (d >= (int)ORC_INF) {",
     "      if (d < (int)ORC_INF && pruned_at(x, k, u, d, T)) continue;\n      if (d >= (int)ORC_INF) {"),
    ("pruned BFS also run from bit-parallel vertices",
     "    if (used[k]) continue;\n    x->cnt[C_ROOTS]++;", "    x->cnt[C_ROOTS]++;"),
]

CASES = [
    ("er30", graphs.erdos_renyi(30, 0.12, 3), 1),
    ("er60", graphs.erdos_renyi(60, 0.05, 4), 5),
    ("ba120", gen.ba_graph(120, 3, 12), 2),
    ("grid4x5", graphs.grid(4, 5), 1),
    ("union", graphs.disjoint_union(graphs.cycle(5), graphs.star(6), graphs.path(4)), 2),
    ("ba200", gen.ba_graph(200, 2, 5), 0),
    ("level255", graphs.level_255_pruned(), 0),
]


@pytest.mark.parametrize("desc,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(desc, old, new, tmp_path):
    src = oracle.source_text()
    assert src.count(old) == 1, f"mutation anchor not found once: {desc}"
    lib = oracle.load_variant(src.replace(old, new), str(tmp_path))
    caught = []
    for name, g, t in CASES:
        g, order = g if isinstance(g, tuple) else (g, gen.degree_order(g))
        try:
            f = pins.run_all(g, order, t, lib=lib)
        except oracle.OracleError as e:  # a crash-free error also counts
            f = [str(e)]
        if f:
            caught.append((name, f[0]))
    assert caught, f"no pin caught: {desc}"
