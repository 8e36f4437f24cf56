"""Host-only checks of the C ABI: the library loads, exports every entry
point include/pll.h declares, and rejects bad arguments before touching a
device (so these run without a GPU)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import graphs
from paper_1304_4661_amd import binding, gen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", f)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(pll_[a-z_]+)\s*\(", txt))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = binding.library()
    decl = declared_symbols()
    assert "pll_build" in decl and "pll_query" in decl
    for name in decl:
        assert hasattr(lib, name), name
    assert set(binding.EXPORTED) <= set(decl)


def test_strerror_and_tuning():
    lib = binding.library()
    assert lib.pll_strerror(0) == b"ok"
    assert b"range" in lib.pll_strerror(-3) or b"8 bits" in lib.pll_strerror(-3)
    old = binding.get_tuning("window")
    binding.set_tuning("window", 64)
    assert binding.get_tuning("window") == 64
    binding.set_tuning("window", old)
    with pytest.raises(binding.PllError):
        binding.set_tuning("window", 0)
    with pytest.raises(binding.PllError):
        binding.set_tuning("group", 12)
    binding.set_tuning("group", 0)  # chosen per window
    assert binding.get_tuning("group") == 0
    with pytest.raises(binding.PllError):
        binding.set_tuning("nope", 1)
    for key, good, bad in [("xgroup", 32, 24), ("window_work", 0, -1), ("window_mem_mb", 64, 0),
                           ("list_cap", 100, -1), ("table_cap", 100, -1),
                           ("window", 16384, 16385), ("group", 64, 128),
                           ("wgroup", 8, 12), ("wwork", 0, -1),
                           ("live_adjacency", 0, 2), ("whole_n", 2048, 16385),
                           ("whole_pool", 1, 0), ("packed_rows", 0, 2)]:
        old = binding.get_tuning(key)
        binding.set_tuning(key, good)
        assert binding.get_tuning(key) == good
        with pytest.raises(binding.PllError):
            binding.set_tuning(key, bad)
        assert binding.get_tuning(key) == good
        binding.set_tuning(key, old)


def test_set_allocator_arguments():
    lib = binding.library()
    f = binding.FREE_FN(lambda p, s, c: None)
    assert lib.pll_set_allocator(None, C.cast(f, C.c_void_p), None) == binding.E_INVAL
    assert lib.pll_set_allocator(None, None, None) == binding.OK


def test_path_queries_reject_bad_arguments():
    lib = binding.library()
    lens = np.zeros(1, np.int32)
    pairs = np.zeros(2, np.int32)
    assert lib.pll_query_path(None, pairs.ctypes.data, 1, 4, None, lens.ctypes.data, 0,
                              None) == binding.E_INVAL
    assert lib.pll_export_parents(None, 0, lens.ctypes.data) == binding.E_INVAL


def test_level_trace_rejects_null():
    lib = binding.library()
    assert lib.pll_level_trace(None, None, 0) == binding.E_INVAL


def _rc_build(rp, col, order, t, flags=0):
    lib = binding.library()
    h = C.c_void_p()
    rp = np.ascontiguousarray(rp, np.int32)
    col = np.ascontiguousarray(col, np.int32)
    order = np.ascontiguousarray(order, np.int32)
    rc = lib.pll_build(len(order), rp.ctypes.data, col.ctypes.data if len(col) else None,
                       order.ctypes.data, t, flags, None, C.byref(h))
    return rc, h


def test_build_rejects_bad_input_before_device_work():
    g = graphs.cycle(6)
    order = gen.degree_order(g)
    bad_order = order.copy()
    bad_order[1] = bad_order[0]
    assert _rc_build(g.row_ptr, g.col, bad_order, 0)[0] == binding.E_INVAL
    col = g.col.copy()
    col[0] = 0  # self-loop
    assert _rc_build(g.row_ptr, col, order, 0)[0] == binding.E_INVAL
    col = g.col.copy()
    col[3] = 99
    assert _rc_build(g.row_ptr, col, order, 0)[0] == binding.E_INVAL
    rp = g.row_ptr.copy()
    rp[0] = 1
    assert _rc_build(rp, g.col, order, 0)[0] == binding.E_INVAL
    assert _rc_build(g.row_ptr, g.col, order, 65)[0] == binding.E_INVAL
    assert _rc_build(g.row_ptr, g.col, order, -1)[0] == binding.E_INVAL
    # asymmetric graph, only caught under PLL_VALIDATE
    rp = np.array([0, 1, 1], np.int32)
    col = np.array([1], np.int32)
    assert _rc_build(rp, col, np.array([0, 1], np.int32), 0, binding.VALIDATE)[0] == binding.E_INVAL
    rc, h = _rc_build(g.row_ptr, g.col, bad_order, 0)
    assert rc == binding.E_INVAL and h.value is None  # *out stays NULL on error


def test_query_rejects_null_index():
    lib = binding.library()
    pairs = np.zeros(2, np.int32)
    out = np.zeros(1, np.uint8)
    assert lib.pll_query(None, pairs.ctypes.data, 1, out.ctypes.data, 0, None) == binding.E_INVAL
    assert lib.pll_stats(None, 0, None, 0) == binding.E_INVAL
    lib.pll_free(None)


def test_build_batch_rejects_bad_input_before_device_work():
    lib = binding.library()
    g1, g2 = graphs.cycle(4), graphs.path(3)
    vtx_off, rp, col, order = gen.pack_batch([g1, g2])

    def rc(vo, rp_, col_, order_, t=0, G=None):
        h = C.c_void_p()
        vo = np.ascontiguousarray(vo, np.int64)
        rp_ = np.ascontiguousarray(rp_, np.int32)
        col_ = np.ascontiguousarray(col_, np.int32)
        order_ = np.ascontiguousarray(order_, np.int32)
        G = len(vo) - 1 if G is None else G
        r = lib.pll_build_batch(G, vo.ctypes.data, rp_.ctypes.data, col_.ctypes.data,
                                order_.ctypes.data, t, 0, None, C.byref(h))
        assert h.value is None or r == 0
        return r

    bad = col.copy()
    bad[0] = 5  # vertex 0 (graph 0) linked into graph 1
    assert rc(vtx_off, rp, bad, order) == binding.E_INVAL
    bo = order.copy()
    bo[4] = 3  # graph 1 has 3 vertices: local id 3 is out of range
    assert rc(vtx_off, rp, col, bo) == binding.E_INVAL
    assert rc(np.array([1, 4, 7]), rp, col, order) == binding.E_INVAL  # vtx_off[0] != 0
    assert rc(np.array([0, 5, 4]), rp, col, order) == binding.E_INVAL  # decreasing
    assert rc(vtx_off, rp, col, order, t=65) == binding.E_INVAL
    assert rc(vtx_off, rp, col, order, G=-1) == binding.E_INVAL


def test_server_rejects_bad_arguments_without_device_work():
    lib = binding.library()
    h = C.c_void_p()
    assert lib.pll_server_start(None, 2, 1024, C.byref(h)) == binding.E_INVAL
    assert h.value is None
    assert lib.pll_server_stop(None, None, 0) == binding.E_INVAL
    assert lib.pll_server_done(None, 0, 0, None) == binding.E_INVAL
    st = np.zeros(9)
    assert lib.pll_serve_bench(None, 1.0, 10, 16, 1, 2, 1024, st.ctypes.data, 9) == binding.E_INVAL


def test_weighted_entry_points_reject_bad_arguments():
    # all of these fail in host-side validation, before any device work
    lib = binding.library()
    g = gen.uniform_weights(graphs.cycle(6), 1, 9, 1)
    order = gen.degree_order(g)
    h = C.c_void_p()
    ptr = lambda a: a.ctypes.data  # noqa: E731
    w0 = g.w.copy()
    w0[3] = 0
    assert lib.pll_build_weighted(g.n, ptr(g.row_ptr), ptr(g.col), ptr(w0), ptr(order), 0, None,
                                  C.byref(h)) == binding.E_INVAL
    w1 = g.w.copy()
    w1[0] += 1  # (0,1) and (1,0) disagree
    assert lib.pll_build_weighted(g.n, ptr(g.row_ptr), ptr(g.col), ptr(w1), ptr(order),
                                  binding.VALIDATE, None, C.byref(h)) == binding.E_INVAL
    assert lib.pll_build_weighted(g.n, ptr(g.row_ptr), ptr(g.col), None, ptr(order), 0, None,
                                  C.byref(h)) == binding.E_INVAL
    assert lib.pll_export_weighted_parents(None, 0, ptr(np.zeros(1, np.uint32))) == binding.E_INVAL
    assert lib.pll_build_weighted(-1, None, None, None, None, 0, None, C.byref(h)) == binding.E_INVAL
    assert lib.pll_build_weighted(g.n, ptr(g.row_ptr), ptr(g.col), ptr(g.w), ptr(order), 0, None,
                                  None) == binding.E_INVAL
    bad = order.copy()
    bad[0] = bad[1]
    assert lib.pll_build_weighted(g.n, ptr(g.row_ptr), ptr(g.col), ptr(g.w), ptr(bad), 0, None,
                                  C.byref(h)) == binding.E_INVAL
    out = np.zeros(1, np.uint32)
    pairs = np.zeros(2, np.int32)
    assert lib.pll_query_weighted(None, ptr(pairs), 1, ptr(out), 0, None) == binding.E_INVAL
    assert lib.pll_export_weighted(None, 0, None, None, None, None, None) == binding.E_INVAL


def test_autotune_rejects_bad_arguments():
    lib = binding.library()
    pairs = np.zeros(2, np.int32)
    best = C.c_int32()
    assert lib.pll_autotune_query(None, pairs.ctypes.data, 1, 0, None, C.byref(best)) == binding.E_INVAL


def test_query_noalloc_rejects_bad_arguments_without_device_work():
    lib = binding.library()
    p = np.zeros(4, np.int32)
    out = np.zeros(2, np.uint8)
    assert lib.pll_query_noalloc(None, p.ctypes.data, 2, out.ctypes.data, 0, None) == binding.E_INVAL
    assert lib.pll_query_noalloc(None, p.ctypes.data, -1, out.ctypes.data, 0, None) == binding.E_INVAL
    assert binding.noalloc_max_pairs() == 1 << 21


def test_recorded_queries_and_build_autotune_reject_bad_arguments():
    lib = binding.library()
    h = C.c_void_p()
    p = np.zeros(4, np.int32)
    out = np.zeros(2, np.uint8)
    assert lib.pll_query_graph_create(None, p.ctypes.data, 2, out.ctypes.data,
                                      binding.DEVICE_PTRS, C.byref(h)) == binding.E_INVAL
    assert lib.pll_query_graph_create(None, p.ctypes.data, 2, out.ctypes.data, 0,
                                      None) == binding.E_INVAL
    assert lib.pll_query_graph_launch(None, None) == binding.E_INVAL
    assert lib.pll_query_graph_status(None, None) == binding.E_INVAL
    lib.pll_query_graph_free(None)
    g = graphs.cycle(5)
    order = gen.degree_order(g)
    assert lib.pll_autotune_build(g.n, g.row_ptr.ctypes.data, g.col.ctypes.data,
                                  order.ctypes.data, 0, binding.PLAIN, None,
                                  None) == binding.E_INVAL


def test_build_query_batch_rejects_bad_input_before_device_work():
    # qoff must start at 0 and not decrease, and every pair (host memory)
    # must lie inside its own graph; all checked before any device work
    lib = binding.library()
    vtx_off, rp, col, order = gen.pack_batch([graphs.cycle(4), graphs.path(3)])
    out = np.zeros(8, np.uint8)

    def rc(qoff, pairs):
        h = C.c_void_p()
        qoff = np.ascontiguousarray(qoff, np.int64)
        pairs = np.ascontiguousarray(pairs, np.int32)
        r = lib.pll_build_query_batch(2, vtx_off.ctypes.data, rp.ctypes.data, col.ctypes.data,
                                      order.ctypes.data, 0, qoff.ctypes.data, pairs.ctypes.data,
                                      out.ctypes.data, 0, None, C.byref(h))
        assert h.value is None
        return r

    good = np.array([[0, 3], [1, 2], [4, 6]], np.int32)
    assert rc([1, 2, 3], good) == binding.E_INVAL        # qoff[0] != 0
    assert rc([0, 3, 2], good) == binding.E_INVAL        # decreasing
    assert rc([0, 1, 3], good) == binding.E_INVAL        # [1, 2] counted in graph 1
    assert rc([0, 2, 3], [[0, 3], [1, 4], [4, 6]]) == binding.E_INVAL  # across graphs
    assert rc([0, 2, 3], [[0, 3], [1, 2], [4, 7]]) == binding.E_INVAL  # past the end
    h = C.c_void_p()
    q = np.array([0, 1, 1], np.int64)
    assert lib.pll_build_query_batch(2, vtx_off.ctypes.data, rp.ctypes.data, col.ctypes.data,
                                     order.ctypes.data, 0, q.ctypes.data, None, None, 0, None,
                                     C.byref(h)) == binding.E_INVAL  # pairs to answer, no buffers


def test_build_query_batch_binding_checks_buffer_sizes():
    # the binding refuses arrays shorter than qoff says before any call
    vtx_off, rp, col, order = gen.pack_batch([graphs.cycle(4), graphs.path(3)])
    with pytest.raises(ValueError):
        binding.build_query_batch(vtx_off, rp, col, order, 0, [0, 2, 3], np.zeros((2, 2), np.int32))
    with pytest.raises(ValueError):
        binding.build_query_batch(vtx_off, rp, col, order, 0, [0, 3], np.zeros((3, 2), np.int32))
    with pytest.raises(ValueError):
        binding.build_query_batch(vtx_off, rp, col, order, 0, [0, 2, 3], np.zeros((3, 2), np.int32),
                                  out=np.zeros(2, np.uint8))
