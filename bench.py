#!/usr/bin/env python3
"""Benchmark: Pruned Landmark Labeling index build + batched queries on one
MI355X.

One step = the whole hot path on one synthetic workload with its inputs
already in HBM: rank relabel, bit-parallel root choice, bit-parallel BFSs,
windowed pruned BFSs with cleaning, final label CSR, then one batch of query
pairs.  Default workload: R-MAT scale 22 (edge factor 16, a/b/c/d =
.57/.19/.19/.05, symmetrized, de-duplicated, self-loops dropped, largest
component kept), Degree order, t_bp = 64, 1e7 uniform random pairs.

Prints ONE JSON line.  "roofline" prices the dominant kernel's launches with
the per-unit byte model of level_kernel_bytes / expand_kernel_bytes below;
"method_bytes" prices the whole build with the method's own model over the
oracle's canonical work counters (s8d_bytes).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PLL index build s & edges/s; queries/s + p99 latency, batched vs plain"
HBM_PEAK_GBS = 8000.0
LEVEL_KERNEL_SRC = os.path.join(ROOT, "paper_1304_4661_amd", "csrc", "pruned.hip")
WSTEP_KERNEL_SRC = os.path.join(ROOT, "paper_1304_4661_amd", "csrc", "weighted.hip")
QUERY_KERNEL_SRC = os.path.join(ROOT, "paper_1304_4661_amd", "csrc", "query.hip")


def describe(name, g, t_bp, q):
    if g.meta.get("weights"):
        lo, hi, ws = g.meta["weights"]
        base = (f"R-MAT scale {g.meta['scale']}, edge factor {g.meta['edge_factor']}, abcd="
                f"{g.meta['abcd']}, symmetrized+dedup+no self-loops+largest component"
                if "scale" in g.meta else f"Barabasi-Albert n={g.n}, m={g.meta.get('m_attach')}")
        return (f"{base} (n'={g.n}, m'={g.m}), integer edge weights uniform in [{lo}, {hi}] "
                f"(seed {ws}); Degree order; pruned Dijkstra, no bit-parallel labels; {q} uniform "
                f"random pairs")
    if name == "ba256":
        return (f"{g.meta['graphs']} Barabasi-Albert graphs, n log-uniform in [1e3, 2e5], "
                f"m uniform in 2..8, seeded per graph (total n={g.n}, m={g.m}), one packed CSR, "
                f"Degree order per graph; t_bp={t_bp} per graph; {q} pairs inside the graphs")
    if g.meta.get("directed"):
        m = g.meta
        return (f"directed R-MAT scale {m['scale']}, edge factor {m['edge_factor']}, abcd="
                f"{m['abcd']}, arcs de-duplicated, no self-loops, largest weakly connected part "
                f"(n'={g.n}, arcs={len(g.col)}); in+out Degree order; t_bp=0; {q} uniform "
                f"random pairs")
    if name.startswith("rmat"):
        m = g.meta
        return (f"R-MAT scale {m['scale']}, edge factor {m['edge_factor']}, abcd="
                f"{m['abcd']}, symmetrized+dedup+no self-loops+largest component "
                f"(n'={g.n}, m'={g.m}); Degree order; t_bp={t_bp}; {q} uniform random pairs")
    m = g.meta
    return (f"Barabasi-Albert n={g.n}, m={m['m_attach']} (m'={g.m}); Degree order; "
            f"t_bp={t_bp}; {q} uniform random pairs")


def pctl(xs, p):
    return float(np.percentile(np.asarray(xs, dtype=np.float64), p)) if len(xs) else None


def file_sha(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def level_kernel_bytes(st, t_bp, sides=1):
    """Algorithmic bytes of the pruned-phase prune-test kernel (k_win_test),
    summed over all its launches in one build (per-unit figures):
      per level entry (root slot, vertex) past level 0: 8 B entry + t_bp B
        distance row (the roots themselves are labeled by the window's init
        kernel and never reach this kernel; a digraph's two search
        directions each label every root),
      per (S^{-1}, S^{0}) slot pair read by a set check: 32 B (root's and
        vertex's pair),
      per normal-label test: 12 B label offset and length, plus 5 B (hub +
        distance) per label entry scanned,
      per candidate label: 18 B (list entry 9 B, window distance 1 B, mask
        word 8 B)."""
    return ((st["visited"] - sides * st["roots"]) * (8 + t_bp) + 32 * st["bp_checks"] + 12 * st["normal_tests"]
            + 5 * st["label_scanned"] + 18 * st["candidates"])


def expand_row_bytes(t_bp):
    """Bytes of a reached neighbour's distance row as the expansion reads
    it: the 4-bit copy (half the padded row) when rows have 32 or 64 slots
    and the "packed_rows" knob is on, else t_bp."""
    from paper_1304_4661_amd import binding

    tpad = (t_bp + 15) & ~15
    if t_bp > 0 and tpad % 32 == 0 and binding.get_tuning("packed_rows"):
        return tpad // 2
    return t_bp


def expand_kernel_bytes(st, t_bp):
    """Algorithmic bytes of the pruned-phase expansion kernel (k_win_expand),
    summed over its launches in one build:
      per candidate expanded: 8 B list entry + 8 B row offsets + t_bp B root
        distance row,
      per adjacency entry expanded inline: 4 B neighbour; unless the
        neighbour is ranked before the window, + its distance row
        (expand_row_bytes); unless that row prunes it too, + 4 B visited word,
      per neighbour claimed: 8 B next-level list entry."""
    e = st["edges"]
    rest = e - st["expand_earlier"]
    return (st["candidates"] * (16 + t_bp) + 4 * e + rest * expand_row_bytes(t_bp)
            + 4 * (rest - st["expand_direct"]) + 8 * st["expand_claims"])


def weighted_step_bytes(st):
    """Algorithmic bytes of the weighted search step kernel (k_ww_step),
    summed over its launches in one build:
      per frontier entry processed: 8 B list entry + 4 B flag word + 4 B
        tentative distance,
      per prune test: 12 B label offset and length, plus 8 B per label entry
        scanned (packed hub and distance),
      per edge relaxed: 4 B neighbour + 4 B weight + 4 B tentative distance,
      per landmark check of a relaxation: 32 B (16 16-bit landmark distances
        of the reached vertex; a filtered edge then skips its tentative
        distance),
      per distance lowered: 4 B atomic minimum + 4 B flag word + 8 B list
        entry."""
    return (16 * st["visited"] + 12 * st["normal_tests"] + 8 * st["label_scanned"]
            + 12 * st["edges"] + 32 * st["land_checks"] - 4 * st["filtered"]
            + 16 * st["improved"])


def edges_of(g):
    """Input edges: undirected edges, or arcs of a directed graph."""
    return len(g.col) if g.meta.get("directed") else g.m


def query_threads():
    """Host threads for the all-core oracle query rate: the cores this process
    may use, at most 16 (one GPU's share of a box)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def oracle_query_rate_mt(fn, ox, pairs, threads):
    """Pairs answered per second by the oracle's query function `fn`, with
    the pairs split over `threads` host threads (the C oracle's queries only
    read the index, and ctypes releases the GIL during the call)."""
    from concurrent.futures import ThreadPoolExecutor

    parts = [p for p in np.array_split(np.ascontiguousarray(pairs), threads) if len(p)]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(lambda p: fn(ox, p), parts))
    return len(pairs) / (time.perf_counter() - t0)


def copy_bandwidth_gbs(dev):
    """Achievable HBM bandwidth on this GPU: a 1 GiB device-to-device copy
    (read + write bytes over the copy time, best of 5, HIP events), measured
    outside the timed region as the reference for the kernels' fractions."""
    import torch

    a = torch.empty(1 << 28, dtype=torch.int32, device=dev).fill_(1)
    b = torch.empty_like(a)
    b.copy_(a)
    best = None
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    gbs = 2 * a.numel() * 4 / (best * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbs


def load_golden(name):
    """The oracle's stored results for a full-size workload (digests, work
    counters, build timing with per-root checkpoints), or None."""
    path = os.path.join(ROOT, "tests", "golden", f"full_{name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def cpu_baseline(g, order, t_bp, pairs, name):
    """The oracle as it stands, one thread.  Small workloads: the whole step
    (index build + every query), live.  Workloads whose full oracle build
    takes minutes to an hour (R-MAT 20 / 22): a bounded live sample of the
    same oracle on the same CSR -- relabel plus the bit-parallel BFSs of the
    first 8 slots, no pruned BFSs -- timed here and on the machine where the
    full oracle run of the workload was stored with its digests; their ratio
    (this host's speed relative to that one) scales the stored full build
    and query times.  Returns the report and the oracle's work counters of
    the whole workload."""
    import oracle

    directed = bool(g.meta.get("directed"))
    gold = None if directed else load_golden(name)
    if gold is None or "calibration" not in gold:
        t0 = time.perf_counter()
        ox = (oracle.build_directed(g.row_ptr, g.col, order) if directed
              else oracle.build(g.row_ptr, g.col, order, t_bp))
        tb = time.perf_counter() - t0
        t0 = time.perf_counter()
        (oracle.query_directed if directed else oracle.query)(ox, pairs)
        tq = time.perf_counter() - t0
        entries = (len(ox.out_hub) + len(ox.in_hub)) if directed else ox.counters["entries"]
        nt = query_threads()
        qmt = oracle_query_rate_mt(oracle.query_directed if directed else oracle.query, ox, pairs,
                                   nt)
        return {
            "value": edges_of(g) / (tb + tq), "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": (f"whole step on the same workload: oracle index build ({tb:.2f} s) + "
                       f"{len(pairs)} queries ({tq:.2f} s), one thread"),
            "build_s": tb, "queries_per_s": len(pairs) / tq,
            "query_threads": nt, "queries_per_s_threads": qmt,
            "entries": entries,
        }, dict(ox.counters)
    assert gen_sha(g, order) == gold["csr_sha256"], "workload differs from the stored oracle run"
    cal = gold["calibration"]
    ts = []
    for _ in range(2):
        t0 = time.perf_counter()
        ox = oracle.build(g.row_ptr, g.col, order, cal["t_bp"], check_symmetric=False,
                          root_limit=cal["root_limit"])
        ts.append(time.perf_counter() - t0)
        ox.close()
    live = min(ts)
    ratio = live / cal["s"]
    build_est = gold["build_s"] * ratio
    q_est = gold["query_s"] * ratio * len(pairs) / gold["pairs"]
    return {
        "value": edges_of(g) / (build_est + q_est), "unit": "edges/s", "cores": 1,
        "kind": "oracle",
        "sample": (f"oracle on the same CSR, one thread: relabel + bit-parallel BFSs of the "
                   f"first {cal['t_bp']} slots, no pruned BFSs ({live:.2f} s here, best of 2; "
                   f"{cal['s']:.2f} s on the {gold['cpu_model']} host where the full oracle "
                   f"run of this workload took {gold['build_s']:.0f} s + {gold['query_s']:.1f} s "
                   f"for {gold['pairs']} queries); build and query times scaled by the ratio "
                   f"{ratio:.3f}"),
        "build_s_estimated": build_est, "query_s_estimated": q_est, "sample_s": live,
        "host_speed_ratio": ratio,
        "full_run": {"build_s": gold["build_s"], "bp_s": gold["times"]["bp_s"],
                     "pruned_s": gold["times"]["pruned_s"], "query_s": gold["query_s"],
                     "pairs": gold["pairs"], "cpu_model": gold["cpu_model"], "threads": 1,
                     "csr_sha256": gold["csr_sha256"], "kind": "cached"},
        "entries": gold["counters"]["entries"],
    }, dict(gold["counters"])


def gen_sha(g, order):
    from paper_1304_4661_amd import gen

    return gen.csr_sha256(g, order)


def s8d_bytes(c, n, t_bp):
    """Algorithmic bytes of the build from the oracle's canonical work
    counters (the visited, labeled and scanned sets are a function of graph,
    order and t_bp alone), per the byte model of the method:
      bit-parallel phase, per slot: 8 B row offsets + 17 B slot write per
        vertex reached, 5 B (neighbour + distance) per adjacency entry
        scanned, 16 B (two 64-bit sets) per E0 / E1 edge;
      pruned phase, per root: 5 B per entry of the root's label staged into
        T, 17 B per slot of its bit-parallel label; per vertex visited:
        16 B label offsets + 17 B per slot of its bit-parallel label, 5 B per
        entry of its label scanned by the normal test; per vertex labeled:
        8 B row offsets + 5 B append; per adjacency entry scanned: 5 B
        (neighbour + visited byte);
      finalize: 2 x (5 B per entry + 8 B per vertex)."""
    bp = 25 * c["bp_reached"] + 5 * c["bp_edges"] + 16 * (c["bp_e0"] + c["bp_e1"])
    pruned = (5 * c["root_staged"] + 17 * t_bp * c["roots"] + (16 + 17 * t_bp) * c["visited"]
              + 5 * c["label_scanned"] + 13 * c["labeled"] + 5 * c["edges"])
    final = 2 * (5 * c["entries"] + 8 * n)
    return bp, pruned, final


def query_pair_bytes(t_bp, lens_s, lens_t):
    """Bytes a batch of distance queries must move whatever the kernel: per
    pair 8 B (the pair) + 1 B (the answer), and per side 16 B label offsets,
    t_bp B bit-parallel distance row and 5 B per label entry up to and
    including the sentinel (hub 4 B + distance 1 B), the merge join reading
    both labels to the end (Section 3.3).  The bit-parallel sets (16 B per
    slot and side, Section 5.3) are read only for slots whose distances can
    still beat the best estimate, so they are not counted (the method's
    per-pair figure counts them all: + 32 x t_bp B per pair, reported
    beside)."""
    q = len(lens_s)
    return 9 * q + 2 * (16 + t_bp) * q + 5 * (int(lens_s.sum()) + int(lens_t.sum()) + 2 * q)


def cpu_baseline_batch(gs, vtx_off, t_bp, pairs, budget_s=20.0):
    """The oracle on a bounded sample of the batch: whole graphs in batch
    order (index build + their own pairs) until about budget_s of CPU time."""
    import oracle

    from paper_1304_4661_amd import gen

    m_done, t_done, q_done, k = 0, 0.0, 0, 0
    per = len(pairs) // len(gs)
    for i, g in enumerate(gs):
        if t_done > budget_s:
            break
        t0 = time.perf_counter()
        ox = oracle.build(g.row_ptr, g.col, gen.degree_order(g), t_bp)
        loc = pairs[i * per:(i + 1) * per] - np.int32(vtx_off[i])
        oracle.query(ox, loc)
        t_done += time.perf_counter() - t0
        m_done += g.m
        q_done += len(loc)
        k += 1
    return {"value": m_done / t_done, "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": (f"first {k} of {len(gs)} graphs ({m_done} edges, {q_done} pairs): "
                       f"oracle index builds + their queries, one thread, {t_done:.1f} s")}


def serving_loads(ix, nreq, max_batch=4096):
    """Serving on a device-resident index: requests of log-uniform size in
    [1, max_batch] pairs arrive as a Poisson process; X_sat = saturated
    requests/s (all requests at once), then offered loads of 0.25, 0.5 and
    0.85 X_sat, each with nreq requests.  Batched = continuous batching over
    4 slots; plain = one launch per request.  Latency counts from the
    scheduled arrival (open loop, so queueing counts)."""
    from paper_1304_4661_amd import binding

    res = {}
    for mode, co in (("batched", 1), ("plain", 0)):
        binding.set_tuning("serve_coalesce", co)
        binding.serve_bench(ix, 0.0, min(nreq, 2000), max_batch=max_batch, seed=104)  # warm-up
        sat = binding.serve_bench(ix, 0.0, nreq, max_batch=max_batch, seed=105)
        loads = {}
        for f in (0.25, 0.5, 0.85):
            r = binding.serve_bench(ix, f * sat["requests_per_s"], nreq, max_batch=max_batch,
                                    seed=106)
            loads[str(f)] = {k: r[k] for k in ("p50_us", "p99_us", "mean_us", "pairs_per_s",
                                                "requests_per_s", "pairs_per_launch",
                                                "launches", "max_launch_us", "max_launch_at",
                                                "max_worker_pause_us")}
        res[mode] = {"x_sat_requests_per_s": sat["requests_per_s"],
                     "x_sat_pairs_per_s": sat["pairs_per_s"], "loads": loads}
    binding.set_tuning("serve_coalesce", 1)
    return res


def serve(args):
    """Serving run on its own (see serving_loads)."""
    import torch

    from paper_1304_4661_amd import binding, gen

    name = args.config
    g, order, t_bp, _ = gen.config_graph(name)
    dev = torch.device("cuda:0")
    weighted = g.w is not None
    arrays = (g.row_ptr, g.col, g.w, order) if weighted else (g.row_ptr, g.col, order)
    d = [torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).to(dev) for a in arrays]

    def build():
        return (binding.build_weighted(*d, device=True) if weighted
                else binding.build_device(*d, t_bp))

    # the first build in a process also allocates the label pools and window
    # state; later builds reuse the library's cached blocks
    t0 = time.perf_counter()
    build().close()
    cold_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    ix = build()
    build_s = time.perf_counter() - t0
    st = ix.stats()
    nreq = args.serve_requests
    res = serving_loads(ix, nreq)
    print(json.dumps({
        "metric": "PLL serving: queries/s and p50/p99 request latency at offered loads",
        "value": res["batched"]["x_sat_pairs_per_s"], "unit": "queries/s",
        "higher_is_better": True, "n_gpus": 1, "dtype": "u32" if weighted else "u8",
        "data": "synthetic",
        "config": {"workload": describe(name, g, t_bp, nreq).replace(
                       f"{nreq} uniform random pairs", f"{nreq} requests per load of uniform "
                       "random pairs") + "; requests log-uniform in "
                   "[1, 4096] pairs, Poisson arrivals", "name": name, "n": g.n, "m": g.m,
                   "t_bp": t_bp, "requests_per_load": nreq},
        "build_s": build_s, "first_build_s": cold_s, "index": {"entries": st["entries"], "bytes": st["index_bytes"],
                                      "LN": f"{st['entries'] / max(g.n, 1):.1f}+{t_bp}"},
        "serving": res,
    }))


def traffic_for(kernel, config, src):
    """HBM bytes per launch of `kernel` on `config`, from the rocprofv3
    FETCH_SIZE and WRITE_SIZE passes stored in
    profiles/traffic_<kernel>_<config>.json (scaled by a plain copy of known
    size); None when the kernel's source changed since they were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{config}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        tr = json.load(f)
    if tr.get("kernel_source_sha") != file_sha(src):
        return None
    return tr.get("bytes_per_launch")


def kernel_roofline(kernel, desc, nbytes, secs, launches, build_ns, copy_gbs, traffic):
    ach = nbytes / secs / 1e9 if secs > 0 else None
    return {
        "kernel": f"{kernel} ({desc})", "bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS,
        "achieved": ach, "frac": (ach / HBM_PEAK_GBS) if ach else None, "traffic": traffic,
        "copy_gbs": copy_gbs, "frac_of_copy": (ach / copy_gbs) if ach else None,
        "launches": launches, "avg_launch_us": (secs / launches * 1e6) if launches else None,
        "algorithmic_bytes_per_launch": nbytes / launches if launches else None,
        "share_of_build": (secs / (build_ns * 1e-9)) if build_ns else None,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="rmat22")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the frontier and query tiles as set (skip both autotuners)")
    ap.add_argument("--knobs", default="",
                    help="library tuning knobs set first, e.g. root_sort=1,window_work=64000000")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the plain-form, serving and latency measurements")
    ap.add_argument("--serve", action="store_true",
                    help="serving run instead: saturated rate, then Poisson loads")
    ap.add_argument("--serve-requests", type=int, default=20000)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 1 GiB device copy (calibrates HBM byte counters)")
    ap.add_argument("--sweep", choices=["tbp", "orders"],
                    help="analysis instead of the step: t_bp sweep (Fig. 6) or vertex "
                         "orders (Table 5); one JSON line per point plus a table")
    ap.add_argument("--sweep-out", default=None, help="markdown table of the sweep")
    ap.add_argument("--max-random-scale", type=int, default=14,
                    help="largest R-MAT scale the Random order is built on")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the index "
              "build and the queries here are single-GPU", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1304_4661_amd import binding, gen

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    for kv in filter(None, args.knobs.split(",")):
        k, v = kv.split("=")
        binding.set_tuning(k.strip(), int(v))
    if args.copy_probe:
        a = torch.empty(1 << 28, dtype=torch.int32, device=dev).fill_(1)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": a.numel() * 4, "copies": 3}))
        return

    if args.serve:
        serve(args)
        return
    if args.sweep:
        sweep(args)
        return
    if args.config.endswith("w"):
        bench_weighted(args)
        return
    batch = args.config == "ba256"
    directed = args.config.endswith("d")
    if batch:
        gs, vtx_off, row_ptr, col, order, t_bp, pairs = gen.batch_workload()
        g = gen.Graph(int(vtx_off[-1]), row_ptr, col, {"kind": "batch", "graphs": len(gs)})
    else:
        g, order, t_bp, pairs = gen.config_graph(args.config)
        gs, vtx_off = [g], np.array([0, g.n], np.int64)
    print(f"workload {args.config}: n={g.n} m={edges_of(g)} t_bp={t_bp} pairs={len(pairs)}",
          file=sys.stderr, flush=True)
    q = len(pairs)
    d_row = torch.from_numpy(g.row_ptr).to(dev)
    d_col = torch.from_numpy(g.col).to(dev)
    d_order = torch.from_numpy(order).to(dev)
    d_pairs = torch.from_numpy(pairs).to(dev)
    d_out = torch.empty(q, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    binding.set_tuning("profile", 1)

    def build():
        if batch:
            return binding.build_batch(vtx_off, d_row, d_col, d_order, t_bp, stream=stream,
                                       device=True)
        return binding.build_device(d_row, d_col, d_order, t_bp, stream=stream, directed=directed)

    def step():
        ix = build()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        ix.query_device(d_pairs, d_out, stream=stream)
        ev1.record(stream)
        return ix, ev0, ev1

    for _ in range(args.warmup):
        ix, _, _ = step()
        ix.sync()
        ix.close()
    # frontier tiles autotuned on whole builds, query tiles on a sample of the
    # pairs, both before the timed region
    tiles = None
    if not args.no_autotune and not batch and not directed:
        tiles = binding.autotune_build(d_row, d_col, d_order, t_bp, stream=stream)
        print(f"build tiles {tiles}", file=sys.stderr, flush=True)
    ix = build()
    qgroup = (ix.autotune_query(d_pairs[: min(q, 200_000)].contiguous(), stream=stream)
              if q > 0 and not args.no_autotune else binding.get_tuning("qgroup"))
    ix.close()
    torch.cuda.synchronize()
    copy_gbs = copy_bandwidth_gbs(dev)
    print(f"warm-up done; timing {args.steps} steps", file=sys.stderr, flush=True)

    build_s, query_ms, stats = [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        tb = time.perf_counter()
        ix, ev0, ev1 = step()
        build_s.append(time.perf_counter() - tb)  # pll_build synchronises
        ix.sync()
        query_ms.append(ev0.elapsed_time(ev1))
        stats.append(ix.stats())
        ix.close()
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    ms_per_step = 1e3 * total / args.steps
    print(f"timed steps done: {ms_per_step:.1f} ms per step", file=sys.stderr, flush=True)

    st = stats[-1]
    launches = st["level_launches"]
    src = LEVEL_KERNEL_SRC
    roofline_test = kernel_roofline(
        "k_win_test", "pruned-BFS prune tests, all roots of a window, one level",
        level_kernel_bytes(st, t_bp, 2 if directed else 1), st["level_ns"] * 1e-9, launches,
        st["build_ns"], copy_gbs, traffic_for("k_win_test", args.config, src))
    roofline_expand = kernel_roofline(
        "k_win_expand", "pruned-BFS expansion, all roots of a window, one level",
        expand_kernel_bytes(st, t_bp), st["expand_ns"] * 1e-9, launches, st["build_ns"],
        copy_gbs, traffic_for("k_win_expand", args.config, src))
    # "roofline" is the level kernel with the larger share of the build; the
    # other one is reported beside it
    if (roofline_expand["share_of_build"] or 0) > (roofline_test["share_of_build"] or 0):
        roofline, other = roofline_expand, ("roofline_prune_test", roofline_test)
    else:
        roofline, other = roofline_test, ("roofline_expand", roofline_expand)

    out = {
        "metric": METRIC,
        "value": edges_of(g) / (ms_per_step / 1e3),
        "unit": "edges/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": describe(args.config, g, t_bp, q), "name": args.config,
                   "n": g.n, "m": edges_of(g), "t_bp": t_bp, "queries": q},
        "build_s": float(np.median(build_s)),
        "build_edges_per_s": edges_of(g) / float(np.median(build_s)),
        "queries_per_s": q / (float(np.median(query_ms)) / 1e3) if q else None,
        "query_batch_ms_p50": pctl(query_ms, 50), "query_batch_ms_p99": pctl(query_ms, 99),
        "query_lanes_per_pair": qgroup,
        "query_form": "persistent" if binding.get_tuning("qpersist") else "static",
        "build_tiles": tiles,
        "index": {"entries": st["entries"], "LN": f"{st['entries'] / max(g.n, 1):.1f}+{t_bp}",
                  "bytes": st["index_bytes"], "windows": st["windows"],
                  "retries": st["retries"], "visited": st["visited"],
                  "candidates": st["candidates"]},
        "counters": {k: int(v) for k, v in st.items()},
        "phases_s": {"bit_parallel": st["bp_ns"] * 1e-9, "pruned": st["pruned_ns"] * 1e-9},
        "roofline": roofline,
        other[0]: other[1],
    }

    if batch:
        # the small graphs built whole in one persistent launch (one
        # workgroup per graph) against the same batch with every graph in
        # the shared windows (whole_n = 0), one build each after the steps
        old_whole = binding.get_tuning("whole_n")
        wt = {}
        for lim in (old_whole, 0):
            binding.set_tuning("whole_n", lim)
            build().close()
            t1 = time.perf_counter()
            bx = build()
            wt[lim] = (time.perf_counter() - t1, bx.stats())
            bx.close()
        binding.set_tuning("whole_n", old_whole)
        # the same step in one call: build and answer every graph's pairs
        # (graphs built whole answer theirs inside the whole-graph launch)
        qoff = np.arange(len(gs) + 1, dtype=np.int64) * (q // len(gs))
        fused = []
        for r in range(2):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            bx, ans = binding.build_query_batch(vtx_off, d_row, d_col, d_order, t_bp, qoff,
                                                d_pairs, out=d_out, stream=stream, device=True)
            fused.append((time.perf_counter() - t1, bx.stats()["whole_pairs"]))
            bx.query_device(d_pairs, d_out2 := torch.empty_like(d_out), stream=stream)
            torch.cuda.synchronize()
            assert torch.equal(ans, d_out2), "fused answers differ from pll_query"
            bx.close()
        sw = wt[old_whole][1]
        out["whole_graph_launch"] = {
            "whole_n": old_whole, "graphs": sw["whole_graphs"],
            "vertices": int(sum(x.n for x in gs if 1 <= x.n <= old_whole)),
            "launch_s": sw["whole_ns"] * 1e-9, "build_s": wt[old_whole][0],
            "windows": sw["windows"], "build_s_all_windowed": wt[0][0],
            "windows_all_windowed": wt[0][1]["windows"],
            "build_and_query_one_call_s": fused[-1][0], "pairs_answered_in_launch": fused[-1][1],
            "step_s_build_then_query": float(np.median(build_s)) + float(np.median(query_ms)) / 1e3}
        print(f"whole-graph launch {out['whole_graph_launch']}", file=sys.stderr, flush=True)

    # the batched query kernel: bytes every pair must move (see
    # query_pair_bytes) over the step's query launches (events on the stream)
    lens_s = lens_t = None
    if q and not batch and not directed:
        ix = build()
        rank, lens = ix.label_lengths()
        ix.close()
        lens_s, lens_t = lens[rank[pairs[:, 0]]], lens[rank[pairs[:, 1]]]
        qb = query_pair_bytes(t_bp, lens_s, lens_t)
        qs = float(np.median(query_ms)) * 1e-3
        qr = kernel_roofline("k_query_group", f"batched distance queries, {q} pairs in one launch",
                             qb, qs, 1, None, copy_gbs,
                             traffic_for("k_query_group", args.config, QUERY_KERNEL_SRC))
        qr.pop("share_of_build")
        qr["bytes_per_pair"] = qb / q
        qr["method_bytes_per_pair"] = qb / q + 32 * t_bp
        qr["method_rate_gbs"] = (qb + 32 * t_bp * q) / qs / 1e9
        out["roofline_query"] = qr

    if not args.no_extras:
        ix = build()
        rates = {}
        for plain in (False, True):
            ix.query_device(d_pairs, d_out, stream=stream, plain=plain)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            reps = 5 if not plain else 2
            e0.record(stream)
            for _ in range(reps):
                ix.query_device(d_pairs, d_out, stream=stream, plain=plain)
            e1.record(stream)
            torch.cuda.synchronize()
            rates["plain" if plain else "batched"] = reps * q / (e0.elapsed_time(e1) / 1e3)
        lat = {}
        for bs in (1, 64, 4096):
            sub = d_pairs[:bs].contiguous()
            so = d_out[:bs]
            xs = []
            for i in range(200):
                t1 = time.perf_counter()
                ix.query_device(sub, so, stream=stream)
                torch.cuda.synchronize()
                xs.append((time.perf_counter() - t1) * 1e6)
            lat[str(bs)] = {"p50_us": pctl(xs[20:], 50), "p99_us": pctl(xs[20:], 99)}
        if args.config in ("rmat22", "rmat20") and not directed:
            out["serving"] = serving_loads(ix, args.serve_requests)
            out["serving"]["requests_per_load"] = args.serve_requests
            print("serving loads done", file=sys.stderr, flush=True)
        ix.close()
        # plain (one root at a time) vs windowed build on the small BA workload
        gb, ob, tb_, _ = gen.config_graph("ba2000")
        bt = {}
        for plain in (False, True):
            binding.build(gb.row_ptr, gb.col, ob, tb_, plain=plain).close()
            t1 = time.perf_counter()
            binding.build(gb.row_ptr, gb.col, ob, tb_, plain=plain).close()
            bt["plain" if plain else "batched"] = time.perf_counter() - t1
        out["plain_vs_batched"] = {
            "query_per_s": rates, "build_s_ba2000": bt,
        }
        out["query_latency_host_us"] = lat
        if not batch:
            out["shortest_paths"] = path_extra(g, d_row, d_col, d_order, t_bp, d_pairs, stream,
                                               directed=directed)

    binding.set_tuning("profile", 0)
    if not args.no_cpu_baseline:
        print("oracle baseline", file=sys.stderr, flush=True)
        if batch:
            out["cpu_baseline"] = cpu_baseline_batch(gs, vtx_off, t_bp, pairs)
            counters = None
        else:
            out["cpu_baseline"], counters = cpu_baseline(g, order, t_bp, pairs, args.config)
        out["cpu_baseline"]["cpu_model"] = cpu_model()
        if counters and not directed:
            # the method's byte model over the oracle's canonical work, per
            # GPU phase; the windowed form's extra work beside it
            bpb, prb, fib = s8d_bytes(counters, g.n, t_bp)
            qm = (query_pair_bytes(t_bp, lens_s, lens_t) + 32 * t_bp * q) if lens_s is not None else 0
            bp_s, pr_s = st["bp_ns"] * 1e-9, st["pruned_ns"] * 1e-9
            out["method_bytes"] = {
                "source": "oracle work counters of the same workload",
                "bit_parallel_bytes": bpb, "pruned_bytes": prb, "finalize_bytes": fib,
                "query_bytes": qm,
                "bit_parallel_frac": bpb / bp_s / 1e9 / HBM_PEAK_GBS if bp_s else None,
                "pruned_frac": (prb + fib) / pr_s / 1e9 / HBM_PEAK_GBS if pr_s else None,
                "whole_step_frac": (bpb + prb + fib + qm) / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
                # TEPS: edges the method scans (pruned BFSs + bit-parallel
                # BFSs, oracle counters) per second of GPU build
                "teps": (counters["edges"] + counters["bp_edges"]) / out["build_s"],
                "gpu_adjacency_entries_read": st["edges"] + st["task_edges"],
                "windowed_overhead": {
                    "gpu_visits": st["visited"], "canonical_visits": counters["visited"],
                    "gpu_candidates": st["candidates"], "entries": counters["entries"],
                    "extra_candidates": st["candidates"] - counters["entries"],
                    "expansion_skips_by_rank": st["earlier_root"],
                    "expansion_skips_by_distance_rows": st["bp_direct"]},
            }
    print(json.dumps(out))


def bench_weighted(args):
    """The weighted step (Section 6): pruned Dijkstra index build from
    device-resident inputs + one batch of queries, timed like the default
    step; roofline of the search step kernel; the oracle as CPU baseline."""
    import torch

    from paper_1304_4661_amd import binding, gen

    dev = torch.device("cuda:0")
    g, order, _, pairs = gen.config_graph(args.config)
    q = len(pairs)
    as_i32 = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).to(dev)  # noqa: E731
    d_row, d_col, d_w, d_order = as_i32(g.row_ptr), as_i32(g.col), as_i32(g.w), as_i32(order)
    d_pairs = torch.from_numpy(pairs).to(dev)
    d_out = torch.empty(q, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    binding.set_tuning("profile", 1)

    def step():
        ix = binding.build_weighted(d_row, d_col, d_w, d_order, stream=stream, device=True)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ix.query_weighted_device(d_pairs, d_out, stream=stream)
        e1.record(stream)
        return ix, e0, e1

    for _ in range(args.warmup):
        ix, _, _ = step()
        ix.sync()
        ix.close()
    ix = binding.build_weighted(d_row, d_col, d_w, d_order, stream=stream, device=True)
    qgroup = (ix.autotune_query(d_pairs[: min(q, 200_000)].contiguous(), stream=stream)
              if q > 0 and not args.no_autotune else binding.get_tuning("qgroup"))
    ix.close()
    torch.cuda.synchronize()
    copy_gbs = copy_bandwidth_gbs(dev)
    build_s, query_ms, stats = [], [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        tb = time.perf_counter()
        ix, e0, e1 = step()
        build_s.append(time.perf_counter() - tb)
        ix.sync()
        query_ms.append(e0.elapsed_time(e1))
        stats.append(ix.stats())
        ix.close()
    torch.cuda.synchronize()
    ms_per_step = 1e3 * (time.perf_counter() - t0) / args.steps
    binding.set_tuning("profile", 0)
    st = stats[-1]
    step_bytes = weighted_step_bytes(st)
    lvl_s = st["level_ns"] * 1e-9
    launches = st["level_launches"]
    achieved = step_bytes / lvl_s / 1e9 if lvl_s > 0 else None
    traffic = traffic_for("k_ww_step", args.config, WSTEP_KERNEL_SRC)
    out = {
        "metric": METRIC, "value": g.m / (ms_per_step / 1e3), "unit": "edges/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": describe(args.config, g, 0, q), "name": args.config, "n": g.n,
                   "m": g.m, "t_bp": 0, "queries": q},
        "build_s": float(np.median(build_s)),
        "build_edges_per_s": g.m / float(np.median(build_s)),
        "queries_per_s": q / (float(np.median(query_ms)) / 1e3),
        "query_batch_ms_p50": pctl(query_ms, 50), "query_batch_ms_p99": pctl(query_ms, 99),
        "query_lanes_per_pair": qgroup,
        "index": {"entries": st["entries"], "LN": f"{st['entries'] / max(g.n, 1):.1f}",
                  "bytes": st["index_bytes"], "windows": st["windows"], "retries": st["retries"],
                  "steps": st["levels"], "touched": st["touched"], "processed": st["visited"],
                  "filtered_relaxations": st["filtered"],
                  "candidates": st["candidates"]},
        "counters": {k: int(v) for k, v in st.items()},
        "roofline": {
            "kernel": "k_ww_step (weighted search step, all roots of a window, one step)",
            "bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS, "achieved": achieved,
            "frac": (achieved / HBM_PEAK_GBS) if achieved else None, "traffic": traffic,
            "copy_gbs": copy_gbs, "frac_of_copy": (achieved / copy_gbs) if achieved else None,
            "launches": launches, "avg_launch_us": (lvl_s / launches * 1e6) if launches else None,
            "algorithmic_bytes_per_launch": step_bytes / launches if launches else None,
            "share_of_build": lvl_s / (st["build_ns"] * 1e-9) if st["build_ns"] else None,
        },
    }
    if not args.no_extras:
        # Section 6 paths on the weighted index: build with parents, restore
        # 1e5 paths on the device (events on the stream)
        binding.build_weighted(d_row, d_col, d_w, d_order, stream=stream, device=True,
                               parents=True).close()
        t1 = time.perf_counter()
        ix = binding.build_weighted(d_row, d_col, d_w, d_order, stream=stream, device=True,
                                    parents=True)
        bs = time.perf_counter() - t1
        sub = d_pairs[:100_000].contiguous()
        paths = torch.empty((len(sub), 64), dtype=torch.int32, device=dev)
        lens = torch.empty(len(sub), dtype=torch.int32, device=dev)
        ix.query_path_device(sub, paths, lens, stream=stream)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(3):
            ix.query_path_device(sub, paths, lens, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ix.sync()
        ln = lens.cpu().numpy()
        ix.close()
        out["shortest_paths"] = {
            "build_s_with_parents": bs,
            "paths_per_s": 3 * len(sub) / (e0.elapsed_time(e1) / 1e3), "pairs": len(sub),
            "mean_vertices": float(ln[ln > 0].mean()) if (ln > 0).any() else 0.0}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_weighted(g, order, pairs)
        out["cpu_baseline"]["cpu_model"] = cpu_model()
    print(json.dumps(out))


def cpu_baseline_weighted(g, order, pairs, budget_q=200_000):
    """The weighted oracle as it stands, one thread: the whole index build
    of the same graph plus the first budget_q of the pairs."""
    import oracle

    t0 = time.perf_counter()
    ox = oracle.build_weighted(g.row_ptr, g.col, g.w, order)
    tb = time.perf_counter() - t0
    sub = pairs[:budget_q]
    t0 = time.perf_counter()
    oracle.query_weighted(ox, sub)
    tq = time.perf_counter() - t0 if len(sub) else 0.0
    tq_all = tq * len(pairs) / max(len(sub), 1)
    nt = query_threads()
    qmt = oracle_query_rate_mt(oracle.query_weighted, ox, sub, nt) if len(sub) else None
    return {
        "value": g.m / (tb + tq_all), "unit": "edges/s", "cores": 1, "kind": "oracle",
        "sample": (f"oracle index build of the whole graph ({tb:.2f} s) + {len(sub)} of the "
                   f"{len(pairs)} queries ({tq:.2f} s, scaled to all), one thread"),
        "build_s": tb, "queries_per_s": len(sub) / tq if tq > 0 else None,
        "query_threads": nt, "queries_per_s_threads": qmt,
        "entries": ox.counters["entries"],
    }


def sweep_point(g, order, t_bp, reps, nq=1_000_000):
    """Build the index reps times from device-resident inputs (median time)
    and time nq uniform random queries (batched and plain kernels, events on
    the stream); label sizes and index bytes from the build's counters."""
    import torch

    from paper_1304_4661_amd import binding, gen

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    d_row = torch.from_numpy(g.row_ptr).to(dev)
    d_col = torch.from_numpy(g.col).to(dev)
    d_order = torch.from_numpy(np.ascontiguousarray(order, np.int32)).to(dev)
    d_pairs = torch.from_numpy(gen.random_pairs(g.n, nq, 11)).to(dev)
    d_out = torch.empty(nq, dtype=torch.uint8, device=dev)
    binding.build_device(d_row, d_col, d_order, t_bp, stream=stream).close()
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ix = binding.build_device(d_row, d_col, d_order, t_bp, stream=stream)
        ts.append(time.perf_counter() - t1)
        st = ix.stats()
        if len(ts) < reps:
            ix.close()
    qns = {}
    for plain in (False, True):
        ix.query_device(d_pairs, d_out, stream=stream, plain=plain)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(3):
            ix.query_device(d_pairs, d_out, stream=stream, plain=plain)
        e1.record(stream)
        torch.cuda.synchronize()
        qns["plain" if plain else "batched"] = e0.elapsed_time(e1) * 1e6 / (3 * nq)
    ix.sync()
    ix.close()
    return {"n": g.n, "m": g.m, "t_bp": t_bp, "build_s": float(np.median(ts)),
            "ln_normal": st["entries"] / max(g.n, 1), "ln_bp": t_bp, "bp_vertices": st["bp_used"],
            "index_bytes": st["index_bytes"], "query_ns_batched": qns["batched"],
            "query_ns_plain": qns["plain"], "visited": st["visited"]}


def sweep(args):
    """The paper's two parameter studies on synthetic graphs: the number of
    bit-parallel roots (Fig. 6: build time, query time, normal label size,
    index size) and the vertex order (Table 5: average label size with no
    bit-parallel roots, Random / Degree / Closeness)."""
    from paper_1304_4661_amd import gen

    rows = []
    if args.sweep == "tbp":
        graphs_ = [("rmat18", gen.rmat_graph(18, seed=1)), ("ba200k_m4", gen.ba_graph(200_000, 4, 3))]
        from paper_1304_4661_amd import binding

        for gname, g in graphs_:
            order = gen.degree_order(g)
            # t_bp = 0 as the paper runs it (plain pruned BFSs) and with the
            # library's landmark rows (same labels, less work)
            for t, land in ((0, 0), (0, 1), (1, 1), (2, 1), (4, 1), (8, 1), (16, 1), (32, 1),
                            (50, 1), (64, 1)):
                binding.set_tuning("landmarks", land)
                r = {"graph": gname, "order": "degree", "landmarks": land if t == 0 else "-",
                     **sweep_point(g, order, t, args.steps)}
                rows.append(r)
                print(json.dumps(r), flush=True)
            binding.set_tuning("landmarks", 1)
        cols = ["graph", "t_bp", "landmarks", "build_s", "query_ns_batched", "query_ns_plain",
                "ln_normal", "ln_bp", "index_bytes"]
    else:
        graphs_ = [(f"rmat{s}", gen.rmat_graph(s, seed=1)) for s in (12, 14, 16, 18)]
        graphs_.append(("ba200k_m4", gen.ba_graph(200_000, 4, 3)))
        for gname, g in graphs_:
            orders = [("degree", gen.degree_order(g)), ("closeness", gen.closeness_order(g, 16, 0))]
            scale = int(gname[4:]) if gname.startswith("rmat") else 99
            if scale <= args.max_random_scale:
                orders.append(("random", gen.random_order(g.n, 0)))
            for oname, order in orders:
                r = {"graph": gname, "order": oname, **sweep_point(g, order, 0, args.steps)}
                rows.append(r)
                print(json.dumps(r), flush=True)
        cols = ["graph", "n", "m", "order", "ln_normal", "build_s", "query_ns_batched",
                "index_bytes"]
    if args.sweep_out:
        def fmt(v):
            return f"{v:.4g}" if isinstance(v, float) else str(v)
        with open(args.sweep_out, "w") as f:
            f.write("| " + " | ".join(cols) + " |\n|" + "---|" * len(cols) + "\n")
            for r in rows:
                f.write("| " + " | ".join(fmt(r[c]) for c in cols) + " |\n")


def path_extra(g, d_row, d_col, d_order, t_bp, d_pairs, stream, nq=100_000, max_len=32,
               directed=False):
    """Build with parents (Section 6) and restore nq shortest paths on the
    device; inputs and outputs in HBM, timed with events on the stream."""
    import torch

    from paper_1304_4661_amd import binding

    binding.build_device(d_row, d_col, d_order, t_bp, stream=stream, parents=True,
                         directed=directed).close()
    t1 = time.perf_counter()
    ix = binding.build_device(d_row, d_col, d_order, t_bp, stream=stream, parents=True,
                              directed=directed)
    bs = time.perf_counter() - t1
    pairs = d_pairs[:nq].contiguous()
    paths = torch.empty((len(pairs), max_len), dtype=torch.int32, device=pairs.device)
    lens = torch.empty(len(pairs), dtype=torch.int32, device=pairs.device)
    ix.query_path_device(pairs, paths, lens, stream=stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(3):
        ix.query_path_device(pairs, paths, lens, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ix.sync()
    ln = lens.cpu().numpy()
    ix.close()
    return {"build_s_with_parents": bs, "paths_per_s": 3 * len(pairs) / (e0.elapsed_time(e1) / 1e3),
            "pairs": len(pairs), "mean_vertices": float(ln[ln > 0].mean()) if (ln > 0).any() else 0.0}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


if __name__ == "__main__":
    main()
