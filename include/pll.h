/*
 * pll.h -- C ABI of the MI355X (gfx950) Pruned Landmark Labeling library.
 *
 * Method: T. Akiba, Y. Iwata, Y. Yoshida, "Fast Exact Shortest-Path Distance
 * Queries on Large Networks by Pruned Landmark Labeling", SIGMOD 2013.
 *
 * The library builds a 2-hop distance-labeling index of an undirected,
 * unweighted graph (bit-parallel labels, Section 5, plus pruned-BFS labels,
 * Section 4) on one GPU and answers exact distance queries from it
 * (Sections 3.3 and 5.3); Section 6's extensions are here too: shortest
 * paths (PLL_PARENTS), directed graphs (PLL_DIRECTED) and weighted graphs
 * (pll_build_weighted).  Every step of the build and of the query runs in
 * the library's own HIP kernels; the index stays in device memory.
 *
 * Conventions shared by all entry points
 *   - Only fixed-width C types cross the ABI.  No C++ exception escapes.
 *   - Return value: PLL_OK (0) or a negative PLL_E_* code.  A failed call
 *     leaks nothing and leaves every output untouched (*out stays NULL).
 *   - Vertex ids are int32 in [0, n).  "Rank" is the position of a vertex in
 *     the caller's order (order[rank] = id); hubs are stored as ranks
 *     (Section 4.5.1, "Sorting Labels").
 *   - Distances are uint8.  255 (PLL_INF) means "unreachable"; a query whose
 *     exact distance is 255 or more also reads 255.  A build in which some
 *     stored distance would reach 255 fails with PLL_E_RANGE.
 *   - stream: a hipStream_t, or NULL for the null stream.
 *   - Not thread-safe against pll_free of the same index; queries on one
 *     index may run concurrently from several host threads and streams.
 */
#ifndef PLL_H_
#define PLL_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pll_index pll_index; /* opaque; owns the index's device memory */

enum {
  PLL_OK = 0,
  PLL_E_INVAL = -1,       /* bad argument, detected before any device work */
  PLL_E_NOMEM = -2,       /* host or device allocation failed */
  PLL_E_RANGE = -3,       /* a stored distance would reach 255 */
  PLL_E_DEVICE = -4,      /* a HIP call failed */
  PLL_E_UNSUPPORTED = -5  /* valid request the library does not handle */
};

#define PLL_INF 255u
#define PLL_MAX_TBP 64 /* bit-parallel slots: one 64-bit word per set (b = 64) */

/* flags */
#define PLL_DEVICE_PTRS 1u /* array arguments are device pointers */
#define PLL_VALIDATE 2u    /* pll_build*: also check that the graph is symmetric */
#define PLL_SYNC 4u        /* block until the call's device work is complete */
#define PLL_PLAIN 8u       /* plain forms: build one root at a time (no
                              concurrent roots); query one thread per pair */
#define PLL_PARENTS 16u    /* pll_build*: keep, with every label entry (h, d) of
                              v, the parent of v in the pruned BFS tree of h
                              (Section 6), plus the graph, for pll_query_path */
#define PLL_DIRECTED 32u   /* pll_build*: the CSR lists out-arcs of a directed
                              graph (Section 6): labels L_OUT and L_IN, queries
                              give the distance from s to t along the arcs;
                              needs t_bp = 0 (else PLL_E_UNSUPPORTED); no
                              symmetry is required; with PLL_PARENTS both
                              labels keep parents and paths follow the arcs */

/*
 * Device allocator for builds and indexes (process-wide; the default is
 * hipMalloc/hipFree behind a cache of freed blocks, see "pool_keep_mb").  alloc(bytes, stream, ctx)
 * returns device memory or NULL (then the call fails with PLL_E_NOMEM);
 * `stream` is the stream of the build that asked, so a stream-ordered
 * allocator (for example a caching allocator's raw alloc/delete) may reuse
 * memory in stream order.
 * free_(ptr, stream, ctx) gets the same stream.  Index memory is released
 * by pll_free, which the caller issues only when no work on the index is
 * pending.  Both NULL restores the default; exactly one NULL is
 * PLL_E_INVAL.  Memory keeps the allocator it came from: changing the hook
 * does not affect existing indexes.
 */
int pll_set_allocator(void *(*alloc)(size_t bytes, void *stream, void *ctx),
                      void (*free_)(void *ptr, void *stream, void *ctx), void *ctx);

/*
 * Build the index of one graph (Algorithm 2 with the bit-parallel phase of
 * Section 5.4 in front).
 *   n        number of vertices (>= 0)
 *   row_ptr  int32[n+1], CSR row offsets: row_ptr[0] = 0, non-decreasing
 *   col      int32[row_ptr[n]], neighbour ids; the graph must be
 *            symmetric (each edge in both rows) with no self-loops;
 *            repeated edges are allowed
 *   order    int32[n], a permutation: order[i] is the vertex of rank i
 *            (Section 4.4; pruned BFSs run in this order)
 *   t_bp     number of bit-parallel roots, 0..PLL_MAX_TBP (Section 5.4: the
 *            root is the lowest-rank unused vertex, its up to 64 lowest-rank
 *            unused neighbours form S_r; an exhausted slot stays empty)
 *   flags    PLL_VALIDATE, PLL_PLAIN, PLL_SYNC, PLL_DEVICE_PTRS, PLL_PARENTS,
 *            PLL_DIRECTED
 *   out      receives the new index on success
 * row_ptr, col and order are host memory, or device memory under
 * PLL_DEVICE_PTRS (then they are checked by a kernel before the build, and
 * PLL_VALIDATE is PLL_E_UNSUPPORTED).  The inputs are copied or only read;
 * the caller may free them when the call returns.
 * Errors: PLL_E_INVAL (bad CSR, self-loop, out-of-range id, order not a
 * permutation, t_bp outside 0..64, asymmetric graph under PLL_VALIDATE),
 * PLL_E_RANGE, PLL_E_NOMEM, PLL_E_DEVICE.  The build always synchronises
 * the stream before returning.
 */
int pll_build(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *order,
              int32_t t_bp, uint32_t flags, void *stream, pll_index **out);

/*
 * Answer q distance queries (Section 3.3 merge join over the normal labels,
 * Section 5.3 bit-parallel rule): out[i] = min(d(pairs[2i], pairs[2i+1]), 255).
 *   pairs  int32[2q], ids (s0,t0,s1,t1,...); host memory, or device memory
 *          under PLL_DEVICE_PTRS
 *   out    uint8[q], same memory kind as pairs
 *   flags  PLL_DEVICE_PTRS, PLL_SYNC, PLL_PLAIN
 * Host pointers: validated on the host, copied, and the call synchronises.
 * Device pointers: a validation kernel runs first; if any id is out of range
 * nothing is written and the error is returned by this call under PLL_SYNC,
 * else by the next pll_sync on the index.  The caller keeps device buffers
 * alive until the stream passes the call.
 * Errors: PLL_E_INVAL (null index, q < 0, id out of range), PLL_E_NOMEM,
 * PLL_E_DEVICE.
 */
int pll_query(const pll_index *idx, const int32_t *pairs, int64_t q, uint8_t *out,
              uint32_t flags, void *stream);

/*
 * Build the indexes of G independent graphs at once (each graph exactly as
 * pll_build would index it alone: its own order, its own t_bp bit-parallel
 * roots, labels over its own vertices).
 *   G        number of graphs (>= 0)
 *   vtx_off  host int64[G+1]: graph g owns global ids [vtx_off[g],
 *            vtx_off[g+1]); vtx_off[0] = 0, non-decreasing, total < 2^31
 *   row_ptr  int32[N+1], col int32[row_ptr[N]]: one CSR over global ids;
 *            every edge stays inside its graph; symmetric, no self-loops
 *   order    int32[N]: order[vtx_off[g] + i] is the LOCAL id (0-based
 *            within graph g) of graph g's vertex of local rank i
 *   t_bp, flags, stream, out: as pll_build (PLL_DEVICE_PTRS applies to
 *            row_ptr, col and order; vtx_off is always host memory)
 * Graphs of 1 .. "whole_n" vertices (a tuning knob, default 4096, at most
 * 16384; 0 turns this off) are built whole, one workgroup per graph, in one persistent
 * launch: each workgroup takes graphs from a shared cursor, largest first,
 * and runs the graph's pruned BFSs root after root with the root's label
 * table, visited bits and BFS queue in LDS (Section 4.2's loop, Section
 * 4.5.1's T array).  The other graphs share the windowed launches: their
 * roots are interleaved by local rank into one build over their disjoint
 * union.  Either way every graph gets its own labels.  Export and
 * statistics take the graph index; pll_stats reports the whole batch.
 * Not used by a directed batch or under PLL_PLAIN.
 * Errors: as pll_build, plus PLL_E_INVAL for a bad vtx_off, an edge leaving
 * its graph, or an order entry outside its graph.
 */
int pll_build_batch(int32_t G, const int64_t *vtx_off, const int32_t *row_ptr, const int32_t *col,
                    const int32_t *order, int32_t t_bp, uint32_t flags, void *stream,
                    pll_index **out);

/*
 * pll_build_batch plus one batch of distance queries per graph (QUERY of
 * Section 3.3 with the bit-parallel rule of Section 5.3, clamped to 255),
 * answered in the same call: a graph built whole answers its pairs inside
 * the whole-graph launch, by the workgroup that built it, as soon as its
 * labels are complete; the pairs of the other graphs are answered after the
 * build by the batched query kernel.  The answers equal pll_query's on the
 * returned index.
 *   G, vtx_off, row_ptr, col, order, t_bp, stream, idx: as pll_build_batch
 *   qoff   host int64[G+1]: graph g's pairs are pairs[2 qoff[g] ..
 *          2 qoff[g+1]) (global ids of graph g; qoff[0] = 0, non-decreasing)
 *   pairs  int32[2 qoff[G]], out uint8[qoff[G]]: host memory, or device
 *          memory under PLL_DEVICE_PTRS (like row_ptr, col and order; then
 *          the answers are complete when the stream passes the call, or on
 *          return under PLL_SYNC; the caller keeps both buffers alive)
 * Errors: as pll_build_batch, plus PLL_E_INVAL for a bad qoff, a null
 * pairs/out with pairs to answer, or an id outside its graph (host
 * pointers) or outside [0, N) (device pointers: a pair across graphs then
 * answers 255).  On an error nothing is returned in idx.
 */
int pll_build_query_batch(int32_t G, const int64_t *vtx_off, const int32_t *row_ptr,
                          const int32_t *col, const int32_t *order, int32_t t_bp,
                          const int64_t *qoff, const int32_t *pairs, uint8_t *out,
                          uint32_t flags, void *stream, pll_index **idx);

/*
 * Queries on an index from pll_build_batch, by global ids: pairs inside one
 * graph get that graph's distance, pairs across graphs get 255.  Same
 * arguments, memory rules and errors as pll_query (which behaves the same
 * on a batch index).
 */
int pll_query_batch(const pll_index *idx, const int32_t *pairs, int64_t q, uint8_t *out,
                    uint32_t flags, void *stream);

/*
 * pll_query without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, answers and errors as pll_query.
 * pll_query allocates per call a 4-byte error flag (device pointers) or
 * device staging for the pairs and answers (host pointers); here both live
 * in one static device array of pll_query_noalloc_max_pairs() * 9 + 256
 * bytes (about 18.9 MB) that every GPU the library runs on holds until the
 * process ends.
 *   - Host pointers: q may not exceed pll_query_noalloc_max_pairs()
 *     (2,097,152): larger q is PLL_E_INVAL, nothing written.  The call
 *     synchronises the stream.
 *   - Device pointers: no limit on q (nothing is staged); the flag is
 *     cleared by a kernel (no memset), so the call may be captured in a HIP
 *     graph when PLL_SYNC is not set.
 * The array is shared by every call on the same GPU and keeps the last
 * call's contents: calls on one GPU that overlap in time (other streams or
 * host threads) race on it and must be serialised by the caller.  Call it
 * with the index's device current.
 */
int pll_query_noalloc(const pll_index *idx, const int32_t *pairs, int64_t q, uint8_t *out,
                      uint32_t flags, void *stream);
int64_t pll_query_noalloc_max_pairs(void);

/*
 * A batch of distance queries recorded once as a HIP graph and replayed
 * (Sections 3.3 and 5.3, as pll_query): for callers that answer a stream of
 * equally sized batches from fixed device buffers, a replay is one graph
 * launch of the three recorded kernels (clear the batch's error flag, check
 * the ids, answer the pairs) instead of three launches and an allocation.
 *   pll_query_graph_create: records the batch for device buffers pairs
 *     int32[2q] and out uint8[q] (flags must hold PLL_DEVICE_PTRS; PLL_PLAIN
 *     records the plain form; otherwise the batched form the "qgroup" and
 *     "qpersist" knobs select at this time).  The buffers' contents may
 *     change between replays, their addresses may not; the caller keeps
 *     them and the index alive until pll_query_graph_free.  Allocates 16
 *     bytes of device memory (the flag and the persistent form's cursor).
 *   pll_query_graph_launch: replays it on stream (asynchronous).
 *   pll_query_graph_status: waits for stream; PLL_E_INVAL if the last replay
 *     met an id outside [0, n) (then it wrote no answer), else PLL_OK.
 *   pll_query_graph_free: releases the graph (NULL is ignored).
 * Replays on one graph must not overlap in time (they share the flag).
 * Errors: PLL_E_INVAL (null index or output, q < 0, host pointers),
 * PLL_E_UNSUPPORTED (weighted index), PLL_E_NOMEM, PLL_E_DEVICE.
 */
typedef struct pll_qgraph pll_qgraph;
int pll_query_graph_create(const pll_index *idx, const int32_t *pairs, int64_t q, uint8_t *out,
                           uint32_t flags, pll_qgraph **g);
int pll_query_graph_launch(pll_qgraph *g, void *stream);
int pll_query_graph_status(pll_qgraph *g, void *stream);
void pll_query_graph_free(pll_qgraph *g);

/*
 * Autotuner of the batched query kernels: times every lane group size
 * (16, 32 and 64 lanes per pair) on q sample pairs of this index, each in
 * the static and (unweighted indexes) the persistent batched form (3 timed
 * launches each after a warm-up, HIP events on stream), sets the
 * process-wide "qgroup" and "qpersist" knobs to the fastest and writes the
 * lanes per pair to *best (may be NULL).  Works for unweighted and weighted indexes.  pairs: int32[2q] ids,
 * host memory or device memory under PLL_DEVICE_PTRS (validated first).
 * Synchronises the stream.  Errors: PLL_E_INVAL (null index or pairs,
 * q <= 0, id out of range), PLL_E_NOMEM, PLL_E_DEVICE.
 */
int pll_autotune_query(const pll_index *idx, const int32_t *pairs, int64_t q, uint32_t flags,
                       void *stream, int32_t *best);

/*
 * Autotuner of the pruned phase's frontier tiles: times whole builds of
 * this graph (arguments as pll_build, which it calls; PLL_PLAIN and
 * PLL_PARENTS are PLL_E_INVAL) while it varies one knob at a time from the
 * current settings, in two passes over the knobs -- "xgroup" (lanes per candidate expansion: 8, 16, 32),
 * "chunk" (edges expanded inline: 128, 256, 512), "window_work" (visits
 * per window: 64M, 128M, 256M) and "sort_level" (level size from which the
 * prune tests are grouped by root: 2^18, 2^20, 2^22) -- keeps each knob at
 * its fastest value (the lanes per prune test are chosen per window by the
 * build itself) and writes the four values to best[4] (may be NULL).  The
 * labels do not depend on these knobs.  Cost: up to 24 builds.  Errors: as
 * pll_build; on an error the knob being tried is restored.
 */
int pll_autotune_build(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *order,
                       int32_t t_bp, uint32_t flags, void *stream, int64_t *best);

/*
 * Wait for the index's work on stream and return (and clear) the error
 * recorded by earlier asynchronous pll_query calls with device pointers.
 */
int pll_sync(const pll_index *idx, void *stream);

/*
 * Sizes of one graph of the index for pll_export: vertices, normal label
 * entries (no sentinels) and bit-parallel slots.  graph is 0 for an index
 * made by pll_build, 0..G-1 for a batch.  Any pointer may be NULL.
 */
int pll_export_sizes(const pll_index *idx, int32_t graph, int64_t *n, int64_t *entries,
                     int32_t *t_bp);

/*
 * Copy one graph's index to host memory in the canonical layout used for
 * bit-exact comparison: vertices in (local) rank order; off int64[n+1]
 * (off[0] = 0), hub uint32[entries] (hub local ranks, ascending within each
 * vertex), dist
 * uint8[entries], no sentinels (Section 4.5.2 keeps a sentinel in storage
 * only); bp_d uint8[n][t_bp], bp_m1 / bp_0 uint64[n][t_bp] (the S^{-1} and
 * S^{0} sets of Section 5.1, bit j = j-th chosen neighbour in ascending rank).
 * Any output pointer may be NULL to skip that array.  rank: int32[n] local
 * id -> local rank.
 */
/*
 * Shortest paths (Section 6, "Shortest-Path Queries") of q pairs, for an
 * index built with PLL_PARENTS (else PLL_E_UNSUPPORTED).  On a weighted
 * index lens[i] counts the vertices of the path (it is not d+1 there): 0
 * if unreachable, -(vertices) if max_len is too small.
 *   pairs    int32[2q] ids, as pll_query
 *   max_len  vertices room per path (>= 0)
 *   paths    int32[q][max_len]: row i gets the ids of a shortest path from
 *            pairs[2i] to pairs[2i+1], both ends included
 *   lens     int32[q]: d+1 (vertices written); 0 if unreachable or 255 or
 *            more away (the distance query's 255); -(d+1) if max_len < d+1
 *            (row not written); INT32_MIN only for an inconsistent index
 * When the best common hub h of the normal labels gives the distance (ties
 * go to it, then to the lowest hub), the path ascends the BFS trees of h
 * from both ends (for a digraph: h is the best hub of L_OUT(s) and L_IN(t),
 * and the path follows the arcs).  When only a bit-parallel slot gives it (lowest slot on
 * ties), the path is walked through neighbours in ascending rank: to the
 * slot's root, or to its chosen neighbour w in S^{-1} / S^{0} (Section 5.1
 * sets) of both ends.  Parents are chosen by a fixed rule (see
 * pll_export_parents), so the same index and pair always give the same
 * path, whatever the window sizes of the build.  Memory kinds,
 * validation, errors and PLL_SYNC as pll_query.
 */
int pll_query_path(const pll_index *idx, const int32_t *pairs, int64_t q, int32_t max_len,
                   int32_t *paths, int32_t *lens, uint32_t flags, void *stream);

/*
 * Parents of one graph's label entries (index built with PLL_PARENTS, else
 * PLL_E_UNSUPPORTED), in pll_export's entry order, as local ranks: the
 * parent of vertex v for entry (h, d) is the lowest-ranked neighbour p of v
 * whose label holds (h, d-1) -- a vertex the BFS from h labeled one step
 * closer, so v's parent in that BFS tree -- and v itself for d = 0 (for
 * L_OUT of a digraph: the lowest-ranked out-neighbour p of v with (h, d-1)
 * in L_OUT(p)).  par: host uint32[entries].
 */
int pll_export_parents(const pll_index *idx, int32_t graph, uint32_t *par);

/*
 * Parents of the L_IN entries of a directed index built with PLL_PARENTS
 * (else PLL_E_UNSUPPORTED), in pll_export_in's entry order, as local ranks:
 * for (h, d) in L_IN(v), the lowest-ranked in-neighbour p of v with (h, d-1)
 * in L_IN(p), and v itself for d = 0.  par: host uint32[entries of
 * pll_export_in].
 */
int pll_export_in_parents(const pll_index *idx, int32_t graph, uint32_t *par);

/*
 * L_IN of one graph of a directed index (built with PLL_DIRECTED, else
 * PLL_E_UNSUPPORTED), in pll_export's layout: vertices in local rank order,
 * off int64[n+1], hub uint32[entries] (local ranks), dist uint8[entries],
 * no sentinels; (h, d) in L_IN(v) means d(h, v) = d.  *entries gets the
 * entry count; pass NULL arrays to ask for it first.  pll_export gives
 * L_OUT of a directed index ((h, d) in L_OUT(v): d(v, h) = d).
 */
int pll_export_in(const pll_index *idx, int32_t graph, int64_t *entries, int64_t *off,
                  uint32_t *hub, uint8_t *dist);

int pll_export(const pll_index *idx, int32_t graph, int64_t *off, uint32_t *hub, uint8_t *dist,
               uint8_t *bp_d, uint64_t *bp_m1, uint64_t *bp_0, int32_t *rank);

/*
 * Weighted graphs (Section 6, "Weighted Graphs"): every vertex, in rank
 * order, runs a pruned Dijkstra search in place of the pruned BFS; there are
 * no bit-parallel labels and distances are uint32.
 *   n, row_ptr, col, order, stream, out: as pll_build (one graph)
 *   wgt      uint32[row_ptr[n]]: weight of edge col[e], >= 1 (0 is
 *            PLL_E_INVAL); an undirected graph lists every edge in both
 *            rows with the same weight (checked under PLL_VALIDATE)
 *   flags    PLL_DEVICE_PTRS (row_ptr, col, wgt and order on the device),
 *            PLL_VALIDATE (host pointers only), PLL_PLAIN (one root at a
 *            time), PLL_DIRECTED (the CSR lists out-arcs; labels L_OUT and
 *            L_IN as for pll_build), PLL_PARENTS (every entry keeps the
 *            parent of its vertex in the hub's search tree: among the
 *            vertices p with an edge p -> v whose label holds
 *            (h, d - w(p, v)), the lowest ranked; pll_query_path then
 *            restores paths)
 * A relaxation whose distance would reach 2^32 - 1 is dropped: a vertex that
 * far from a root counts as unreachable from it, so the labels are the
 * exact ones with distance below 2^32 - 1 and queries read 2^32 - 1
 * (PLL_WINF) for pairs that are unreachable or at least that far apart.
 * Errors: as pll_build.  The index answers only pll_query_weighted,
 * pll_export_weighted, pll_export_weighted_parents, pll_query_path (with
 * PLL_PARENTS), pll_export_sizes, pll_stats, pll_sync and pll_free (other
 * calls return PLL_E_UNSUPPORTED).  Always synchronises the stream.
 */
#define PLL_WINF 0xFFFFFFFFu
int pll_build_weighted(int32_t n, const int32_t *row_ptr, const int32_t *col, const uint32_t *wgt,
                       const int32_t *order, uint32_t flags, void *stream, pll_index **out);

/*
 * Distance queries on a weighted index: out[i] = min(d(s_i, t_i), PLL_WINF)
 * as uint32 (along the arcs for a digraph), merge join of Section 3.3 with
 * 64-bit sums.  pairs, out: host memory, or device memory under
 * PLL_DEVICE_PTRS; validation, PLL_SYNC, PLL_PLAIN and errors as
 * pll_query.  PLL_E_UNSUPPORTED on an unweighted index.
 */
int pll_query_weighted(const pll_index *idx, const int32_t *pairs, int64_t q, uint32_t *out,
                       uint32_t flags, void *stream);

/*
 * Labels of a weighted index in rank order without sentinels: side 0 is L
 * (L_OUT of a digraph: (h, d) means d(v, h) = d), side 1 is L_IN of a
 * digraph ((h, d): d(h, v) = d).  entries gets the entry count; off
 * int64[n+1], hub uint32[entries] (ranks, ascending per vertex), dist
 * uint32[entries], rank int32[n] (id -> rank); any pointer may be NULL.
 * PLL_E_UNSUPPORTED on an unweighted index or side 1 of an undirected one.
 */
int pll_export_weighted(const pll_index *idx, int32_t side, int64_t *entries, int64_t *off,
                        uint32_t *hub, uint32_t *dist, int32_t *rank);

/*
 * Parents (ranks) of the entries pll_export_weighted gives for `side`, in
 * the same order, for a weighted index built with PLL_PARENTS (else
 * PLL_E_UNSUPPORTED): for (h, d) in L(v) (L_IN(v)) an edge p -> v with
 * d(h, p) + w(p, v) = d, for L_OUT(v) an arc v -> p with w(v, p) + d(p, h)
 * = d; v itself for d = 0.  par: host uint32[entries].
 */
int pll_export_weighted_parents(const pll_index *idx, int32_t side, uint32_t *par);

/*
 * Work counters of the build (PLL_STAT_* below), for reporting and for the
 * algorithmic-byte model.  Copies min(ncounters, PLL_NSTATS) values.  For a
 * weighted build: VISITED counts frontier entries processed by the search
 * steps (an entry is processed again each time its distance drops), LEVELS
 * the steps, EDGES the edges relaxed, NORMAL_TESTS / LABEL_SCANNED the prune
 * tests, LEVEL_LAUNCHES / LEVEL_NS the step kernels; the bit-parallel and
 * task counters stay 0.
 */
enum {
  PLL_STAT_N = 0,        /* vertices */
  PLL_STAT_TBP,          /* bit-parallel slots */
  PLL_STAT_ENTRIES,      /* normal label entries, no sentinels */
  PLL_STAT_BP_USED,      /* vertices used as bit-parallel roots or neighbours */
  PLL_STAT_ROOTS,        /* pruned BFSs run */
  PLL_STAT_VISITED,      /* (root, vertex) visits of the pruned phase (entries
                            of the BFS levels, each tested once) */
  PLL_STAT_CANDIDATES,   /* labels appended before cleaning */
  PLL_STAT_WINDOWS,      /* root windows */
  PLL_STAT_RETRIES,      /* windows re-run smaller after overflow */
  PLL_STAT_BP_VISITED,   /* (slot, vertex) visits of the bit-parallel phase */
  PLL_STAT_LEVELS,       /* level kernels launched */
  PLL_STAT_INDEX_BYTES,  /* device bytes of the finished index */
  PLL_STAT_BUILD_NS,     /* wall time of the build, ns */
  PLL_STAT_BP_NS,        /* bit-parallel phase, ns */
  PLL_STAT_PRUNED_NS,    /* pruned phase, ns */
  PLL_STAT_NORMAL_TESTS, /* visits that reached the normal-label test */
  PLL_STAT_LABEL_SCANNED,/* label entries read by normal-label tests */
  PLL_STAT_EDGES,        /* adjacency entries expanded by the level kernel */
  PLL_STAT_TASK_EDGES,   /* adjacency entries expanded as long-list tasks */
  PLL_STAT_LEVEL_LAUNCHES, /* launches of the pruned-phase level kernel */
  PLL_STAT_LEVEL_NS,     /* their summed duration from HIP events, ns; only
                            with the "profile" knob set, else 0 */
  PLL_STAT_BP_DIRECT,    /* adjacency entries whose neighbour bit-parallel
                            distances alone prune at the next level; it is not
                            visited through them (counted per edge) */
  PLL_STAT_BP_SETS,      /* visits whose bit-parallel test read slot sets */
  PLL_STAT_BP_CHECKS,    /* slot set pairs read by those tests */
  PLL_STAT_IMPROVED,     /* weighted builds: tentative distances lowered */
  PLL_STAT_TOUCHED,      /* weighted builds: (root, vertex) entries reached */
  PLL_STAT_FILTERED,     /* weighted builds: relaxations skipped because
                            distances through 16 exact landmark hubs already
                            prune the vertex at the new distance */
  PLL_STAT_LAND_CHECKS,  /* weighted builds: relaxations checked that way */
  PLL_STAT_EARLIER_ROOT, /* unweighted builds: adjacency entries that lead to
                            a vertex ranked before the window: an earlier root
                            (or bit-parallel vertex), whose committed labels
                            already give its exact distance from every later
                            root (Section 4.2), so its test would prune it; it
                            is left unvisited without one (counted per edge;
                            weighted builds leave this to the landmark bound,
                            which already stops these relaxations) */
  PLL_STAT_EXPAND_NS,    /* summed duration of the expansion kernel
                            (k_win_expand, lists up to "chunk" entries) from
                            HIP events, ns; only with the "profile" knob */
  PLL_STAT_EXPAND_DIRECT,  /* PLL_STAT_BP_DIRECT's share of that kernel */
  PLL_STAT_EXPAND_EARLIER, /* PLL_STAT_EARLIER_ROOT's share of that kernel */
  PLL_STAT_EXPAND_CLAIMS,  /* neighbours that kernel claimed for the next level */
  PLL_STAT_WHOLE_GRAPHS,   /* graphs of a batch whose pruned phase ran whole in
                              one workgroup (see pll_build_batch) */
  PLL_STAT_WHOLE_NS,       /* wall time of that launch, ns (with any re-run
                              after the label pool ran out) */
  PLL_STAT_WHOLE_PAIRS,    /* query pairs that launch answered
                              (pll_build_query_batch) */
  PLL_NSTATS
};
int pll_stats(const pll_index *idx, int32_t graph, int64_t *counters, int32_t ncounters);

/*
 * Per-level profile of the pruned phase, recorded only when the "profile"
 * tuning knob was set during the build (else there are no rows).  Each row
 * has PLL_TRACE_COLS values: window index, first root rank of the window,
 * roots in the window, BFS level d, (root, vertex) entries at level d,
 * candidate labels made at level d, and the duration in ns of the level's
 * kernels (HIP events on the build stream).  Copies up to max_rows rows
 * into rows (row-major) and returns the total number of rows, or
 * PLL_E_INVAL.
 */
#define PLL_TRACE_COLS 7
int64_t pll_level_trace(const pll_index *idx, int64_t *rows, int64_t max_rows);

/* Release the index and all its device memory.  NULL is ignored. */
void pll_free(pll_index *idx);

/* Static description of an error code. */
const char *pll_strerror(int code);

/*
 * Serving: continuous batching of query requests over a device-resident
 * index (the index must outlive the server).
 *
 * pll_server_start: a worker thread with nslots (1..32) slots, each a HIP
 *   stream with pinned staging for slot_pairs pairs.  Requests queue FIFO;
 *   each free slot takes the oldest requests that fit, so requests arriving
 *   while others run on the GPU are admitted as slots free up and run
 *   concurrently with them.  Every request gets exactly the answers
 *   pll_query would give it alone.
 *   On a weighted index (pll_build_weighted) the answers are pll_query_
 *   weighted's 32-bit distances.
 * pll_server_submit: queue q (>= 1) pairs from host memory; the answers go
 *   to out[q] (host).  A request of more than slot_pairs pairs is queued as
 *   consecutive parts of slot_pairs pairs (the last one shorter), each
 *   dispatched like a request; it is done when its last part is.  The caller keeps pairs and out alive until
 *   the request is done.  *ticket identifies the request.  Ids are checked
 *   on submission (PLL_E_INVAL).  PLL_E_UNSUPPORTED on a server of a
 *   weighted index.
 * pll_server_submit_weighted: the same for a server of a weighted index,
 *   answers as uint32 (PLL_WINF = unreachable); PLL_E_UNSUPPORTED on a
 *   server of an unweighted index.
 * pll_server_done: 1 if the request is answered (optionally waiting), 0 if
 *   not yet; *latency_us = answer time - submission time.  Once it has
 *   returned 1 the request's record is recycled and the ticket is no longer
 *   valid (PLL_E_INVAL), so a ticket is waited for by one thread; the
 *   server's host memory stays bounded by the requests in flight.
 * pll_server_stop: answer everything queued, stop the worker, free the
 *   server.  stats (optional, up to 7): launches, pairs launched, max queue
 *   length, the longest launch in ns (from its dispatch to the worker seeing
 *   its completion event), its number among the launches, the longest
 *   pause in ns between two passes of the worker while it had work, and the
 *   request records ever allocated (records are recycled).
 * pll_serve_bench: open-loop load test in native code: nreq requests of
 *   log-uniform size in [1, max_batch] with uniform random pairs, Poisson
 *   arrivals at `rate` requests/s (rate <= 0: all at once = saturation),
 *   SplitMix64 randomness from seed.  stats[12]: p50 / p99 / mean latency
 *   in us (from the scheduled arrival, so queueing counts), pairs/s,
 *   requests/s, seconds, launches, mean pairs per launch, max queue length,
 *   the longest launch in us, its launch number and the worker's longest
 *   pause in us.
 */
typedef struct pll_server pll_server;
int pll_server_start(const pll_index *idx, int32_t nslots, int64_t slot_pairs, pll_server **out);
int pll_server_submit(pll_server *srv, const int32_t *pairs, int64_t q, uint8_t *out,
                      int64_t *ticket);
int pll_server_submit_weighted(pll_server *srv, const int32_t *pairs, int64_t q, uint32_t *out,
                               int64_t *ticket);
int pll_server_done(pll_server *srv, int64_t ticket, int32_t wait, double *latency_us);
int pll_server_stop(pll_server *srv, int64_t *stats, int32_t nstats);
int pll_serve_bench(const pll_index *idx, double rate, int64_t nreq, int64_t max_batch,
                    uint64_t seed, int32_t nslots, int64_t slot_pairs, double *stats,
                    int32_t nstats);

/*
 * Tuning knobs (process-wide), each a power of two where it is a lane
 * count.  Pruned phase: "window" (most concurrent roots, 1..16384),
 * "window_work" (visits aimed at per window: the window grows or shrinks
 * toward it after each window; 0 keeps every window at the maximum),
 * "window_mem_mb" (device memory the per-root window state may take, about
 * 1.4 n bytes per root, twice that for a directed graph; default 65536,
 * and never more than the device's free memory less a fifth of the device
 * (at least 8 GB) kept for the label pool and lists), "group" (lanes per frontier
 * entry in the prune tests: 4..64, or 0 (default): chosen per window from
 * the label entries a test scanned in the window before), "root_sort" (0:
 * prune tests straight from the frontier, the root's label through a table
 * in global memory; 1: each level's entries grouped by root first, every
 * root's label table and bit-parallel row staged in LDS; 2 (default): 1 for
 * windows after one that averaged at least "sort_level" (default 2^20)
 * visits or "sort_scan" (default 2^23) scanned label entries per level,
 * else 0; same labels), "xgroup" (lanes per candidate expanding
 * its adjacency list: 4..64, default 8), "list_cap" (upper bound on the entries of
 * the frontier, candidate and task lists, never below what one root needs;
 * 0 = sized from the window; a window that overflows is re-run with a
 * quarter of the roots), "table_cap" (first size of the root-table area in
 * entries; 0 = sized from the window; it grows when a window needs more),
 * "chunk" (edges a group expands inline before
 * handing the rest to whole waves), "levels_per_sync" (levels launched
 * between host checks), "profile" (0/1: time every level with HIP events on
 * the build stream).  Weighted builds: "wgroup" (lanes per frontier entry
 * of a search step: 4..64), "wwork" ((root, vertex) entries a window aims
 * to reach: the window grows or shrinks toward it; 0 keeps every window
 * after the first at the maximum), and "window", "window_mem_mb", "list_cap",
 * "table_cap", "levels_per_sync" (steps between host checks) and "profile"
 * as above.  Bit-parallel phase: "bp_chunk" (adjacency entries per
 * work item).  Batches: "whole_n" (graphs of up to this many vertices,
 * 0..16384, default 4096, are built one workgroup per graph; 0 never) and
 * "whole_pool" (label pool entries first reserved per vertex of those
 * graphs, default 256; the launch is redone with twice the pool if it runs
 * out; same labels).  "landmarks" (0/1: builds without bit-parallel labels --
 * t_bp = 0, directed, weighted -- keep exact distances from their first 16
 * roots and skip expansions those already prune; the labels do not
 * change).  "live_adjacency" (0/1: each time the window start s has
 * doubled, the expansion's adjacency (a weighted build's relaxation
 * adjacency, weights included) is rebuilt without the neighbours ranked
 * below s, which would be pruned anyway; same labels).  "expand_prune"
 * (0/1, unweighted builds: a candidate's expansion leaves a neighbour
 * unvisited when the neighbour ranks before the window or its distance row
 * already prunes it at the next level; 0 visits and tests every reached
 * neighbour as Algorithm 1 does, and also turns "live_adjacency" and the
 * landmark rows off, so that a PLL_PLAIN build's visits, labels and
 * scanned edges are the sequential algorithm's; same labels).
 * "packed_rows" (0/1, default 1: with t_bp giving rows of 32 or 64 slots,
 * the expansion's prune reads 4-bit copies of the reached vertices'
 * bit-parallel distance rows, distances of 15 or more counting as none;
 * same labels).  Memory: "pool_keep_mb" (device memory of freed build
 * scratch and indexes kept for reuse by later builds, MB; reuse on another
 * stream waits for the stream that freed it; lowering the value releases
 * the excess at once, 0 keeps nothing).  Queries: "qgroup" (lanes per pair: 16, 32, 64), "qpersist" (0/1: batched queries with
 * a static pair-to-group assignment, or persistent groups that take chunks
 * of pairs from a shared cursor; pll_autotune_query chooses both),
 * "serve_coalesce" (0/1: servers started afterwards launch one request at a
 * time / pack several).  Returns PLL_E_INVAL for an unknown key or value.
 */
int pll_set_tuning(const char *key, int64_t value);
int64_t pll_get_tuning(const char *key);

#ifdef __cplusplus
}
#endif
#endif /* PLL_H_ */
