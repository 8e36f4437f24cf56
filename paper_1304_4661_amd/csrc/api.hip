// Host side of the C ABI (include/pll.h): argument validation, device
// memory, the level loops of both BFS phases, the root-window loop of the
// pruned phase, finalisation, queries, export and statistics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "pll_internal.h"

using namespace pll;

namespace {

struct Tuning {
  int window = 16384;  // most concurrent roots of the pruned phase
  int64_t window_work = 128000000;  // visits aimed at per window (0: fixed size)
  int64_t window_mem_mb = 65536;  // device memory allowed for per-root state
  int64_t list_cap = 0;   // cap on frontier / candidate / task lists (0: sized from W)
  int64_t table_cap = 0;  // first size of the root-table area (0: sized from W)
  int group = 0;      // lanes per frontier entry (prune tests; 0: chosen per window)
  int xgroup = 8;     // lanes per candidate expanding its adjacency list
  int wgroup = 64;    // lanes per frontier entry of a weighted search step
  int64_t wwork = 2000000;  // touched entries aimed at per weighted window
  int64_t pool_keep_mb = 16384;  // freed device memory kept for reuse by later builds
  int landmarks = 1;  // landmark rows for builds without bit-parallel labels
  int live_adjacency = 1;  // drop neighbours ranked below the window from the expansion's CSR
  int chunk = 256;    // edges expanded inline before splitting into tasks
  int qgroup = 64;    // lanes per query pair
  int qpersist = 0;   // batched queries: 1 = persistent groups taking chunks from a cursor
  int levels_per_sync = 4;
  int profile = 0;
  int bp_chunk = 64;  // adjacency entries per bit-parallel work item
  int serve_coalesce = 1;  // servers pack several requests per launch
  int expand_prune = 1;  // expansion leaves neighbours unvisited that a test would prune
  int root_sort = 2;  // prune tests grouped by root: 0 never, 1 always, 2 for large levels
  int64_t sort_level = 1 << 20;  // visits per level from which "root_sort" 2 groups by root
  int64_t sort_scan = 8 << 20;   // ... or label entries scanned per level
  int64_t whole_n = 4096;  // batch graphs of at most this many vertices are built
                           // whole, one workgroup each (0: never; at most kGMaxN)
  int64_t whole_pool = 256;  // label pool entries reserved per vertex of those graphs
  int packed_rows = 1;  // the expansion reads 4-bit copies of the distance rows
};
Tuning g_tune;
std::mutex g_tune_mu;

Tuning tuning() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return g_tune;
}

// Thrown internally, turned into a return code at the ABI boundary.
struct Fail {
  int code;
};

void check(hipError_t e) {
  if (e == hipErrorOutOfMemory) throw Fail{PLL_E_NOMEM};
  if (e != hipSuccess) throw Fail{PLL_E_DEVICE};
}

// Owning device buffer.
// Device memory of builds and indexes: hipMalloc, or a caller's allocator
// (pll_set_allocator), which receives the stream of the build so that a
// stream-ordered allocator can reuse memory safely.
struct AllocHook {
  void *(*alloc)(size_t, void *, void *) = nullptr;
  void (*free_)(void *, void *, void *) = nullptr;
  void *ctx = nullptr;
};
AllocHook g_alloc_hook;
std::mutex g_alloc_mu;
thread_local hipStream_t t_alloc_stream = nullptr;

AllocHook alloc_hook() {
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  return g_alloc_hook;
}

// Sets the stream passed to the allocator for this thread's allocations.
struct AllocStream {
  hipStream_t old;
  explicit AllocStream(hipStream_t s) : old(t_alloc_stream) { t_alloc_stream = s; }
  ~AllocStream() { t_alloc_stream = old; }
};

// Default device allocations go through a small cache of freed blocks: a
// build allocates and frees the same multi-GB scratch every time, and
// hipMalloc/hipFree (or the stream-ordered pool's free) cost milliseconds
// per build.  A freed block is kept (up to "pool_keep_mb" in total) with an
// event recorded on the stream it was released on; a later allocation of
// the same rounded size takes it and, on another stream, waits for that
// event first, so reuse is stream-ordered.
struct CachedBlock {
  void *p;
  int dev;
  hipEvent_t ev;
  hipStream_t stream;
};
struct BlockCache {
  std::mutex mu;
  std::multimap<size_t, CachedBlock> blocks;  // by rounded size
  size_t total = 0;
};
BlockCache g_blocks;

size_t round_bytes(size_t b) {
  const size_t mb = (size_t)1 << 20;
  return b <= mb ? ((b + 255) & ~(size_t)255) : ((b + mb - 1) & ~(mb - 1));
}

// Free every cached block (all devices) beyond `keep` bytes.
void cache_trim(size_t keep) {
  std::vector<CachedBlock> drop;
  {
    std::lock_guard<std::mutex> lk(g_blocks.mu);
    while (g_blocks.total > keep && !g_blocks.blocks.empty()) {
      auto it = std::prev(g_blocks.blocks.end());  // largest first
      g_blocks.total -= it->first;
      drop.push_back(it->second);
      g_blocks.blocks.erase(it);
    }
  }
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (auto &b : drop) {
    (void)hipSetDevice(b.dev);
    (void)hipEventSynchronize(b.ev);
    (void)hipEventDestroy(b.ev);
    (void)hipFree(b.p);
  }
  (void)hipSetDevice(cur);
}

hipError_t cache_alloc(void **p, size_t bytes, hipStream_t st) {
  const size_t rb = round_bytes(bytes);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  {
    std::lock_guard<std::mutex> lk(g_blocks.mu);
    auto range = g_blocks.blocks.equal_range(rb);
    for (auto it = range.first; it != range.second; ++it) {
      if (it->second.dev != dev) continue;
      CachedBlock b = it->second;
      g_blocks.blocks.erase(it);
      g_blocks.total -= rb;
      if (b.stream != st) e = hipStreamWaitEvent(st, b.ev, 0);
      (void)hipEventDestroy(b.ev);
      if (e != hipSuccess) {
        (void)hipFree(b.p);
        return e;
      }
      *p = b.p;
      return hipSuccess;
    }
  }
  e = hipMalloc(p, rb);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    cache_trim(0);  // give the cached blocks back and try once more
    e = hipMalloc(p, rb);
  }
  return e;
}

void cache_free(void *p, size_t bytes, hipStream_t st) {
  const size_t rb = round_bytes(bytes);
  const size_t keep = (size_t)tuning().pool_keep_mb << 20;
  int dev = 0;
  hipEvent_t ev = nullptr;
  if (rb <= keep && hipGetDevice(&dev) == hipSuccess &&
      hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess) {
    if (hipEventRecord(ev, st) == hipSuccess) {
      std::lock_guard<std::mutex> lk(g_blocks.mu);
      g_blocks.blocks.emplace(rb, CachedBlock{p, dev, ev, st});
      g_blocks.total += rb;
      if (g_blocks.total <= keep) return;
    } else {
      (void)hipEventDestroy(ev);
      ev = nullptr;
      (void)hipGetLastError();
      (void)hipStreamSynchronize(st);
      (void)hipFree(p);
      return;
    }
    cache_trim(keep);  // over the limit: drop the largest blocks
    return;
  }
  (void)hipGetLastError();
  (void)hipStreamSynchronize(st);
  (void)hipFree(p);
}

template <typename T>
struct DBuf {
  T *p = nullptr;
  size_t count = 0;
  AllocHook hook;                // allocator the memory came from
  hipStream_t stream = nullptr;  // stream it was allocated for
  DBuf() = default;
  explicit DBuf(size_t c) { alloc(c); }
  DBuf(const DBuf &) = delete;
  DBuf &operator=(const DBuf &) = delete;
  DBuf(DBuf &&o) noexcept : p(o.p), count(o.count), hook(o.hook), stream(o.stream) {
    o.p = nullptr;
    o.count = 0;
  }
  DBuf &operator=(DBuf &&o) noexcept {
    if (this != &o) {
      reset();
      p = o.p;
      count = o.count;
      hook = o.hook;
      stream = o.stream;
      o.p = nullptr;
      o.count = 0;
    }
    return *this;
  }
  void alloc(size_t c) {
    reset();
    const size_t bytes = std::max<size_t>(c * sizeof(T), 1);
    hook = alloc_hook();
    stream = t_alloc_stream;
    if (hook.alloc) {
      p = static_cast<T *>(hook.alloc(bytes, (void *)stream, hook.ctx));
      if (!p) throw Fail{PLL_E_NOMEM};
    } else {
      hipError_t e = cache_alloc((void **)&p, bytes, stream);
      if (e != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
        throw Fail{e == hipErrorOutOfMemory ? PLL_E_NOMEM : PLL_E_DEVICE};
      }
    }
    count = c;
  }
  void reset() {
    if (p) {
      if (hook.alloc)
        hook.free_(p, (void *)stream, hook.ctx);
      else
        cache_free(p, std::max<size_t>(count * sizeof(T), 1), stream);
    }
    p = nullptr;
    count = 0;
  }
  ~DBuf() { reset(); }
  size_t bytes() const { return count * sizeof(T); }
};

template <typename T>
void h2d(T *dst, const T *src, size_t count, hipStream_t st) {
  if (count) check(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyHostToDevice, st));
}
template <typename T>
void d2h(T *dst, const T *src, size_t count, hipStream_t st) {
  if (count) check(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyDeviceToHost, st));
}
template <typename T>
void fill(DBuf<T> &b, int byte, hipStream_t st) {
  if (b.count) check(hipMemsetAsync(b.p, byte, b.bytes(), st));
}

using Clock = std::chrono::steady_clock;
int64_t ns_since(Clock::time_point t0) {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now() - t0).count();
}

}  // namespace

// ---------------------------------------------------------------------------

struct pll_index {
  int32_t n = 0, t = 0, tpad = 0;
  // graphs of a batch (one for pll_build): graph g owns ids
  // [vtx_off[g], vtx_off[g+1]); its vertex of local rank l has global rank
  // grank(g, l): gblk[g] + l for a graph built whole by one workgroup (a
  // block of consecutive ranks after the interleaved ones), else
  // lbase[l] + gpos[g]
  int32_t G = 1;
  std::vector<int64_t> vtx_off, lbase, g_entries, gblk;
  std::vector<int32_t> gpos;
  int64_t grank(int32_t g, int64_t l) const {
    return gblk[g] >= 0 ? gblk[g] + l : lbase[l] + gpos[g];
  }
  std::vector<int32_t> lrank_h;  // local rank of every global rank (host copy)
  std::vector<int64_t> hoff;     // host copy of off
  DBuf<int32_t> rgid;   // graph of every global rank (batches only)
  DBuf<int32_t> lrank;  // local rank of every global rank
  DBuf<int32_t> rank;   // id -> rank
  DBuf<uint8_t> bpd;    // [n][tpad], padding 255
  DBuf<uint64_t> bpm;   // [n][t][2] (S^{-1}, S^{0}) pairs
  DBuf<int64_t> off;   // [n+1], sentinel-inclusive CSR
  DBuf<uint32_t> hub;
  DBuf<uint8_t> dist;
  DBuf<int32_t> err;  // sticky error of asynchronous device-pointer queries
  // kept by builds with PLL_PARENTS: parents (layout of hub), the
  // rank-space graph and rank -> id, for path queries
  bool parents = false;
  DBuf<uint32_t> par;
  // a directed graph (PLL_DIRECTED): off/hub/dist hold L_OUT, these L_IN
  // (ipar: parents of the L_IN entries)
  bool directed = false;
  DBuf<int64_t> ioff;
  DBuf<uint32_t> ihub, ipar;
  DBuf<uint8_t> idist;
  DBuf<int64_t> grow;
  DBuf<int32_t> gcol;
  DBuf<int32_t> ord;
  // a weighted graph (pll_build_weighted): labels as packed entries
  // hub << 32 | distance at off (L, or L_OUT of a digraph) and ioff (L_IN)
  bool weighted = false;
  DBuf<uint64_t> went, iwent;
  int64_t entries = 0;
  int64_t stats[PLL_NSTATS] = {};
  std::vector<int64_t> level_trace;  // pruned-phase levels, PLL_TRACE_COLS per row
  std::vector<int32_t> bp_root, bp_nsel, bp_sel;  // per slot record (graph * t + slot)

  // The index outlives the stream it was built on: its memory is released
  // in order on the null stream (pll_free requires no pending work on it).
  void detach_streams() {
    for (auto *b : {&rgid, &lrank, &rank, &err, &gcol, &ord})
      if (!b->hook.alloc) b->stream = nullptr;
    for (auto *b : {&bpd, &dist, &idist})
      if (!b->hook.alloc) b->stream = nullptr;
    for (auto *b : {&bpm, &went, &iwent})
      if (!b->hook.alloc) b->stream = nullptr;
    for (auto *b : {&off, &ioff, &grow})
      if (!b->hook.alloc) b->stream = nullptr;
    for (auto *b : {&hub, &par, &ihub, &ipar})
      if (!b->hook.alloc) b->stream = nullptr;
  }

  DIndex view() const {
    DIndex v;
    v.n = n;
    v.t = t;
    v.tpad = tpad;
    v.rank = rank.p;
    v.rgid = G > 1 ? rgid.p : nullptr;
    v.bpd = bpd.p;
    v.bpm = bpm.p;
    v.off = off.p;
    v.hub = hub.p;
    v.dist = dist.p;
    v.toff = directed ? ioff.p : off.p;
    v.thub = directed ? ihub.p : hub.p;
    v.tdist = directed ? idist.p : dist.p;
    v.par = par.p;
    v.tpar = directed ? ipar.p : par.p;
    v.grow = grow.p;
    v.gcol = gcol.p;
    v.ord = ord.p;
    v.went = went.p;
    v.twent = directed ? iwent.p : went.p;
    return v;
  }
};

namespace {

// ---------------------------------------------------------------------------
// Validation (before any device work).

// A batch of G graphs packed into one CSR with global ids: graph g owns ids
// [vtx_off[g], vtx_off[g+1]) and its edges stay inside that range; order
// holds each graph's local order (local ranks -> local ids) at the graph's
// offsets.  A single graph is G = 1, vtx_off = {0, n}.
int validate_batch(int32_t G, const int64_t *vtx_off, const int32_t *row_ptr, const int32_t *col,
                   const int32_t *order, int32_t t_bp, bool symmetric) {
  if (G < 0 || t_bp < 0 || t_bp > PLL_MAX_TBP || (G > 0 && !vtx_off)) return PLL_E_INVAL;
  if (G == 0) return PLL_OK;
  if (vtx_off[0] != 0) return PLL_E_INVAL;
  for (int32_t g = 0; g < G; g++)
    if (vtx_off[g + 1] < vtx_off[g]) return PLL_E_INVAL;
  const int64_t N = vtx_off[G];
  if (N > INT32_MAX - 1) return PLL_E_INVAL;
  if (N == 0) return PLL_OK;
  if (!row_ptr || !order) return PLL_E_INVAL;
  if (row_ptr[0] != 0) return PLL_E_INVAL;
  for (int64_t v = 0; v < N; v++)
    if (row_ptr[v + 1] < row_ptr[v]) return PLL_E_INVAL;
  const int64_t nnz = row_ptr[N];
  if (nnz > 0 && !col) return PLL_E_INVAL;
  std::vector<char> seen((size_t)N, 0);
  for (int32_t g = 0; g < G; g++) {
    const int64_t lo = vtx_off[g], hi = vtx_off[g + 1];
    for (int64_t v = lo; v < hi; v++) {
      for (int32_t j = row_ptr[v]; j < row_ptr[v + 1]; j++)
        if (col[j] < lo || col[j] >= hi || col[j] == v) return PLL_E_INVAL;
      const int32_t o = order[v];
      if (o < 0 || o >= hi - lo || seen[lo + o]) return PLL_E_INVAL;
      seen[lo + o] = 1;
    }
  }
  if (symmetric) {
    std::vector<int32_t> sorted(col, col + nnz);
    for (int64_t v = 0; v < N; v++)
      std::sort(sorted.begin() + row_ptr[v], sorted.begin() + row_ptr[v + 1]);
    for (int64_t v = 0; v < N; v++)
      for (int32_t j = row_ptr[v]; j < row_ptr[v + 1]; j++) {
        const int32_t w = sorted[j];
        if (!std::binary_search(sorted.begin() + row_ptr[w], sorted.begin() + row_ptr[w + 1],
                                (int32_t)v))
          return PLL_E_INVAL;
      }
  }
  return PLL_OK;
}

// Interleaving of a batch's graphs by local rank: graphs sorted by
// decreasing size (ties by index) get positions gpos; lbase[l] = number of
// vertices of local rank < l over all graphs.  Then global rank
// lbase[l] + gpos[g] is a bijection, and restricted to one graph it is that
// graph's own order, so the union's labels are each graph's labels.  It also
// puts every graph's early (heavy) roots in the same windows, where roots of
// different graphs never interact.
//
// Graphs listed in `whole` (built by one workgroup each, largest first)
// take no part in the interleaving: they get blocks of consecutive ranks
// after it, in list order (gblk[g] = first rank, -1 for the others), which
// keeps each graph's order just the same.  Returns the interleaved ranks'
// count (the windows' range).
int64_t interleave(int32_t G, const std::vector<int64_t> &vtx_off,
                   const std::vector<int32_t> &whole, std::vector<int32_t> &gpos,
                   std::vector<int64_t> &lbase, std::vector<int64_t> &gblk) {
  auto size = [&](int32_t g) { return vtx_off[g + 1] - vtx_off[g]; };
  gblk.assign((size_t)G, -1);
  for (int32_t g : whole) gblk[g] = 0;
  std::vector<int32_t> idx;
  for (int32_t g = 0; g < G; g++)
    if (gblk[g] < 0) idx.push_back(g);
  std::stable_sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) { return size(a) > size(b); });
  gpos.assign((size_t)G, 0);
  const int32_t K = (int32_t)idx.size();
  for (int32_t i = 0; i < K; i++) gpos[idx[i]] = i;
  const int64_t maxn = K ? size(idx[0]) : 0;
  lbase.assign((size_t)maxn + 1, 0);
  // graphs with size > l form the prefix idx[0 .. cnt) of the size order
  int32_t cnt = K;
  for (int64_t l = 0; l < maxn; l++) {
    while (cnt > 0 && size(idx[cnt - 1]) <= l) cnt--;
    lbase[l + 1] = lbase[l] + cnt;
  }
  int64_t next = lbase[maxn];
  for (int32_t g : whole) {
    gblk[g] = next;
    next += size(g);
  }
  return lbase[maxn];
}

// Graphs of a batch built whole by one workgroup each: those of 1 ..
// min(limit, kGMaxN) vertices, largest first (ties by index).  None for a
// single graph, a directed batch or the plain form.
std::vector<int32_t> whole_graphs(int32_t G, const std::vector<int64_t> &vtx_off, int64_t limit) {
  std::vector<int32_t> w;
  if (G < 2) return w;
  const int64_t lim = std::min<int64_t>(limit, kGMaxN);
  for (int32_t g = 0; g < G; g++) {
    const int64_t ng = vtx_off[g + 1] - vtx_off[g];
    if (ng >= 1 && ng <= lim) w.push_back(g);
  }
  std::stable_sort(w.begin(), w.end(), [&](int32_t a, int32_t b) {
    return vtx_off[a + 1] - vtx_off[a] > vtx_off[b + 1] - vtx_off[b];
  });
  return w;
}

// Reads a LevelCtl back to the host (synchronising the stream).
// Pinned host mirror of the level control block and the pool top, read back
// together with one synchronisation per batch of levels.
struct CtlMirror {
  LevelCtl ctl;
  unsigned long long top;
};
// Pinned host blocks are recycled across builds: hipHostMalloc/hipHostFree
// cost milliseconds each, a build needs only a few small ones.
template <typename T>
struct PinnedPool {
  std::mutex mu;
  std::vector<T *> free_list;
  T *get() {
    {
      std::lock_guard<std::mutex> lk(mu);
      if (!free_list.empty()) {
        T *p = free_list.back();
        free_list.pop_back();
        return p;
      }
    }
    T *p = nullptr;
    if (hipHostMalloc((void **)&p, sizeof(T), hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      throw Fail{PLL_E_NOMEM};
    }
    return p;
  }
  void put(T *p) {
    std::lock_guard<std::mutex> lk(mu);
    free_list.push_back(p);
  }
};
PinnedPool<CtlMirror> g_ctl_pinned;

struct PinnedMirror {
  CtlMirror *p = nullptr;
  PinnedMirror() { p = g_ctl_pinned.get(); }
  ~PinnedMirror() {
    if (p) g_ctl_pinned.put(p);
  }
  PinnedMirror(const PinnedMirror &) = delete;
  PinnedMirror &operator=(const PinnedMirror &) = delete;
};

constexpr size_t kTraceCols = PLL_TRACE_COLS;

// ---------------------------------------------------------------------------
// The build of one graph, in rank space, into `ix`.

struct Builder {
  hipStream_t st;
  Tuning tu;
  bool plain = false;
  bool parents = false;  // keep the BFS-tree parent of every label entry
  int32_t n, t, nwords;
  int64_t nnz;
  DBuf<int64_t> row;
  DBuf<int32_t> col;
  DBuf<uint8_t> used;
  int64_t stat_levels = 0, stat_bp_visited = 0, stat_visited = 0, stat_cand = 0,
          stat_windows = 0, stat_retries = 0, stat_roots = 0, stat_tests = 0, stat_scanned = 0,
          stat_edges = 0, stat_hedges = 0, stat_level_launches = 0, stat_level_ns = 0,
          stat_bp_direct = 0, stat_bp_sets = 0, stat_bp_checks = 0, stat_earlier = 0,
          stat_expand_ns = 0, stat_x_direct = 0, stat_x_earlier = 0, stat_x_claims = 0;
  // with the "profile" knob: one row per level, kTraceCols values each
  std::vector<int64_t> level_trace;
  size_t trace_mark = 0;

  DGraph graph() const { return DGraph{n, nwords, row.p, col.p}; }

  // a1: global ranks (interleaved graphs; for one graph rank[order[i]] = i)
  // and the rank-space CSR.  Inputs are host arrays, or device arrays
  // (already validated) when `device` is set.
  int32_t G = 1;
  std::vector<int64_t> vtx_off;
  DBuf<int64_t> d_vtx_off, d_lbase, d_gblk;
  DBuf<int32_t> d_gpos;
  // graphs built whole by one workgroup each (largest first) and the
  // interleaved ranks' count: the windows run roots [0, nwin)
  std::vector<int32_t> whole;
  int64_t nwin = 0;
  // query pairs answered by the whole-graph launch (pll_build_query_batch):
  // graph g's pairs at qpairs[2 qoff[g] ..), answers at qout[qoff[g] ..)
  // (device memory); qpairs null: none
  const int32_t *qpairs = nullptr;
  uint8_t *qout = nullptr;
  std::vector<int64_t> qoff;
  int64_t stat_whole_pairs = 0;

  const int32_t *rank_p = nullptr;  // id -> rank (the index's array)
  void relabel(const int32_t *in_row_p, const int32_t *in_col_p, const int32_t *order_p,
               bool device, pll_index *ix, DBuf<int32_t> *gid_in) {
    DBuf<int32_t> in_row, in_col, order;
    if (!device) {
      in_row.alloc((size_t)n + 1);
      in_col.alloc((size_t)std::max<int64_t>(nnz, 1));
      order.alloc((size_t)n);
      h2d(in_row.p, in_row_p, (size_t)n + 1, st);
      h2d(in_col.p, in_col_p, (size_t)nnz, st);
      h2d(order.p, order_p, (size_t)n, st);
      in_row_p = in_row.p;
      in_col_p = in_col.p;
      order_p = order.p;
    }
    if (!plain && !directed && tu.whole_n > 0) whole = whole_graphs(G, vtx_off, tu.whole_n);
    nwin = interleave(G, vtx_off, whole, ix->gpos, ix->lbase, ix->gblk);
    ix->G = G;
    ix->vtx_off = vtx_off;
    if (!d_vtx_off.p) {
      d_vtx_off.alloc((size_t)G + 1);
      h2d(d_vtx_off.p, vtx_off.data(), (size_t)G + 1, st);
    }
    d_lbase.alloc(ix->lbase.size());
    d_gpos.alloc((size_t)std::max(G, 1));
    d_gblk.alloc((size_t)std::max(G, 1));
    h2d(d_lbase.p, ix->lbase.data(), ix->lbase.size(), st);
    h2d(d_gpos.p, ix->gpos.data(), (size_t)G, st);
    h2d(d_gblk.p, ix->gblk.data(), (size_t)G, st);
    DBuf<int32_t> gid_own;
    DBuf<int32_t> *gid = gid_in;
    if (!gid || !gid->p) {
      gid_own.alloc((size_t)std::max(n, 1));
      check(launch_fill_gid(d_vtx_off.p, G, gid_own.p, st));
      gid = &gid_own;
    }
    ix->rank.alloc((size_t)n);
    rank_p = ix->rank.p;
    ix->lrank.alloc((size_t)n);
    ix->rgid.alloc((size_t)n);
    DBuf<int32_t> gorder((size_t)n);
    check(launch_batch_rank(n, gid->p, d_vtx_off.p, order_p, d_lbase.p, d_gpos.p, d_gblk.p,
                            ix->rank.p,
                            gorder.p, ix->lrank.p, ix->rgid.p, st));
    DBuf<int64_t> deg((size_t)n), tmp((size_t)scan_tmp_elems(n));
    row.alloc((size_t)n + 1);
    col.alloc((size_t)std::max<int64_t>(nnz, 1));
    check(launch_degrees(in_row_p, gorder.p, deg.p, n, st));
    check(launch_exclusive_scan(deg.p, row.p, n, tmp.p, st));
    check(launch_relabel_cols(in_row_p, in_col_p, gorder.p, ix->rank.p, row.p, col.p, n, st));
    ix->lrank_h.resize((size_t)n);
    d2h(ix->lrank_h.data(), ix->lrank.p, (size_t)n, st);
    check(hipStreamSynchronize(st));
  }

  // a2 + a3: bit-parallel roots and BFSs
  void bit_parallel(pll_index *ix) {
    used.alloc((size_t)n);
    fill(used, 0, st);
    const int32_t tpad = bp_pad(t);
    ix->tpad = tpad;
    ix->bpd.alloc((size_t)n * tpad);
    ix->bpm.alloc((size_t)n * t * 2);
    const size_t nrec = (size_t)G * t;  // slot records: graph * t + slot
    ix->bp_root.assign(nrec, -1);
    ix->bp_nsel.assign(nrec, 0);
    ix->bp_sel.assign(nrec * 64, -1);
    if (t == 0) return;
    fill(ix->bpd, 0xFF, st);
    if (n == 0) return;
    DBuf<uint32_t> used_bits((size_t)nwords), tmp_bits((size_t)nwords + 1);
    DBuf<int32_t> root(nrec), nsel(nrec), sel(nrec * 64);
    fill(used_bits, 0, st);
    fill(tmp_bits, 0, st);
    fill(sel, 0xFF, st);
    check(launch_bp_select(graph(), G, t, d_vtx_off.p, d_lbase.p, d_gpos.p, d_gblk.p,
                           ix->lrank.p,
                           used_bits.p, tmp_bits.p, used.p, root.p, nsel.p, sel.p, st));
    d2h(ix->bp_root.data(), root.p, nrec, st);
    d2h(ix->bp_nsel.data(), nsel.p, nrec, st);
    d2h(ix->bp_sel.data(), sel.p, nrec * 64, st);
    // distances start at infinity, sets empty
    fill(ix->bpd, 0xFF, st);
    fill(ix->bpm, 0, st);
    DBuf<uint64_t> found((size_t)n);
    fill(found, 0, st);
    // work items: (vertex, chunk of its adjacency list)
    const int bchunk = tu.bp_chunk;
    int64_t nitems = 0;
    DBuf<int32_t> it_v, it_c;
    {
      DBuf<int64_t> icnt((size_t)n), ioff((size_t)n + 1), tmp((size_t)scan_tmp_elems(n));
      check(launch_bpv_items_count(graph(), bchunk, icnt.p, ioff.p, tmp.p, st));
      d2h(&nitems, ioff.p + n, 1, st);
      check(hipStreamSynchronize(st));
      it_v.alloc((size_t)std::max<int64_t>(nitems, 1));
      it_c.alloc((size_t)std::max<int64_t>(nitems, 1));
      check(launch_bpv_items_fill(graph(), ioff.p, it_v.p, it_c.p, st));
    }
    DBpW b{t, tpad, ix->bpd.p, ix->bpm.p, found.p};
    check(launch_bpv_init((int32_t)nrec, t, b, root.p, nsel.p, sel.p, st));
    // per-level counts of newly reached (slot, vertex) pairs, and flags
    DBuf<unsigned long long> lcnt(kMaxLevels + 2);
    DBuf<int32_t> flags(1);
    fill(lcnt, 0, st);
    fill(flags, 0, st);
    std::vector<unsigned long long> hc(kMaxLevels + 2, 0);
    int L = 0;
    bool done = false;
    while (!done) {
      const int upto = std::min(L + tu.levels_per_sync, kMaxLevels - 1);
      for (; L < upto; L++) {
        check(launch_bpv_level(graph(), b, it_v.p, it_c.p, nitems, bchunk, L, lcnt.p + L, flags.p,
                               st));
        stat_levels++;
      }
      int32_t hf = 0;
      d2h(hc.data(), lcnt.p, hc.size(), st);
      d2h(&hf, flags.p, 1, st);
      check(hipStreamSynchronize(st));
      if (hf & kFlagRange) throw Fail{PLL_E_RANGE};
      // level L-1 found nothing new: every slot's BFS is over
      if (hc[L - 1] == 0 || L >= kMaxLevels - 1) done = true;
    }
    int64_t reached = 0;
    for (size_t i = 0; i < nrec; i++) reached += (ix->bp_root[i] >= 0 ? 1 : 0) + ix->bp_nsel[i];
    for (auto c : hc) reached += (int64_t)c;
    stat_bp_visited = reached;
    check(launch_bpv_finish((int64_t)n * t, ix->bpm.p, st));
    check(hipStreamSynchronize(st));
  }

  // Growing label store of one side (the labels of an undirected graph, or
  // L_IN / L_OUT of a directed one): per-vertex slots in a pool.
  struct Store {
    DBuf<int64_t> off;
    DBuf<int32_t> len, cap;
    DBuf<uint32_t> hub;
    DBuf<uint8_t> dist;
    DBuf<unsigned long long> top;
    DBuf<uint4> hdr;
    int64_t pool_cap = 0;
    DStore view() const {
      return DStore{off.p, len.p, cap.p, hub.p, dist.p, top.p, pool_cap, hdr.p};
    }
  };

  // One search direction of the pruned phase: the graph its BFSs follow,
  // the store it labels, the store the roots' tables come from, and its
  // window state.
  struct Side {
    DGraph g;
    DBuf<int64_t> lrow;  // live adjacency (g points here once compacted)
    DBuf<int32_t> lcol;
    Store *own = nullptr, *roots = nullptr;
    int64_t htcap = 0, fcap = 0, hcap = 0, ccap = 0;
    DBuf<uint32_t> vis;
    DBuf<uint8_t> wd, cd, cdes;
    DBuf<uint64_t> ht, cmask, kmask, sig, csum;
    DBuf<int64_t> htoff, hsize, htmp;
    DBuf<int32_t> fslot, fv, h1, cu, cj;
    DBuf<LevelCtl> ctl;
    PinnedMirror mirror;  // level counters and the own store's pool top
    DFrontier f;
    // each level's entries grouped by root for the prune tests
    DBuf<uint32_t> rc, rfill;
    DBuf<int64_t> roff, toff;
    DBuf<int32_t> sv;
    DRootSort rsort{};
    DWindow window(int32_t s, int32_t nr, int words, const uint8_t *used) const {
      return DWindow{s,       nr,      words,  vis.p, ht.p, htoff.p, htcap, sig.p, wd.p,
                     cmask.p, kmask.p, csum.p, cu.p,  cj.p, cd.p,    cdes.p, ccap,  used};
    }
  };

  void store_init(Store &S, int64_t pool_cap) {
    S.off.alloc((size_t)n);
    S.len.alloc((size_t)n);
    S.cap.alloc((size_t)n);
    fill(S.off, 0, st);
    fill(S.len, 0, st);
    fill(S.cap, 0, st);
    S.pool_cap = pool_cap;
    S.hub.alloc((size_t)pool_cap);
    S.dist.alloc((size_t)pool_cap);
    S.top.alloc(1);
    fill(S.top, 0, st);
    S.hdr.alloc((size_t)std::max<int32_t>(n, 1));  // set once the bit-parallel masks exist
  }

  // Grow the pool so that a commit of ncand candidates cannot run out
  // (each touched vertex takes at most 2*(len+new)+32 slots).
  void store_reserve(Store &S, int64_t entries_bound, int64_t ncand, unsigned long long htop) {
    const int64_t need = 2 * (entries_bound + ncand) + 32 * ncand + 64;
    if (S.pool_cap - (int64_t)htop >= need) return;
    const int64_t ncap = std::max<int64_t>(3 * S.pool_cap, (int64_t)htop + 2 * need);
    DBuf<uint32_t> nh((size_t)ncap);
    DBuf<uint8_t> nd((size_t)ncap);
    check(hipMemcpyAsync(nh.p, S.hub.p, (size_t)htop * sizeof(uint32_t), hipMemcpyDeviceToDevice,
                         st));
    check(hipMemcpyAsync(nd.p, S.dist.p, (size_t)htop, hipMemcpyDeviceToDevice, st));
    check(hipStreamSynchronize(st));
    S.hub = std::move(nh);
    S.dist = std::move(nd);
    S.pool_cap = ncap;
  }

  void side_init(Side &D, DGraph g, Store *own, Store *roots, int wmax, int words) {
    D.g = g;
    D.own = own;
    D.roots = roots;
    const int64_t wstride = (int64_t)words * 64;
    D.vis.alloc((size_t)wmax * nwords);
    D.wd.alloc((size_t)n * wstride);
    D.htcap = tu.table_cap > 0 ? tu.table_cap : std::max<int64_t>(1 << 20, 32 * (int64_t)wmax);
    D.ht.alloc((size_t)D.htcap);
    D.htoff.alloc((size_t)wmax + 1);
    D.hsize.alloc((size_t)wmax + 1);
    D.htmp.alloc((size_t)scan_tmp_elems((int64_t)wmax + 1));
    D.cmask.alloc((size_t)n * words);
    D.kmask.alloc((size_t)n * words);
    D.sig.alloc((size_t)wmax * 4);
    D.csum.alloc((size_t)n * 4);
    fill(D.vis, 0, st);
    fill(D.cmask, 0, st);
    fill(D.kmask, 0, st);
    fill(D.csum, 0, st);
    // list capacities: sized from the window, never below what one root
    // needs (a window of one root always fits); `list_cap` lowers them
    const int64_t lcap = tu.list_cap > 0 ? tu.list_cap : INT64_MAX;
    const int64_t m = g.row ? nnz : 0;
    D.fcap = std::max<int64_t>(2 * (int64_t)n + 64,
                               std::min<int64_t>({(int64_t)wmax * n, 96ll << 20, lcap}));
    D.hcap = std::max<int64_t>((int64_t)n + m / tu.chunk + 64,
                               std::min<int64_t>({(int64_t)wmax * (m / tu.chunk + 1), 16ll << 20,
                                                  lcap}));
    D.ccap = std::max<int64_t>((int64_t)n + 64,
                               std::min<int64_t>({(int64_t)wmax * n, 32ll << 20, lcap}));
    D.fslot.alloc((size_t)D.fcap);
    D.fv.alloc((size_t)D.fcap);
    D.h1.alloc((size_t)D.hcap * 3);
    D.cu.alloc((size_t)D.ccap);
    D.cj.alloc((size_t)D.ccap);
    D.cd.alloc((size_t)D.ccap);
    D.cdes.alloc((size_t)D.ccap);
    D.ctl.alloc(1);
    D.f = DFrontier{D.fslot.p, D.fv.p,  D.fcap,  D.h1.p, D.h1.p + D.hcap, D.h1.p + 2 * D.hcap,
                    D.hcap,    nullptr, nullptr, nullptr, D.ctl.p};
    D.rc.alloc(2 * (size_t)wmax);
    D.rfill.alloc((size_t)wmax);
    D.roff.alloc((size_t)wmax + 1);
    D.toff.alloc((size_t)wmax + 1);
    D.sv.alloc((size_t)D.fcap);
    fill(D.rc, 0, st);
    fill(D.rfill, 0, st);
    D.rsort = DRootSort{D.rc.p, D.rc.p + wmax, D.rfill.p, D.roff.p, D.toff.p, D.sv.p, D.fcap};
    D.mirror.p->ctl = LevelCtl{};
    D.mirror.p->top = 0;
  }

  // The pruned phase of the graphs in `whole`, one workgroup per graph, in
  // an empty store (before any window commits).  The pool is sized from
  // whole_pool entries per vertex of those graphs; if it runs out the store
  // is cleared and the launch redone with twice the pool.
  int64_t stat_whole_ns = 0;
  void whole_phase(Store &S, Side &D, const DBp &bp) {
    const auto t0 = Clock::now();
    const int32_t ng = (int32_t)whole.size();
    std::vector<int64_t> hb((size_t)ng);
    std::vector<int32_t> hn((size_t)ng);
    int64_t verts = 0;
    for (int32_t i = 0; i < ng; i++) {
      const int32_t g = whole[i];
      hb[i] = nwin + verts;
      hn[i] = (int32_t)(vtx_off[g + 1] - vtx_off[g]);
      verts += hn[i];
    }
    DBuf<int64_t> dbase((size_t)ng);
    DBuf<int32_t> dn((size_t)ng);
    DBuf<GraphCtl> ctl(1);
    h2d(dbase.p, hb.data(), (size_t)ng, st);
    h2d(dn.p, hn.data(), (size_t)ng, st);
    GraphPairs qp{nullptr, nullptr, nullptr, nullptr};
    DBuf<int64_t> qrange;
    if (qpairs) {
      std::vector<int64_t> hr(2 * (size_t)ng);
      stat_whole_pairs = 0;
      for (int32_t i = 0; i < ng; i++) {
        hr[2 * i] = qoff[whole[i]];
        hr[2 * i + 1] = qoff[whole[i] + 1];
        stat_whole_pairs += hr[2 * i + 1] - hr[2 * i];
      }
      qrange.alloc(hr.size());
      h2d(qrange.p, hr.data(), hr.size(), st);
      qp = GraphPairs{qpairs, qrange.p, rank_p, qout};
    }
    int dev = 0, cus = 0;
    check(hipGetDevice(&dev));
    check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int32_t grid = std::max(1, std::min(ng, 2 * cus));
    // whole_pool entries per vertex here, and the windows' first share (as
    // store_init gives every vertex of a single graph); at most half the
    // free device memory (5 bytes an entry), at least 16 entries a vertex
    // (a pool that runs out is doubled below)
    int64_t want = verts * tu.whole_pool + 32 * nwin + 64;
    {
      size_t fr = 0, tot = 0;
      if (hipMemGetInfo(&fr, &tot) == hipSuccess) {
        const int64_t cap = std::max<int64_t>((int64_t)(fr / 2 / 5), 16 * verts + 32 * nwin + 64);
        want = std::min<int64_t>(want, cap);
      } else {
        (void)hipGetLastError();
      }
    }
    for (;;) {
      if (want != S.pool_cap) {  // nothing to keep: the windows have not run
        S.hub.alloc((size_t)want);
        S.dist.alloc((size_t)want);
        S.pool_cap = want;
      }
      fill(ctl, 0, st);
      check(launch_graph_pruned(graph(), bp, used.p, S.view(), dbase.p, dn.p, ng, ctl.p, qp,
                                grid, st));
      GraphCtl h{};
      unsigned long long top = 0;
      d2h(&h, ctl.p, 1, st);
      d2h(&top, S.top.p, 1, st);
      check(hipStreamSynchronize(st));
      if (h.flags & kFlagRange) throw Fail{PLL_E_RANGE};
      if (h.flags & kFlagOvfPool) {
        // start over: no labels, an empty pool twice as large
        fill(S.off, 0, st);
        fill(S.len, 0, st);
        fill(S.cap, 0, st);
        fill(S.top, 0, st);
        want = 2 * S.pool_cap;
        stat_retries++;
        continue;
      }
      D.mirror.p->top = top;
      stat_visited += (int64_t)h.visited;
      stat_tests += (int64_t)h.tests;
      stat_scanned += (int64_t)h.scanned;
      stat_edges += (int64_t)h.edges;
      stat_cand += (int64_t)h.labeled;
      break;
    }
    stat_whole_ns = ns_since(t0);
  }

  // One window's BFS levels in one direction, until every root's search has
  // ended or a list overflowed.  Returns the last level index.
  int side_levels(Side &D, const DBp &bp, const DBp &rb, const DBp &vb, const DWindow &w,
                  int64_t window_index, std::vector<hipEvent_t> &evs, bool sorted) {
    LevelCtl &h = D.mirror.p->ctl;
    const DStore sto = D.own->view(), rsto = D.roots->view();
    const size_t mark0 = level_trace.size();
    check(launch_win_reset_ctl(D.ctl.p, st));
    check(launch_win_init(D.g, w, D.roots->view(), D.f, w.W, D.hsize.p, D.htmp.p, st));
    int d = 0;
    for (bool done = false; !done;) {
      const int d0 = d;
      const int upto = std::min(d + tu.levels_per_sync, kMaxLevels - 1);
      for (; d < upto; d++) {
        hipEvent_t *e = evs.empty() ? nullptr : &evs[4 * (size_t)(d - d0)];
        const DRootSort rs = sorted ? D.rsort : DRootSort{};
        check(launch_win_level(D.g, bp, rb, vb, sto, rsto, w, D.f, rs, d, test_group, tu.xgroup,
                               tu.chunk,
                               tu.expand_prune ? w.s : 0, st, e ? e[0] : nullptr,
                               e ? e[1] : nullptr, e ? e[2] : nullptr, e ? e[3] : nullptr));
        stat_levels++;
        stat_level_launches++;
      }
      check(hipMemcpyAsync(&h, D.ctl.p, sizeof(LevelCtl), hipMemcpyDeviceToHost, st));
      check(hipStreamSynchronize(st));
      for (int i = 0; !evs.empty() && i < d - d0; i++) {
        float ms = 0.f, xms = 0.f;
        check(hipEventElapsedTime(&ms, evs[4 * i], evs[4 * i + 1]));
        check(hipEventElapsedTime(&xms, evs[4 * i + 2], evs[4 * i + 3]));
        stat_level_ns += (int64_t)(ms * 1e6);
        stat_expand_ns += (int64_t)(xms * 1e6);
        const int lv = d0 + i;
        level_trace.insert(level_trace.end(), {window_index, (int64_t)w.s, (int64_t)w.W,
                                               (int64_t)lv, (int64_t)h.cnt[lv], 0,
                                               (int64_t)(ms * 1e6)});
      }
      if (h.flags || h.cnt[d] == 0 || d >= kMaxLevels - 1) done = true;
    }
    // candidates made at each traced level
    for (size_t r = mark0; r < level_trace.size(); r += kTraceCols) {
      const int lv = (int)level_trace[r + 3];
      const unsigned long long c1 = lv + 1 < d ? h.cmark[lv + 1] : h.ccnt;
      level_trace[r + 5] = (int64_t)(c1 - h.cmark[lv]);
    }
    return d;
  }

  // a4 + a5: pruned BFSs in root windows, cleaning, commit; final CSR.
  // An undirected graph has one side; a directed one (Section 6) a forward
  // side (follows the arcs, labels L_IN, root tables from L_OUT) and a
  // reverse side (in-edges, labels L_OUT, root tables from L_IN).
  bool directed = false;
  DBuf<int64_t> irow;  // in-edges of a directed graph (rank space)
  DBuf<int32_t> icol;

  // Lanes per prune test for an average scan of `len` label entries: short
  // labels keep many tests in flight per wave, long ones split a scan.  The
  // root-grouped kernel reads four entries per lane at a time.
  static int group_for_scan(int64_t len, bool sorted) {
    if (!sorted) return len < 48 ? 4 : len < 96 ? 8 : 16;
    return len < 24 ? 4 : len < 48 ? 8 : len < 96 ? 16 : len < 160 ? 32 : 64;
  }
  int test_group = 4;
  // prune tests grouped by root (each root's data in LDS) pay a sort per
  // level and win on long label scans; short ones test straight from the
  // frontier
  bool use_sort = false;

  void pruned(pll_index *ix) {
    const int nsides = directed ? 2 : 1;
    test_group = tu.group > 0 ? tu.group : 4;
    use_sort = tu.root_sort == 1;
    // per-root window state per side: distance column of wd (n B), visited
    // bits (n/8 B) and two mask bits per vertex (n/4 B)
    const int64_t per_root = nsides * ((int64_t)n + (n + 7) / 8 + (n + 3) / 4 + 1);
    // window_mem_mb, but no more than the device has free beyond a reserve
    // for the label pool and the lists (a fifth of the device, at least 8 GB)
    int64_t wbytes = tu.window_mem_mb << 20;
    {
      size_t fr = 0, tot = 0;
      if (hipMemGetInfo(&fr, &tot) == hipSuccess && tot > 0) {
        const int64_t reserve = std::max<int64_t>(8ll << 30, (int64_t)(tot / 5));
        wbytes = std::min<int64_t>(wbytes, std::max<int64_t>((int64_t)fr - reserve, 0));
      } else {
        (void)hipGetLastError();
      }
    }
    const int64_t wmem = std::max<int64_t>(64, wbytes / per_root);
    const int wmax =
        plain ? 1 : (int)std::max<int64_t>(1, std::min<int64_t>({tu.window, kMaxWindow, wmem}));
    const int words = (wmax + 63) / 64;
    const int64_t pool0 = std::max<int64_t>(32 * (int64_t)n, 1 << 20);
    Store stores[2];
    Side sides[2];
    if (!directed) {
      store_init(stores[0], pool0);
      side_init(sides[0], graph(), &stores[0], &stores[0], wmax, words);
    } else {
      irow.alloc((size_t)n + 1);
      icol.alloc((size_t)std::max<int64_t>(nnz, 1));
      {
        DBuf<int64_t> work((size_t)n + 1), tmp((size_t)scan_tmp_elems((int64_t)n + 1));
        check(launch_transpose(row.p, col.p, n, irow.p, icol.p, work.p, tmp.p, st));
        check(hipStreamSynchronize(st));
      }
      // stores[0] = L_IN (forward side), stores[1] = L_OUT (reverse side)
      store_init(stores[0], pool0);
      store_init(stores[1], pool0);
      side_init(sides[0], graph(), &stores[0], &stores[1], wmax, words);
      side_init(sides[1], DGraph{n, nwords, irow.p, icol.p}, &stores[1], &stores[0], wmax, words);
    }
    DBuf<uint64_t> bpz((size_t)std::max<int32_t>(n, 1));
    check(launch_bpv_nonempty(n, t, ix->bpm.p, bpz.p, st));
    for (int k = 0; k < nsides; k++)
      check(launch_store_hdr(stores[k].view(), t > 0 ? bpz.p : nullptr, n, st));
    DBp bp{t, ix->tpad, ix->bpd.p, ix->bpm.p, bpz.p};
    // 4-bit distance rows for the expansion's prune (half the bytes per
    // reached neighbour; same labels: a saturated distance never prunes)
    DBuf<uint4> bpq;
    if (t > 0 && ix->tpad % 32 == 0 && tu.packed_rows && n > 0) {
      bpq.alloc((size_t)n * (ix->tpad / 32));
      check(launch_bp_pack(ix->bpd.p, n, ix->tpad, bpq.p, st));
    }
    int64_t entries_bound[2] = {0, 0};
    // Expansion-time prune rows.  With bit-parallel labels they are the
    // bit-parallel distance rows (Section 5.4).  Without them (t = 0, and
    // every directed build) the first window's first kLandmarks roots prune
    // nothing, so its window distances are exact BFS distances from them;
    // kept as rows, they bound QUERY(root, x) over the committed labels for
    // every later window (the minimum of d(root, h) + d(h, x) over committed
    // hubs h), so a neighbour at or below the bound is left unvisited as a
    // bit-parallel row would leave it.  land[k] comes from side k.
    DBuf<uint8_t> land[2];
    bool have_land = false;
    const DBp no_rows{0, 0, nullptr, nullptr, nullptr};

    // optional timing of each level kernel (events on the build stream)
    std::vector<hipEvent_t> evs;
    if (tu.profile) {
      evs.resize(4 * (size_t)tu.levels_per_sync);
      for (auto &e : evs) check(hipEventCreate(&e));
    }
    struct EvGuard {
      std::vector<hipEvent_t> &v;
      ~EvGuard() {
        for (auto e : v) (void)hipEventDestroy(e);
      }
    } ev_guard{evs};

    // graphs built whole, one workgroup each, before the windows: their
    // ranks follow the windows' range and no window root reaches them
    if (!whole.empty()) whole_phase(stores[0], sides[0], bp);

    // Window size: fixed at wmax, or adapted so that each window does about
    // window_work visits (early roots have large pruned BFSs, late ones
    // tiny; one launch per level must still fill the device).
    int32_t s = 0;
    const bool adaptive = tu.window_work > 0 && wmax > 1;
    int W = adaptive ? std::min(wmax, 256) : wmax;
    // live adjacency: rebuilt without the neighbours ranked below s each
    // time s has doubled (the expansion skips them anyway)
    int32_t live_s = 0;
    while (s < nwin) {
      if (!plain && tu.live_adjacency && tu.expand_prune && s >= 1024 && s >= 2 * live_s) {
        for (int k = 0; k < nsides; k++) {
          Side &D = sides[k];
          DBuf<int64_t> nrow((size_t)n + 1), cnt((size_t)n), tmp((size_t)scan_tmp_elems(n));
          DBuf<int32_t> ncol((size_t)std::max<int64_t>(nnz, 1));
          check(launch_live_adjacency(D.g, s, nrow.p, ncol.p, cnt.p, tmp.p, st));
          D.lrow = std::move(nrow);
          D.lcol = std::move(ncol);
          D.g = DGraph{n, nwords, D.lrow.p, D.lcol.p};
        }
        live_s = s;
      }
      const int32_t e = (int32_t)std::min<int64_t>((int64_t)s + W, nwin);
      const int32_t nr = e - s;
      DWindow w[2];
      int last[2] = {0, 0};
      bool ran[2] = {false, false};
      int flags = 0;
      for (int k = 0; k < nsides && !flags; k++) {  // after an overflow the window is redone
        w[k] = sides[k].window(s, nr, words, used.p);
        DBp rb = t > 0 && tu.expand_prune ? bp : no_rows, vb = rb;
        if (t > 0 && tu.expand_prune) vb.q = bpq.p;
        if (t == 0 && have_land && s >= kLandmarks && tu.expand_prune) {
          rb = DBp{kLandmarks, kLandmarks, land[nsides - 1 - k].p, nullptr, nullptr};
          vb = DBp{kLandmarks, kLandmarks, land[k].p, nullptr, nullptr};
        }
        last[k] = side_levels(sides[k], bp, rb, vb, w[k], stat_windows, evs, use_sort);
        ran[k] = true;
        flags |= sides[k].mirror.p->ctl.flags;
      }
      int64_t nvisited[2] = {0, 0}, ncand[2] = {0, 0};
      for (int k = 0; k < nsides; k++) {
        if (!ran[k]) continue;
        const LevelCtl &h = sides[k].mirror.p->ctl;
        for (int i = 0; i <= last[k]; i++) nvisited[k] += (int64_t)h.cnt[i];
        ncand[k] = std::min<int64_t>((int64_t)h.ccnt, sides[k].ccap);
      }
      if (flags) {
        // undo the window (both sides) and run it again
        int reset_flags = 0;
        for (int k = 0; k < nsides; k++) {
          if (!ran[k]) continue;
          Side &D = sides[k];
          const LevelCtl &h = D.mirror.p->ctl;
          reset_flags |= h.flags;
          check(launch_win_reset(D.g, w[k], D.own->view(), D.f, nr,
                                 std::min(nvisited[k], D.fcap), st));
          check(launch_win_abort(D.g, w[k], ncand[k], st));
          if (h.flags & kFlagOvfFrontier) fill(D.vis, 0, st);
          // candidates past the list's end set mask bits the list cannot undo
          if (h.flags & kFlagOvfCand) {
            fill(D.cmask, 0, st);
            fill(D.csum, 0, st);
          }
        }
        check(hipStreamSynchronize(st));
        level_trace.resize(trace_mark);
        if (reset_flags == kFlagOvfHash) {
          // same window again with room for its root tables
          for (int k = 0; k < nsides; k++) {
            if (!ran[k]) continue;
            Side &D = sides[k];
            const unsigned long long tot = D.mirror.p->ctl.httotal;
            if ((int64_t)tot > D.htcap) {
              D.htcap = std::max<int64_t>(2 * D.htcap, (int64_t)tot + (int64_t)tot / 4);
              D.ht.alloc((size_t)D.htcap);
            }
          }
          continue;
        }
        if (W == 1) throw Fail{(reset_flags & kFlagRange) ? PLL_E_RANGE : PLL_E_NOMEM};
        W = std::max(1, W / 4);
        stat_retries++;
        continue;
      }
      if (t == 0 && s == 0 && nr >= kLandmarks && !have_land && !plain && tu.landmarks) {
        for (int k = 0; k < nsides; k++) {
          land[k].alloc((size_t)n * kLandmarks);
          check(launch_win_landmarks(w[k], n, land[k].p, st));
        }
        have_land = true;
      }
      for (int k = 0; k < nsides; k++) {
        store_reserve(*sides[k].own, entries_bound[k], ncand[k], sides[k].mirror.p->top);
        check(launch_win_reset(sides[k].g, w[k], sides[k].own->view(), sides[k].f, nr,
                               nvisited[k], st));
      }
      // cleaning reads both sides' masks; then each side commits its store
      for (int k = 0; k < nsides; k++)
        check(launch_win_clean(w[k], w[nsides - 1 - k], ncand[k], st));
      double work = 0;
      int64_t wtests = 0, wscanned = 0, wvisits = 0, wlevels = 0;
      for (int k = 0; k < nsides; k++) {
        check(launch_win_commit(w[k], sides[k].own->view(), ncand[k], st));
        // the pool top only moves in commits: read back once per window (the
        // next window's first synchronisation completes the copy)
        check(hipMemcpyAsync(&sides[k].mirror.p->top, sides[k].own->top.p,
                             sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
        const LevelCtl &h = sides[k].mirror.p->ctl;
        entries_bound[k] += ncand[k];
        stat_visited += (int64_t)h.visited;
        stat_tests += (int64_t)h.ntests;
        stat_scanned += (int64_t)h.lscanned;
        stat_edges += (int64_t)h.edges;
        stat_hedges += (int64_t)h.hedges;
        stat_bp_direct += (int64_t)(h.bp_direct + h.hdirect);
        stat_earlier += (int64_t)(h.earlier + h.hearlier);
        stat_x_direct += (int64_t)h.bp_direct;
        stat_x_earlier += (int64_t)h.earlier;
        stat_x_claims += (int64_t)h.xclaims;
        stat_bp_sets += (int64_t)h.bp_sets;
        stat_bp_checks += (int64_t)h.bp_checks;
        stat_cand += ncand[k];
        work += (double)h.visited + (double)h.bp_direct;
        wtests += (int64_t)h.ntests;
        wscanned += (int64_t)h.lscanned;
        wvisits += (int64_t)h.visited;
        wlevels += last[k] + 1;
      }
      // "group" 0: lanes per prune test follow the label entries a test
      // scanned in this window (labels grow as roots commit)
      // root grouping pays a sort per level: worth it once levels are large
      // or their label scans long
      use_sort = tu.root_sort == 1 ||
                 (tu.root_sort == 2 && wlevels > 0 &&
                  (wvisits / wlevels >= tu.sort_level || wscanned / wlevels >= tu.sort_scan));
      if (tu.group == 0 && wtests >= 1024) test_group = group_for_scan(wscanned / wtests, use_sort);
      stat_windows++;
      trace_mark = level_trace.size();
      s = e;
      if (adaptive) {
        double f = (double)tu.window_work / std::max(work, 1.0);
        f = std::min(4.0, std::max(0.25, f));
        W = (int)std::min<double>(wmax, std::max(1.0, W * f));
      } else if (W < wmax) {
        W = std::min(wmax, W * 2);
      }
    }
    check(hipStreamSynchronize(st));
    {
      std::vector<uint8_t> hused((size_t)n);
      d2h(hused.data(), used.p, (size_t)n, st);
      check(hipStreamSynchronize(st));
      for (uint8_t x : hused) stat_roots += x ? 0 : 1;
    }

    // a5: final CSR with sentinels (L_OUT in off/hub/dist, L_IN apart)
    ix->entries = 0;
    for (int k = nsides - 1; k >= 0; k--) {
      Store &S = stores[k];
      const bool in_side = directed && k == 0;
      DBuf<int64_t> &foff = in_side ? ix->ioff : ix->off;
      DBuf<uint32_t> &fhub = in_side ? ix->ihub : ix->hub;
      DBuf<uint8_t> &fdist = in_side ? ix->idist : ix->dist;
      DBuf<int64_t> cnt((size_t)n), tmp((size_t)scan_tmp_elems(n));
      foff.alloc((size_t)n + 1);
      check(launch_final_count(S.len.p, cnt.p, n, st));
      check(launch_exclusive_scan(cnt.p, foff.p, n, tmp.p, st));
      int64_t total = 0;
      if (n > 0) d2h(&total, foff.p + n, 1, st);
      check(hipStreamSynchronize(st));
      fhub.alloc((size_t)std::max<int64_t>(total, 1));
      fdist.alloc((size_t)std::max<int64_t>(total, 1));
      check(launch_final_copy(S.view(), foff.p, fhub.p, fdist.p, n, st));
      if (parents) {
        // the search of side k reaches u from p over an edge p -> u of its
        // graph: p's row in the other direction's CSR (the same CSR for an
        // undirected graph)
        DBuf<uint32_t> &fpar = in_side ? ix->ipar : ix->par;
        fpar.alloc((size_t)std::max<int64_t>(total, 1));
        const DGraph pred = !directed ? graph() : k == 0 ? DGraph{n, nwords, irow.p, icol.p}
                                                         : graph();
        DBuf<int64_t> icnt((size_t)std::max(n, 1)), ioff((size_t)n + 1),
            itmp((size_t)scan_tmp_elems((int64_t)n + 1));
        check(launch_tree_count(pred, icnt.p, n, st));
        check(launch_exclusive_scan(icnt.p, ioff.p, n, itmp.p, st));
        int64_t nitems = 0;
        if (n > 0) d2h(&nitems, ioff.p + n, 1, st);
        check(hipStreamSynchronize(st));
        DBuf<int32_t> items((size_t)std::max<int64_t>(nitems, 1));
        check(launch_tree_parents(pred, foff.p, fhub.p, fdist.p, fpar.p, n, ioff.p, items.p,
                                  nitems, st));
      }
      check(hipStreamSynchronize(st));
      ix->entries += total - n;
    }
  }
};

// ---------------------------------------------------------------------------
// Weighted graphs (Section 6): pruned Dijkstra searches in root windows
// (weighted.hip), 32-bit distances, no bit-parallel labels.

// Pinned host copy of a weighted window's control block and its store's
// pool top, read back with one synchronisation.
struct WMirrorData {
  WCtl ctl;
  unsigned long long top;
};
PinnedPool<WMirrorData> g_wctl_pinned;
struct WMirror {
  WMirrorData *p = nullptr;
  WMirror() { p = g_wctl_pinned.get(); }
  ~WMirror() {
    if (p) g_wctl_pinned.put(p);
  }
  WMirror(const WMirror &) = delete;
  WMirror &operator=(const WMirror &) = delete;
};

constexpr int32_t kMaxWWindow = 4096;  // roots per weighted window (64 mask words)

struct WBuilder {
  hipStream_t st;
  Tuning tu;
  bool plain = false, directed = false, parents = false;
  int32_t n = 0;
  int64_t nnz = 0;
  DBuf<int64_t> row, irow;
  DBuf<int32_t> col, icol;
  DBuf<uint32_t> wt, iwt;
  int64_t stat_windows = 0, stat_retries = 0, stat_steps = 0, stat_proc = 0, stat_tests = 0,
          stat_scanned = 0, stat_edges = 0, stat_improved = 0, stat_cand = 0, stat_touched = 0,
          stat_level_ns = 0, stat_step_launches = 0, stat_filtered = 0,
          stat_checked = 0;

  struct WStore {
    DBuf<int64_t> off;
    DBuf<int32_t> len, cap;
    DBuf<uint64_t> ent;
    DBuf<uint32_t> par;  // null unless parents are kept
    DBuf<unsigned long long> top;
    int64_t pool_cap = 0;
    int64_t entries = 0;  // committed so far (host count)
    DWStore view() const { return DWStore{off.p, len.p, cap.p, ent.p, top.p, pool_cap, par.p}; }
  };

  // One search direction: the graph it follows, the store it labels, the
  // store its root tables come from, and its window state.
  struct WSide {
    DWGraph g;
    DBuf<int64_t> lrow;  // live adjacency (g points here once compacted)
    DBuf<int32_t> lcol;
    DBuf<uint32_t> lwt;
    WStore *own = nullptr, *roots = nullptr;
    int64_t htcap = 0, fcap = 0, tcap = 0, ccap = 0;
    int32_t wmax = 0;
    DBuf<uint32_t> td, cd, cp;
    DBuf<uint64_t> tdp;
    DBuf<uint8_t> fl, cdes;
    DBuf<uint64_t> ht, lm, km, lsum, sig;
    DBuf<int64_t> htoff, hsize, htmp;
    DBuf<int32_t> fj0, fu0, fj1, fu1, tj, tu, cj, cu;
    DBuf<WCtl> ctl;
    WMirror mirror;
    DWWindow window(int32_t s, int32_t W, int32_t nn, const uint16_t *lroot,
                    const uint16_t *lvert, const uint8_t *lskip) const {
      DWWindow w;
      w.lroot = lroot;
      w.lvert = lvert;
      w.lskip = lskip;
      w.s = s;
      w.W = W;
      w.n = nn;
      w.words = (W + 63) / 64;
      w.td = td.p;
      w.tdp = tdp.p;
      w.cp = cp.p;
      w.fl = fl.p;
      w.ht = ht.p;
      w.htoff = htoff.p;
      w.htcap = htcap;
      w.sig = sig.p;
      w.lm = lm.p;
      w.km = km.p;
      w.lsum = lsum.p;
      w.fj0 = fj0.p;
      w.fu0 = fu0.p;
      w.fj1 = fj1.p;
      w.fu1 = fu1.p;
      w.fcap = fcap;
      w.tj = tj.p;
      w.tu = tu.p;
      w.tcap = tcap;
      w.cj = cj.p;
      w.cu = cu.p;
      w.cd = cd.p;
      w.cdes = cdes.p;
      w.ccap = ccap;
      w.ctl = ctl.p;
      return w;
    }
  };

  void store_init(WStore &S, int64_t pool_cap) {
    S.off.alloc((size_t)n);
    S.len.alloc((size_t)n);
    S.cap.alloc((size_t)n);
    fill(S.off, 0, st);
    fill(S.len, 0, st);
    fill(S.cap, 0, st);
    S.pool_cap = pool_cap;
    S.ent.alloc((size_t)pool_cap);
    if (parents) S.par.alloc((size_t)pool_cap);
    S.top.alloc(1);
    fill(S.top, 0, st);
  }

  // Grow the pool so that committing ncand candidates cannot run out (a
  // vertex that grows takes at most 2*(len+new)+16 slots).
  void store_reserve(WStore &S, int64_t ncand, unsigned long long htop) {
    const int64_t need = 2 * (S.entries + ncand) + 16 * ncand + 64;
    if (S.pool_cap - (int64_t)htop >= need) return;
    const int64_t ncap = std::max<int64_t>(2 * S.pool_cap, (int64_t)htop + 2 * need);
    DBuf<uint64_t> ne((size_t)ncap);
    DBuf<uint32_t> np;
    check(hipMemcpyAsync(ne.p, S.ent.p, (size_t)htop * sizeof(uint64_t), hipMemcpyDeviceToDevice,
                         st));
    if (parents) {
      np.alloc((size_t)ncap);
      check(hipMemcpyAsync(np.p, S.par.p, (size_t)htop * sizeof(uint32_t),
                           hipMemcpyDeviceToDevice, st));
    }
    check(hipStreamSynchronize(st));
    S.ent = std::move(ne);
    if (parents) S.par = std::move(np);
    S.pool_cap = ncap;
  }

  void side_init(WSide &D, DWGraph g, WStore *own, WStore *roots, int32_t wmax) {
    D.g = g;
    D.own = own;
    D.roots = roots;
    D.wmax = wmax;
    const int64_t cells = (int64_t)wmax * n;
    if (parents) {
      D.tdp.alloc((size_t)cells);
      fill(D.tdp, 0xFF, st);
    } else {
      D.td.alloc((size_t)cells);
      fill(D.td, 0xFF, st);
    }
    D.fl.alloc((size_t)((cells + 3) & ~(int64_t)3));
    fill(D.fl, 0, st);
    const int64_t words = (wmax + 63) / 64;
    D.lm.alloc((size_t)n * words);
    D.km.alloc((size_t)n * words);
    D.lsum.alloc((size_t)n);
    fill(D.lm, 0, st);
    fill(D.km, 0, st);
    fill(D.lsum, 0, st);
    D.htcap = tu.table_cap > 0 ? tu.table_cap : std::max<int64_t>(1 << 20, 64 * (int64_t)wmax);
    D.ht.alloc((size_t)D.htcap);
    D.htoff.alloc((size_t)wmax + 1);
    D.hsize.alloc((size_t)wmax + 1);
    D.htmp.alloc((size_t)scan_tmp_elems((int64_t)wmax + 1));
    D.sig.alloc((size_t)wmax * 4);
    // every list holds at least one root's worth (n entries), so one root
    // always fits
    const int64_t budget = tu.list_cap > 0 ? tu.list_cap : (int64_t)1 << 25;
    const int64_t cap = std::max<int64_t>(std::max<int64_t>(n, 1), std::min<int64_t>(cells, budget));
    D.fcap = D.tcap = D.ccap = cap;
    D.fj0.alloc((size_t)cap);
    D.fu0.alloc((size_t)cap);
    D.fj1.alloc((size_t)cap);
    D.fu1.alloc((size_t)cap);
    D.tj.alloc((size_t)cap);
    D.tu.alloc((size_t)cap);
    D.cj.alloc((size_t)cap);
    D.cu.alloc((size_t)cap);
    D.cd.alloc((size_t)cap);
    D.cdes.alloc((size_t)cap);
    if (parents) D.cp.alloc((size_t)cap);
    D.ctl.alloc(1);
  }

  // Back to the all-clear state after an aborted window (lists may have
  // overflowed, so no reset list can be trusted).
  void side_clear(WSide &D, int32_t W) {
    const int64_t cells = (int64_t)W * n;
    if (parents)
      check(hipMemsetAsync(D.tdp.p, 0xFF, (size_t)cells * sizeof(uint64_t), st));
    else
      check(hipMemsetAsync(D.td.p, 0xFF, (size_t)cells * sizeof(uint32_t), st));
    check(hipMemsetAsync(D.fl.p, 0, (size_t)((cells + 3) & ~(int64_t)3), st));
    fill(D.lm, 0, st);
    fill(D.km, 0, st);
    fill(D.lsum, 0, st);
  }

  void pruned(pll_index *ix) {
    const int nsides = directed ? 2 : 1;
    WStore stores[2];
    const int64_t pool0 = std::max<int64_t>(1 << 16, 8 * (int64_t)n);
    for (int k = 0; k < nsides; k++) store_init(stores[k], pool0);
    // memory: td and fl take 5 bytes per (root, vertex) cell per side (9
    // with parents)
    const int64_t mem = std::max<int64_t>(1, tu.window_mem_mb) << 20;
    const int64_t per_root = (parents ? 9 : 5) * (int64_t)std::max(n, 1) * nsides;
    int32_t wmax = (int32_t)std::max<int64_t>(
        1, std::min<int64_t>({(int64_t)tu.window, (int64_t)kMaxWWindow, mem / per_root,
                              (int64_t)std::max(n, 1)}));
    if (plain) wmax = 1;
    WSide sides[2];
    // an undirected graph: one side labeling L with tables from L.  A
    // digraph: side 0 follows the arcs (labels L_IN of what it reaches,
    // tables from L_OUT(root)), side 1 follows them backwards (labels L_OUT,
    // tables from L_IN(root)).
    const DWGraph gf{n, row.p, col.p, wt.p};
    if (!directed) {
      side_init(sides[0], gf, &stores[0], &stores[0], wmax);
    } else {
      const DWGraph gr{n, irow.p, icol.p, iwt.p};
      side_init(sides[0], gf, &stores[1], &stores[0], wmax);
      side_init(sides[1], gr, &stores[0], &stores[1], wmax);
    }
    check(hipStreamSynchronize(st));
    const int64_t target = std::max<int64_t>(1, tu.wwork);
    // the first window: the kWLand landmark searches, unpruned and exact
    int32_t W = plain ? 1 : std::min<int32_t>(wmax, kWLand);
    // with the "profile" knob: an event pair around every step kernel of a
    // batch, read after the batch's synchronisation
    struct EvPool {
      std::vector<hipEvent_t> ev;
      ~EvPool() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
      }
    } evp;
    if (tu.profile) {
      evp.ev.resize((size_t)2 * tu.levels_per_sync * nsides, nullptr);
      for (auto &e : evp.ev) check(hipEventCreate(&e));
    }
    // landmark rows for the relaxation filter (weighted.hip): land[k] from
    // side k's first window, vertex-major
    DBuf<uint16_t> land[2];
    DBuf<uint8_t> lskip[2];
    bool have_land = false;
    int32_t s = 0;
    // live adjacency as in the unweighted build: relaxations toward
    // vertices ranked below s would be pruned, so each time s has doubled
    // the CSR is rebuilt without them
    int32_t live_s = 0;
    while (s < n) {
      if (!plain && tu.live_adjacency && s >= 1024 && s >= 2 * live_s) {
        for (int k = 0; k < nsides; k++) {
          WSide &D = sides[k];
          DBuf<int64_t> nrow((size_t)n + 1), cnt((size_t)n), tmp((size_t)scan_tmp_elems(n));
          DBuf<int32_t> ncol((size_t)std::max<int64_t>(nnz, 1));
          DBuf<uint32_t> nwt((size_t)std::max<int64_t>(nnz, 1));
          check(launch_live_adjacency(DGraph{n, 0, D.g.row, D.g.col}, s, nrow.p, ncol.p, cnt.p,
                                      tmp.p, st, D.g.wt, nwt.p));
          D.lrow = std::move(nrow);
          D.lcol = std::move(ncol);
          D.lwt = std::move(nwt);
          D.g = DWGraph{n, D.lrow.p, D.lcol.p, D.lwt.p};
        }
        live_s = s;
      }
      const int32_t nr = std::min<int32_t>(W, n - s);
      DWWindow win[2];
      for (int k = 0; k < nsides; k++) {
        const bool filt = have_land && s >= kWLand;
        win[k] = sides[k].window(s, nr, n, filt ? land[nsides - 1 - k].p : nullptr,
                                 filt ? land[k].p : nullptr, filt ? lskip[k].p : nullptr);
        check(launch_ww_reset_ctl(sides[k].ctl.p, st));
        check(launch_ww_init(sides[k].roots->view(), win[k], sides[k].hsize.p, sides[k].htmp.p,
                             st));
      }
      // steps until every side's frontier is empty
      int cur = 0;
      int32_t flags = 0;
      int64_t wsteps = 0;
      for (;;) {
        // step i settles every entry whose search path has at most i edges,
        // so n + 1 steps always suffice
        if (wsteps > (int64_t)n + 1 + tu.levels_per_sync) throw Fail{PLL_E_DEVICE};
        wsteps += tu.levels_per_sync;
        size_t ne = 0;
        for (int b = 0; b < tu.levels_per_sync; b++) {
          for (int k = 0; k < nsides; k++) {
            check(launch_ww_zero_list(sides[k].ctl.p, cur ^ 1, st));
            check(launch_ww_step(sides[k].g, sides[k].own->view(), win[k], cur, tu.wgroup, st,
                                 evp.ev.empty() ? nullptr : evp.ev[ne],
                                 evp.ev.empty() ? nullptr : evp.ev[ne + 1]));
            ne += 2;
            stat_step_launches++;
          }
          cur ^= 1;
          stat_steps++;
        }
        for (int k = 0; k < nsides; k++)
          check(hipMemcpyAsync(&sides[k].mirror.p->ctl, sides[k].ctl.p, sizeof(WCtl),
                               hipMemcpyDeviceToHost, st));
        check(hipStreamSynchronize(st));
        for (size_t e = 0; e < evp.ev.size(); e += 2) {
          float ms = 0.f;
          check(hipEventElapsedTime(&ms, evp.ev[e], evp.ev[e + 1]));
          stat_level_ns += (int64_t)((double)ms * 1e6);
        }
        bool more = false;
        for (int k = 0; k < nsides; k++) {
          flags |= sides[k].mirror.p->ctl.flags;
          more |= sides[k].mirror.p->ctl.fcnt[cur].v != 0;
        }
        if (flags || !more) break;
      }
      if (!flags) {
        for (int k = 0; k < nsides; k++) check(launch_ww_collect(win[k], st));
        for (int k = 0; k < nsides; k++) check(launch_ww_clean(win[k], win[nsides - 1 - k], st));
        for (int k = 0; k < nsides; k++) {
          check(hipMemcpyAsync(&sides[k].mirror.p->ctl, sides[k].ctl.p, sizeof(WCtl),
                               hipMemcpyDeviceToHost, st));
          check(hipMemcpyAsync(&sides[k].mirror.p->top, sides[k].own->top.p,
                               sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
        }
        check(hipStreamSynchronize(st));
        for (int k = 0; k < nsides; k++) flags |= sides[k].mirror.p->ctl.flags;
      }
      if (flags) {
        // run the window again: bigger tables, or fewer roots
        stat_retries++;
        for (int k = 0; k < nsides; k++) side_clear(sides[k], nr);
        if (flags & kWOvfHash) {
          for (int k = 0; k < nsides; k++) {
            WSide &D = sides[k];
            const int64_t want = (int64_t)D.mirror.p->ctl.httotal;
            if (want > D.htcap) {
              D.htcap = std::max<int64_t>(2 * D.htcap, want + want / 2);
              D.ht.alloc((size_t)D.htcap);
            }
          }
        } else if (W > 1) {
          W = std::max<int32_t>(1, W / 4);
        } else {
          throw Fail{PLL_E_NOMEM};  // one root's lists cannot overflow
        }
        check(hipStreamSynchronize(st));
        continue;
      }
      const bool make_land = s == 0 && nr >= kWLand && !have_land && !plain && tu.landmarks;
      if (make_land) {
        // the first window's searches had no labels to prune with: its
        // first kWLand distance rows are exact
        for (int k = 0; k < nsides; k++) {
          land[k].alloc((size_t)n * kWLand);
          check(launch_ww_landmarks(win[k], land[k].p, st));
        }
      }
      for (int k = 0; k < nsides; k++)
        store_reserve(*sides[k].own, (int64_t)sides[k].mirror.p->ctl.ccnt,
                      sides[k].mirror.p->top);
      for (int k = 0; k < nsides; k++) check(launch_ww_commit(win[k], sides[k].own->view(), st));
      if (make_land) {
        // landmark hubs at the head of every label, once they are committed
        for (int k = 0; k < nsides; k++) {
          lskip[k].alloc((size_t)n);
          check(launch_ww_lskip(sides[k].own->view(), n, lskip[k].p, st));
        }
        have_land = true;
      }
      for (int k = 0; k < nsides; k++) check(launch_ww_reset(win[k], st));
      int64_t touched = 0;
      for (int k = 0; k < nsides; k++) {
        const WCtl &c = sides[k].mirror.p->ctl;
        sides[k].own->entries += (int64_t)c.survivors;
        stat_proc += (int64_t)c.processed;
        stat_tests += (int64_t)c.tests;
        stat_scanned += (int64_t)c.scanned;
        stat_edges += (int64_t)c.edges;
        stat_improved += (int64_t)c.improved;
        stat_filtered += (int64_t)c.filtered;
        stat_checked += (int64_t)c.checked;
        stat_cand += (int64_t)c.ccnt;
        touched += (int64_t)c.tcnt;
      }
      stat_touched += touched;
      stat_windows++;
      s += nr;
      if (!plain && tu.wwork == 0) {
        W = wmax;  // fixed windows
      } else if (!plain) {
        // aim the next window at `target` touched entries
        int64_t nw = touched > 0 ? (int64_t)((double)W * target / (double)touched) : 4 * (int64_t)W;
        nw = std::max<int64_t>(nw, std::max<int64_t>(1, W / 4));
        nw = std::min<int64_t>(nw, 4 * (int64_t)W);
        W = (int32_t)std::max<int64_t>(1, std::min<int64_t>(nw, wmax));
      }
    }
    check(hipStreamSynchronize(st));
    // final CSR with sentinels: L (or L_OUT) at off/went, L_IN at ioff/iwent
    ix->entries = 0;
    for (int k = 0; k < nsides; k++) {
      WStore &S = stores[k];
      const bool in_side = directed && k == 1;
      DBuf<int64_t> &foff = in_side ? ix->ioff : ix->off;
      DBuf<uint64_t> &fent = in_side ? ix->iwent : ix->went;
      DBuf<uint32_t> &fpar = in_side ? ix->ipar : ix->par;
      DBuf<int64_t> cnt((size_t)std::max(n, 1)), tmp((size_t)scan_tmp_elems(n));
      foff.alloc((size_t)n + 1);
      check(launch_wfinal_count(S.len.p, cnt.p, n, st));
      check(launch_exclusive_scan(cnt.p, foff.p, n, tmp.p, st));
      int64_t total = 0;
      if (n > 0) d2h(&total, foff.p + n, 1, st);
      check(hipStreamSynchronize(st));
      fent.alloc((size_t)std::max<int64_t>(total, 1));
      if (parents) fpar.alloc((size_t)std::max<int64_t>(total, 1));
      check(launch_wfinal_copy(S.view(), foff.p, fent.p, parents ? fpar.p : nullptr, n, st));
      check(hipStreamSynchronize(st));
      ix->entries += total - n;
    }
  }
};

// Host-side checks of a weighted graph: weights >= 1 and, for an undirected
// graph under PLL_VALIDATE, every (u, v, w) matched by (v, u, w).
int validate_weights(int32_t n, const int32_t *row_ptr, const int32_t *col, const uint32_t *wgt,
                     bool symmetric) {
  const int64_t nnz = n > 0 ? row_ptr[n] : 0;
  if (nnz > 0 && !wgt) return PLL_E_INVAL;
  for (int64_t j = 0; j < nnz; j++)
    if (wgt[j] == 0) return PLL_E_INVAL;
  if (!symmetric) return PLL_OK;
  std::vector<std::pair<int32_t, uint32_t>> e((size_t)nnz);
  for (int64_t j = 0; j < nnz; j++) e[j] = {col[j], wgt[j]};
  for (int32_t v = 0; v < n; v++) std::sort(e.begin() + row_ptr[v], e.begin() + row_ptr[v + 1]);
  for (int32_t v = 0; v < n; v++)
    for (int32_t j = row_ptr[v]; j < row_ptr[v + 1]; j++) {
      const int32_t u = e[j].first;
      if (!std::binary_search(e.begin() + row_ptr[u], e.begin() + row_ptr[u + 1],
                              std::make_pair(v, e[j].second)))
        return PLL_E_INVAL;
    }
  return PLL_OK;
}

int build_weighted(int32_t n, const int32_t *row_ptr, const int32_t *col, const uint32_t *wgt,
                   const int32_t *order, int64_t nnz, uint32_t flags, hipStream_t st,
                   pll_index *ix) {
  const auto t0 = Clock::now();
  const bool device = (flags & PLL_DEVICE_PTRS) != 0;
  WBuilder wb;
  wb.st = st;
  wb.tu = tuning();
  wb.plain = (flags & PLL_PLAIN) != 0;
  wb.directed = (flags & PLL_DIRECTED) != 0;
  wb.parents = (flags & PLL_PARENTS) != 0;
  wb.n = n;
  wb.nnz = nnz;
  ix->weighted = true;
  ix->directed = wb.directed;
  ix->n = n;
  ix->t = 0;
  // inputs on the device (copies of host arrays)
  DBuf<int32_t> h_row, h_col, h_order;
  DBuf<uint32_t> h_w;
  const int32_t *d_row = row_ptr, *d_col = col, *d_order = order;
  const uint32_t *d_w = wgt;
  if (!device) {
    h_row.alloc((size_t)n + 1);
    h_col.alloc((size_t)std::max<int64_t>(nnz, 1));
    h_order.alloc((size_t)std::max(n, 1));
    h_w.alloc((size_t)std::max<int64_t>(nnz, 1));
    h2d(h_row.p, row_ptr, (size_t)n + 1, st);
    h2d(h_col.p, col, (size_t)nnz, st);
    h2d(h_order.p, order, (size_t)n, st);
    h2d(h_w.p, wgt, (size_t)nnz, st);
    d_row = h_row.p;
    d_col = h_col.p;
    d_order = h_order.p;
    d_w = h_w.p;
  }
  // a1: ranks and the rank-space CSR (the unweighted relabel), weights
  // moved along with their edges
  {
    Builder b;
    b.st = st;
    b.tu = wb.tu;
    b.G = 1;
    b.vtx_off = {0, (int64_t)n};
    b.n = n;
    b.t = 0;
    b.nwords = (n + 31) / 32;
    b.nnz = nnz;
    b.relabel(d_row, d_col, d_order, true, ix, nullptr);
    wb.row = std::move(b.row);
    wb.col = std::move(b.col);
  }
  wb.wt.alloc((size_t)std::max<int64_t>(nnz, 1));
  check(launch_relabel_weights(d_row, d_w, d_order, wb.row.p, wb.wt.p, n, st));
  if (wb.directed) {
    wb.irow.alloc((size_t)n + 1);
    wb.icol.alloc((size_t)std::max<int64_t>(nnz, 1));
    wb.iwt.alloc((size_t)std::max<int64_t>(nnz, 1));
    DBuf<int64_t> work((size_t)n + 1), tmp((size_t)scan_tmp_elems((int64_t)n + 1));
    check(launch_transpose(wb.row.p, wb.col.p, n, wb.irow.p, wb.icol.p, work.p, tmp.p, st, wb.wt.p,
                           wb.iwt.p));
  }
  check(hipStreamSynchronize(st));
  h_row.reset();
  h_col.reset();
  h_order.reset();
  h_w.reset();
  const auto t2 = Clock::now();
  wb.pruned(ix);
  const int64_t pr_ns = ns_since(t2);
  if (wb.parents) {
    ix->parents = true;
    ix->ord.alloc((size_t)std::max<int32_t>(n, 1));
    check(launch_invert_rank(ix->rank.p, ix->ord.p, n, st));
  }
  ix->err.alloc(1);
  check(hipMemsetAsync(ix->err.p, 0, sizeof(int32_t), st));
  ix->g_entries.assign(1, ix->entries);
  ix->hoff.clear();
  check(hipStreamSynchronize(st));
  int64_t *S = ix->stats;
  S[PLL_STAT_N] = n;
  S[PLL_STAT_TBP] = 0;
  S[PLL_STAT_ENTRIES] = ix->entries;
  S[PLL_STAT_ROOTS] = (int64_t)n * (wb.directed ? 2 : 1);
  S[PLL_STAT_VISITED] = wb.stat_proc;
  S[PLL_STAT_CANDIDATES] = wb.stat_cand;
  S[PLL_STAT_WINDOWS] = wb.stat_windows;
  S[PLL_STAT_RETRIES] = wb.stat_retries;
  S[PLL_STAT_LEVELS] = wb.stat_steps;
  S[PLL_STAT_INDEX_BYTES] = (int64_t)(ix->rank.bytes() + ix->off.bytes() + ix->went.bytes() +
                                      ix->ioff.bytes() + ix->iwent.bytes() + ix->par.bytes() +
                                      ix->ipar.bytes() + ix->ord.bytes());
  S[PLL_STAT_PRUNED_NS] = pr_ns;
  S[PLL_STAT_NORMAL_TESTS] = wb.stat_tests;
  S[PLL_STAT_LABEL_SCANNED] = wb.stat_scanned;
  S[PLL_STAT_EDGES] = wb.stat_edges;
  S[PLL_STAT_LEVEL_LAUNCHES] = wb.stat_step_launches;
  S[PLL_STAT_LEVEL_NS] = wb.stat_level_ns;
  S[PLL_STAT_IMPROVED] = wb.stat_improved;
  S[PLL_STAT_TOUCHED] = wb.stat_touched;
  S[PLL_STAT_FILTERED] = wb.stat_filtered;
  S[PLL_STAT_LAND_CHECKS] = wb.stat_checked;
  S[PLL_STAT_BUILD_NS] = ns_since(t0);
  return PLL_OK;
}

// Query pairs handed to a batch build (pll_build_query_batch): device
// memory, graph g's pairs at pairs[2 qoff[g] ..), answers at out[qoff[g] ..).
struct QueryJob {
  const int32_t *pairs = nullptr;
  uint8_t *out = nullptr;
  std::vector<int64_t> qoff;
};

int build_graphs(int32_t G, const std::vector<int64_t> &vtx_off, const int32_t *row_ptr,
                 const int32_t *col, const int32_t *order, int64_t nnz, int32_t t_bp,
                 uint32_t flags, hipStream_t st, pll_index *ix, DBuf<int64_t> *d_vtx_off,
                 DBuf<int32_t> *gid, const QueryJob *job = nullptr) {
  const auto t0 = Clock::now();
  const int32_t n = (int32_t)vtx_off[G];
  Builder b;
  b.st = st;
  b.tu = tuning();
  b.plain = (flags & PLL_PLAIN) != 0;
  b.parents = (flags & PLL_PARENTS) != 0;
  b.directed = (flags & PLL_DIRECTED) != 0;
  ix->directed = b.directed;
  b.G = G;
  b.vtx_off = vtx_off;
  if (d_vtx_off && d_vtx_off->p) b.d_vtx_off = std::move(*d_vtx_off);
  b.n = n;
  b.t = t_bp;
  b.nwords = (n + 31) / 32;
  b.nnz = nnz;
  ix->n = n;
  ix->t = t_bp;
  if (job) {
    b.qpairs = job->pairs;
    b.qout = job->out;
    b.qoff = job->qoff;
  }
  b.relabel(row_ptr, col, order, (flags & PLL_DEVICE_PTRS) != 0, ix, gid);
  const auto t1 = Clock::now();
  b.bit_parallel(ix);
  const int64_t bp_ns = ns_since(t1);
  const auto t2 = Clock::now();
  b.pruned(ix);
  const int64_t pr_ns = ns_since(t2);
  if (b.parents) {
    ix->parents = true;
    ix->grow = std::move(b.row);
    ix->gcol = std::move(b.col);
    ix->ord.alloc((size_t)std::max<int32_t>(n, 1));
    check(launch_invert_rank(ix->rank.p, ix->ord.p, n, st));
  }
  ix->err.alloc(1);
  check(hipMemsetAsync(ix->err.p, 0, sizeof(int32_t), st));
  {
    // entries per graph (for export sizes): label lengths by global rank
    std::vector<int64_t> &hoff = ix->hoff;
    hoff.assign((size_t)n + 1, 0);
    if (n) d2h(hoff.data(), ix->off.p, (size_t)n + 1, st);
    check(hipStreamSynchronize(st));
    ix->g_entries.assign((size_t)G, 0);
    for (int32_t g = 0; g < G; g++) {
      const int64_t ng = vtx_off[g + 1] - vtx_off[g];
      for (int64_t l = 0; l < ng; l++) {
        const int64_t r = ix->grank(g, l);
        ix->g_entries[g] += hoff[r + 1] - hoff[r] - 1;
      }
    }
  }
  check(hipStreamSynchronize(st));
  int64_t bp_used = 0;
  for (size_t i = 0; i < ix->bp_root.size(); i++)
    bp_used += (ix->bp_root[i] >= 0 ? 1 : 0) + ix->bp_nsel[i];
  int64_t *S = ix->stats;
  ix->level_trace = std::move(b.level_trace);
  S[PLL_STAT_N] = n;
  S[PLL_STAT_TBP] = t_bp;
  S[PLL_STAT_ENTRIES] = ix->entries;
  S[PLL_STAT_BP_USED] = bp_used;
  S[PLL_STAT_ROOTS] = b.stat_roots;
  S[PLL_STAT_VISITED] = b.stat_visited;
  S[PLL_STAT_CANDIDATES] = b.stat_cand;
  S[PLL_STAT_WINDOWS] = b.stat_windows;
  S[PLL_STAT_RETRIES] = b.stat_retries;
  S[PLL_STAT_BP_VISITED] = b.stat_bp_visited;
  S[PLL_STAT_LEVELS] = b.stat_levels;
  S[PLL_STAT_INDEX_BYTES] = (int64_t)(ix->rank.bytes() + ix->rgid.bytes() + ix->bpd.bytes() +
                                      ix->bpm.bytes() +
                                      ix->off.bytes() + ix->hub.bytes() + ix->dist.bytes() +
                                      ix->par.bytes() + ix->grow.bytes() + ix->gcol.bytes() +
                                      ix->ord.bytes() + ix->ioff.bytes() + ix->ihub.bytes() + ix->ipar.bytes() +
                                      ix->idist.bytes());
  S[PLL_STAT_BP_NS] = bp_ns;
  S[PLL_STAT_PRUNED_NS] = pr_ns;
  S[PLL_STAT_NORMAL_TESTS] = b.stat_tests;
  S[PLL_STAT_LABEL_SCANNED] = b.stat_scanned;
  S[PLL_STAT_EDGES] = b.stat_edges;
  S[PLL_STAT_TASK_EDGES] = b.stat_hedges;
  S[PLL_STAT_LEVEL_LAUNCHES] = b.stat_level_launches;
  S[PLL_STAT_LEVEL_NS] = b.stat_level_ns;
  S[PLL_STAT_BP_DIRECT] = b.stat_bp_direct;
  S[PLL_STAT_BP_SETS] = b.stat_bp_sets;
  S[PLL_STAT_BP_CHECKS] = b.stat_bp_checks;
  S[PLL_STAT_EARLIER_ROOT] = b.stat_earlier;
  S[PLL_STAT_EXPAND_NS] = b.stat_expand_ns;
  S[PLL_STAT_EXPAND_DIRECT] = b.stat_x_direct;
  S[PLL_STAT_EXPAND_EARLIER] = b.stat_x_earlier;
  S[PLL_STAT_EXPAND_CLAIMS] = b.stat_x_claims;
  S[PLL_STAT_WHOLE_GRAPHS] = (int64_t)b.whole.size();
  S[PLL_STAT_WHOLE_NS] = b.stat_whole_ns;
  S[PLL_STAT_WHOLE_PAIRS] = b.stat_whole_pairs;
  S[PLL_STAT_BUILD_NS] = ns_since(t0);
  return PLL_OK;
}

template <typename F>
int guarded(F &&fn) {
  try {
    return fn();
  } catch (const Fail &f) {
    (void)hipGetLastError();
    return f.code;
  } catch (const std::bad_alloc &) {
    return PLL_E_NOMEM;
  } catch (...) {
    return PLL_E_DEVICE;
  }
}

}  // namespace

// accessors for the serving loop (serve.hip)
namespace pll {
DIndex index_view(const pll_index *idx) { return idx->view(); }
int32_t index_n(const pll_index *idx) { return idx->n; }
bool index_weighted(const pll_index *idx) { return idx->weighted; }
int32_t *index_err(const pll_index *idx) { return idx->err.p; }
int64_t query_group_size() { return tuning().qgroup; }
bool query_persistent() { return tuning().qpersist != 0; }
int64_t serve_coalesce() { return tuning().serve_coalesce; }
}  // namespace pll

// ---------------------------------------------------------------------------
// ABI

extern "C" {

static int build_entry(int32_t G, const int64_t *vtx_off, const int32_t *row_ptr,
                       const int32_t *col, const int32_t *order, int32_t t_bp, uint32_t flags,
                       void *stream, pll_index **out, const QueryJob *job = nullptr) {
  if (!out) return PLL_E_INVAL;
  *out = nullptr;
  hipStream_t st = (hipStream_t)stream;
  const AllocStream alloc_stream(st);
  const bool device = (flags & PLL_DEVICE_PTRS) != 0;
  if (G < 0 || t_bp < 0 || t_bp > PLL_MAX_TBP || (G > 0 && !vtx_off)) return PLL_E_INVAL;
  // directed graphs: no bit-parallel labels
  if ((flags & PLL_DIRECTED) && t_bp > 0) return PLL_E_UNSUPPORTED;
  std::vector<int64_t> voff(vtx_off, vtx_off + (G > 0 ? G + 1 : 0));
  if (G == 0) voff.assign(1, 0);
  if (voff[0] != 0) return PLL_E_INVAL;
  for (int32_t g = 0; g < G; g++)
    if (voff[g + 1] < voff[g]) return PLL_E_INVAL;
  const int64_t N = voff.back();
  if (N > INT32_MAX - 1) return PLL_E_INVAL;
  int64_t nnz = 0;
  DBuf<int64_t> d_voff;
  DBuf<int32_t> gid;
  if (!device) {
    // symmetry is the undirected precondition; a directed graph has none
    int rc = validate_batch(G, vtx_off, row_ptr, col, order, t_bp,
                            (flags & PLL_VALIDATE) != 0 && !(flags & PLL_DIRECTED));
    if (rc != PLL_OK) return rc;
    nnz = N > 0 ? row_ptr[N] : 0;
  } else {
    if (flags & PLL_VALIDATE) return PLL_E_UNSUPPORTED;
    if (N > 0 && (!row_ptr || !order)) return PLL_E_INVAL;
    if (N > 0) {
      int rc = guarded([&] {
        int32_t hn = 0, h0 = 0;
        d2h(&hn, row_ptr + N, 1, st);
        d2h(&h0, row_ptr, 1, st);
        check(hipStreamSynchronize(st));
        nnz = hn;
        if (h0 != 0 || nnz < 0 || (nnz > 0 && !col)) return PLL_E_INVAL;
        d_voff.alloc((size_t)std::max(G, 1) + 1);
        h2d(d_voff.p, voff.data(), voff.size(), st);
        gid.alloc((size_t)N);
        check(launch_fill_gid(d_voff.p, G, gid.p, st));
        DBuf<uint32_t> seen((size_t)(N + 31) / 32);
        DBuf<int32_t> err(1);
        fill(seen, 0, st);
        fill(err, 0, st);
        check(launch_validate_graph((int32_t)N, row_ptr, col, order, gid.p, d_voff.p, seen.p,
                                    err.p, st));
        int32_t herr = 0;
        d2h(&herr, err.p, 1, st);
        check(hipStreamSynchronize(st));
        return herr ? PLL_E_INVAL : PLL_OK;
      });
      if (rc != PLL_OK) return rc;
    }
  }
  pll_index *ix = new (std::nothrow) pll_index();
  if (!ix) return PLL_E_NOMEM;
  const int32_t Gb = G > 0 ? G : 1;
  if (G == 0) voff.push_back(0);
  int rc = guarded([&] {
    return build_graphs(Gb, voff, row_ptr, col, order, nnz, t_bp, flags, st, ix, &d_voff, &gid,
                        job);
  });
  if (rc != PLL_OK) {
    (void)hipStreamSynchronize(st);
    delete ix;
    return rc;
  }
  *out = ix;
  return PLL_OK;
}

int pll_set_allocator(void *(*alloc)(size_t, void *, void *), void (*free_)(void *, void *, void *),
                      void *ctx) {
  if ((alloc == nullptr) != (free_ == nullptr)) return PLL_E_INVAL;
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_alloc_hook = AllocHook{alloc, free_, alloc ? ctx : nullptr};
  return PLL_OK;
}

int pll_build(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *order,
              int32_t t_bp, uint32_t flags, void *stream, pll_index **out) {
  if (n < 0) return PLL_E_INVAL;
  const int64_t voff[2] = {0, n};
  return build_entry(1, voff, row_ptr, col, order, t_bp, flags, stream, out);
}

int pll_build_batch(int32_t G, const int64_t *vtx_off, const int32_t *row_ptr, const int32_t *col,
                    const int32_t *order, int32_t t_bp, uint32_t flags, void *stream,
                    pll_index **out) {
  return build_entry(G, vtx_off, row_ptr, col, order, t_bp, flags, stream, out);
}

int pll_build_query_batch(int32_t G, const int64_t *vtx_off, const int32_t *row_ptr,
                          const int32_t *col, const int32_t *order, int32_t t_bp,
                          const int64_t *qoff, const int32_t *pairs, uint8_t *out,
                          uint32_t flags, void *stream, pll_index **idx) {
  if (!idx) return PLL_E_INVAL;
  *idx = nullptr;
  if (G < 0 || (G > 0 && (!vtx_off || !qoff))) return PLL_E_INVAL;
  if (G > 0 && qoff[0] != 0) return PLL_E_INVAL;
  for (int32_t g = 0; g < G; g++)
    if (qoff[g + 1] < qoff[g]) return PLL_E_INVAL;
  const int64_t q = G > 0 ? qoff[G] : 0;
  if (q > 0 && (!pairs || !out)) return PLL_E_INVAL;
  if (q > INT64_MAX / 4) return PLL_E_INVAL;
  hipStream_t st = (hipStream_t)stream;
  const AllocStream alloc_stream(st);
  const bool device = (flags & PLL_DEVICE_PTRS) != 0;
  if (!device) {
    // every pair inside its graph (before any device work)
    for (int32_t g = 0; g < G; g++) {
      if (vtx_off[g + 1] < vtx_off[g]) return PLL_E_INVAL;
      for (int64_t i = 2 * qoff[g]; i < 2 * qoff[g + 1]; i++)
        if (pairs[i] < vtx_off[g] || pairs[i] >= vtx_off[g + 1]) return PLL_E_INVAL;
    }
  } else if (q > 0) {
    const int64_t N = vtx_off[G];
    if (N <= 0 || N > INT32_MAX - 1) return PLL_E_INVAL;
    int rc = guarded([&] {
      DBuf<int32_t> err(1);
      fill(err, 0, st);
      check(launch_validate_pairs(pairs, q, (int32_t)N, err.p, st));
      int32_t herr = 0;
      d2h(&herr, err.p, 1, st);
      check(hipStreamSynchronize(st));
      return herr ? PLL_E_INVAL : PLL_OK;
    });
    if (rc != PLL_OK) return rc;
  }
  pll_index *ix = nullptr;
  int rc = guarded([&]() -> int {
    DBuf<int32_t> hp;
    DBuf<uint8_t> hout;
    QueryJob job;
    job.qoff.assign(qoff, qoff + (G > 0 ? G + 1 : 0));
    job.pairs = pairs;
    job.out = out;
    if (!device && q > 0) {
      hp.alloc((size_t)(2 * q));
      hout.alloc((size_t)q);
      h2d(hp.p, pairs, (size_t)(2 * q), st);
      job.pairs = hp.p;
      job.out = hout.p;
    }
    if (q == 0) job.pairs = nullptr;
    int brc = build_entry(G, vtx_off, row_ptr, col, order, t_bp, flags, stream, &ix,
                          job.pairs ? &job : nullptr);
    if (brc != PLL_OK) return brc;
    // pairs of the graphs not built whole: one batched launch per run of
    // consecutive such graphs, over the finished index
    const Tuning tu = tuning();
    for (int32_t g = 0; q > 0 && g < G;) {
      if (ix->gblk[g] >= 0) {
        g++;
        continue;
      }
      int32_t g1 = g;
      while (g1 < G && ix->gblk[g1] < 0) g1++;
      const int64_t a = qoff[g], nq = qoff[g1] - qoff[g];
      if (nq > 0)
        check(launch_query(ix->view(), job.pairs + 2 * a, nq, job.out + a, nullptr, false,
                           tu.qgroup, st, nullptr));
      g = g1;
    }
    if (!device && q > 0) d2h(out, job.out, (size_t)q, st);
    if (!device || (flags & PLL_SYNC)) check(hipStreamSynchronize(st));
    return PLL_OK;
  });
  if (rc != PLL_OK) {
    if (ix) {
      (void)hipStreamSynchronize(st);
      pll_free(ix);
    }
    return rc;
  }
  *idx = ix;
  return PLL_OK;
}

int pll_build_weighted(int32_t n, const int32_t *row_ptr, const int32_t *col, const uint32_t *wgt,
                       const int32_t *order, uint32_t flags, void *stream, pll_index **out) {
  if (!out) return PLL_E_INVAL;
  *out = nullptr;
  if (n < 0) return PLL_E_INVAL;
  hipStream_t st = (hipStream_t)stream;
  const AllocStream alloc_stream(st);
  const bool device = (flags & PLL_DEVICE_PTRS) != 0;
  const bool directed = (flags & PLL_DIRECTED) != 0;
  int64_t nnz = 0;
  if (!device) {
    const int64_t voff[2] = {0, n};
    int rc = validate_batch(1, voff, row_ptr, col, order, 0, false);
    if (rc != PLL_OK) return rc;
    nnz = n > 0 ? row_ptr[n] : 0;
    rc = validate_weights(n, row_ptr, col, wgt, (flags & PLL_VALIDATE) != 0 && !directed);
    if (rc != PLL_OK) return rc;
  } else {
    if (flags & PLL_VALIDATE) return PLL_E_UNSUPPORTED;
    if (n > 0 && (!row_ptr || !order)) return PLL_E_INVAL;
    if (n > 0) {
      int rc = guarded([&] {
        int32_t hn = 0, h0 = 0;
        d2h(&hn, row_ptr + n, 1, st);
        d2h(&h0, row_ptr, 1, st);
        check(hipStreamSynchronize(st));
        nnz = hn;
        if (h0 != 0 || nnz < 0 || (nnz > 0 && (!col || !wgt))) return PLL_E_INVAL;
        const std::vector<int64_t> voff = {0, (int64_t)n};
        DBuf<int64_t> d_voff(2);
        h2d(d_voff.p, voff.data(), 2, st);
        DBuf<int32_t> gid((size_t)n);
        check(launch_fill_gid(d_voff.p, 1, gid.p, st));
        DBuf<uint32_t> seen((size_t)(n + 31) / 32);
        DBuf<int32_t> err(1);
        fill(seen, 0, st);
        fill(err, 0, st);
        check(launch_validate_graph(n, row_ptr, col, order, gid.p, d_voff.p, seen.p, err.p, st));
        check(launch_validate_weights(wgt, nnz, err.p, st));
        int32_t herr = 0;
        d2h(&herr, err.p, 1, st);
        check(hipStreamSynchronize(st));
        return herr ? PLL_E_INVAL : PLL_OK;
      });
      if (rc != PLL_OK) return rc;
    }
  }
  pll_index *ix = new (std::nothrow) pll_index();
  if (!ix) return PLL_E_NOMEM;
  int rc = guarded([&] { return build_weighted(n, row_ptr, col, wgt, order, nnz, flags, st, ix); });
  if (rc != PLL_OK) {
    (void)hipStreamSynchronize(st);
    delete ix;
    return rc;
  }
  *out = ix;
  return PLL_OK;
}

int pll_export_weighted_parents(const pll_index *idx, int32_t side, uint32_t *par) {
  if (!idx || side < 0 || side > 1 || !par) return PLL_E_INVAL;
  if (!idx->weighted || !idx->parents || (side == 1 && !idx->directed)) return PLL_E_UNSUPPORTED;
  return guarded([&] {
    hipStream_t st = nullptr;
    const int32_t n = idx->n;
    const DBuf<int64_t> &doff = side ? idx->ioff : idx->off;
    const DBuf<uint32_t> &dpar = side ? idx->ipar : idx->par;
    std::vector<int64_t> ho((size_t)n + 1, 0);
    if (n) d2h(ho.data(), doff.p, (size_t)n + 1, st);
    check(hipStreamSynchronize(st));
    const int64_t total = n ? ho[n] : 0;
    if (total <= n) return PLL_OK;
    std::vector<uint32_t> hp((size_t)total);
    d2h(hp.data(), dpar.p, (size_t)total, st);
    check(hipStreamSynchronize(st));
    int64_t o = 0;
    for (int32_t r = 0; r < n; r++)
      for (int64_t e = ho[r]; e < ho[r + 1] - 1; e++) par[o++] = hp[e];
    return PLL_OK;
  });
}

int pll_query_weighted(const pll_index *idx, const int32_t *pairs, int64_t q, uint32_t *out,
                       uint32_t flags, void *stream) {
  if (!idx || q < 0) return PLL_E_INVAL;
  if (!idx->weighted) return PLL_E_UNSUPPORTED;
  if (q == 0) return PLL_OK;
  if (!pairs || !out) return PLL_E_INVAL;
  hipStream_t st = (hipStream_t)stream;
  const AllocStream alloc_stream(st);
  const Tuning tu = tuning();
  const bool plain = (flags & PLL_PLAIN) != 0;
  if (!(flags & PLL_DEVICE_PTRS)) {
    for (int64_t i = 0; i < 2 * q; i++)
      if (pairs[i] < 0 || pairs[i] >= idx->n) return PLL_E_INVAL;
    return guarded([&] {
      DBuf<int32_t> dp((size_t)(2 * q));
      DBuf<uint32_t> dout((size_t)q);
      h2d(dp.p, pairs, (size_t)(2 * q), st);
      check(launch_wquery(idx->view(), dp.p, q, dout.p, nullptr, plain, tu.qgroup, st));
      d2h(out, dout.p, (size_t)q, st);
      check(hipStreamSynchronize(st));
      return PLL_OK;
    });
  }
  return guarded([&] {
    int32_t *err = nullptr;
    check(hipMallocAsync((void **)&err, sizeof(int32_t), st));
    check(hipMemsetAsync(err, 0, sizeof(int32_t), st));
    check(launch_validate_pairs(pairs, q, idx->n, err, st));
    check(launch_wquery(idx->view(), pairs, q, out, err, plain, tu.qgroup, st));
    int32_t herr = 0;
    if (flags & PLL_SYNC) {
      check(hipMemcpyAsync(&herr, err, sizeof(int32_t), hipMemcpyDeviceToHost, st));
      check(hipFreeAsync(err, st));
      check(hipStreamSynchronize(st));
      return herr ? PLL_E_INVAL : PLL_OK;
    }
    check(launch_or_flag(err, idx->err.p, st));
    check(hipFreeAsync(err, st));
    return PLL_OK;
  });
}

int pll_export_weighted(const pll_index *idx, int32_t side, int64_t *entries, int64_t *off,
                        uint32_t *hub, uint32_t *dist, int32_t *rank) {
  if (!idx || side < 0 || side > 1) return PLL_E_INVAL;
  if (!idx->weighted || (side == 1 && !idx->directed)) return PLL_E_UNSUPPORTED;
  return guarded([&] {
    hipStream_t st = nullptr;
    const int32_t n = idx->n;
    const DBuf<int64_t> &doff = side ? idx->ioff : idx->off;
    const DBuf<uint64_t> &dent = side ? idx->iwent : idx->went;
    std::vector<int64_t> ho((size_t)n + 1, 0);
    if (n) d2h(ho.data(), doff.p, (size_t)n + 1, st);
    check(hipStreamSynchronize(st));
    const int64_t total = n ? ho[n] : 0;
    if (entries) *entries = total - n;
    if (off) {
      for (int32_t r = 0; r <= n; r++) off[r] = ho[r] - r;  // without sentinels
    }
    if ((hub || dist) && total > n) {
      std::vector<uint64_t> he((size_t)total);
      d2h(he.data(), dent.p, (size_t)total, st);
      check(hipStreamSynchronize(st));
      int64_t o = 0;
      for (int32_t r = 0; r < n; r++)
        for (int64_t e = ho[r]; e < ho[r + 1] - 1; e++, o++) {
          if (hub) hub[o] = (uint32_t)(he[e] >> 32);
          if (dist) dist[o] = (uint32_t)he[e];
        }
    }
    if (rank && n) {
      d2h(rank, idx->rank.p, (size_t)n, st);
      check(hipStreamSynchronize(st));
    }
    return PLL_OK;
  });
}

int pll_query(const pll_index *idx, const int32_t *pairs, int64_t q, uint8_t *out, uint32_t flags,
              void *stream) {
  if (!idx || q < 0) return PLL_E_INVAL;
  if (idx->weighted) return PLL_E_UNSUPPORTED;
  if (q == 0) return PLL_OK;
  if (!pairs || !out) return PLL_E_INVAL;
  hipStream_t st = (hipStream_t)stream;
  const AllocStream alloc_stream(st);
  const Tuning tu = tuning();
  const bool plain = (flags & PLL_PLAIN) != 0;
  if (!(flags & PLL_DEVICE_PTRS)) {
    for (int64_t i = 0; i < 2 * q; i++)
      if (pairs[i] < 0 || pairs[i] >= idx->n) return PLL_E_INVAL;
    return guarded([&] {
      DBuf<int32_t> dp((size_t)(2 * q));
      DBuf<uint8_t> dout((size_t)q);
      DBuf<unsigned long long> cur(1);
      h2d(dp.p, pairs, (size_t)(2 * q), st);
      check(launch_query(idx->view(), dp.p, q, dout.p, nullptr, plain, tu.qgroup, st,
                         tu.qpersist ? cur.p : nullptr));
      d2h(out, dout.p, (size_t)q, st);
      check(hipStreamSynchronize(st));
      return PLL_OK;
    });
  }
  return guarded([&] {
    // the call's error flag, and with the persistent form its work cursor
    int32_t *err = nullptr;
    check(hipMallocAsync((void **)&err, 16, st));
    check(hipMemsetAsync(err, 0, 16, st));
    unsigned long long *cur =
        tu.qpersist ? reinterpret_cast<unsigned long long *>(reinterpret_cast<char *>(err) + 8)
                    : nullptr;
    check(launch_validate_pairs(pairs, q, idx->n, err, st));
    check(launch_query(idx->view(), pairs, q, out, err, plain, tu.qgroup, st, cur));
    int32_t herr = 0;
    if (flags & PLL_SYNC) {
      check(hipMemcpyAsync(&herr, err, sizeof(int32_t), hipMemcpyDeviceToHost, st));
      check(hipFreeAsync(err, st));
      check(hipStreamSynchronize(st));
      return herr ? PLL_E_INVAL : PLL_OK;
    }
    // fold this call's outcome into the index's sticky error
    check(launch_or_flag(err, idx->err.p, st));
    check(hipFreeAsync(err, st));
    return PLL_OK;
  });
}

int pll_query_batch(const pll_index *idx, const int32_t *pairs, int64_t q, uint8_t *out,
                    uint32_t flags, void *stream) {
  return pll_query(idx, pairs, q, out, flags, stream);
}

}  // extern "C"

struct pll_qgraph {
  int32_t *flag = nullptr;  // error flag at +0, persistent-form cursor at +8
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~pll_qgraph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (flag) (void)hipFree(flag);
  }
};

extern "C" {

int pll_query_graph_create(const pll_index *idx, const int32_t *pairs, int64_t q, uint8_t *out,
                           uint32_t flags, pll_qgraph **g) {
  if (!g) return PLL_E_INVAL;
  *g = nullptr;
  if (!idx || q < 0 || !(flags & PLL_DEVICE_PTRS) || (q > 0 && (!pairs || !out)))
    return PLL_E_INVAL;
  if (idx->weighted) return PLL_E_UNSUPPORTED;
  const Tuning tu = tuning();
  const bool plain = (flags & PLL_PLAIN) != 0;
  auto qg = std::make_unique<pll_qgraph>();
  if (hipMalloc((void **)&qg->flag, 16) != hipSuccess) {
    (void)hipGetLastError();
    qg->flag = nullptr;
    return PLL_E_NOMEM;
  }
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return PLL_E_DEVICE;
  unsigned long long *cur =
      tu.qpersist ? reinterpret_cast<unsigned long long *>(reinterpret_cast<char *>(qg->flag) + 8)
                  : nullptr;
  // the recorded launches: clear the flag (a kernel, not a memset), check
  // the ids, answer the pairs
  bool ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    ok = launch_zero_flag(qg->flag, cs) == hipSuccess &&
         launch_validate_pairs(pairs, q, idx->n, qg->flag, cs) == hipSuccess &&
         launch_query(idx->view(), pairs, q, out, qg->flag, plain, tu.qgroup, cs, cur) ==
             hipSuccess;
    ok = hipStreamEndCapture(cs, &qg->graph) == hipSuccess && ok;
  }
  ok = ok && hipGraphInstantiate(&qg->exec, qg->graph, nullptr, nullptr, 0) == hipSuccess;
  (void)hipStreamDestroy(cs);
  if (!ok) {
    (void)hipGetLastError();
    return PLL_E_DEVICE;
  }
  *g = qg.release();
  return PLL_OK;
}

int pll_query_graph_launch(pll_qgraph *g, void *stream) {
  if (!g) return PLL_E_INVAL;
  return hipGraphLaunch(g->exec, (hipStream_t)stream) == hipSuccess ? PLL_OK : PLL_E_DEVICE;
}

int pll_query_graph_status(pll_qgraph *g, void *stream) {
  if (!g) return PLL_E_INVAL;
  int32_t herr = 0;
  if (hipMemcpyAsync(&herr, g->flag, sizeof(int32_t), hipMemcpyDeviceToHost,
                     (hipStream_t)stream) != hipSuccess ||
      hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
    return PLL_E_DEVICE;
  return herr ? PLL_E_INVAL : PLL_OK;
}

void pll_query_graph_free(pll_qgraph *g) { delete g; }

int pll_autotune_query(const pll_index *idx, const int32_t *pairs, int64_t q, uint32_t flags,
                       void *stream, int32_t *best) {
  if (!idx || q <= 0 || !pairs) return PLL_E_INVAL;
  hipStream_t st = (hipStream_t)stream;
  const AllocStream alloc_stream(st);
  const bool device = (flags & PLL_DEVICE_PTRS) != 0;
  if (!device)
    for (int64_t i = 0; i < 2 * q; i++)
      if (pairs[i] < 0 || pairs[i] >= idx->n) return PLL_E_INVAL;
  return guarded([&] {
    DBuf<int32_t> dp;
    const int32_t *pp = pairs;
    if (!device) {
      dp.alloc((size_t)(2 * q));
      h2d(dp.p, pairs, (size_t)(2 * q), st);
      pp = dp.p;
    } else {
      // device ids are validated first, as in pll_query
      DBuf<int32_t> err(1);
      fill(err, 0, st);
      check(launch_validate_pairs(pairs, q, idx->n, err.p, st));
      int32_t herr = 0;
      d2h(&herr, err.p, 1, st);
      check(hipStreamSynchronize(st));
      if (herr) return PLL_E_INVAL;
    }
    DBuf<uint32_t> out((size_t)q);  // room for 8- or 32-bit answers
    DBuf<unsigned long long> cur(1);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    check(hipEventCreate(&e0));
    check(hipEventCreate(&e1));
    struct EvGuard {
      hipEvent_t a, b;
      ~EvGuard() {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
      }
    } evg{e0, e1};
    const DIndex v = idx->view();
    auto launch = [&](int g, bool persist) {
      if (idx->weighted)
        check(launch_wquery(v, pp, q, out.p, nullptr, false, g, st));
      else
        check(launch_query(v, pp, q, reinterpret_cast<uint8_t *>(out.p), nullptr, false, g, st,
                           persist ? cur.p : nullptr));
    };
    // lanes per pair, and for unweighted indexes the static or the
    // persistent batched form
    int32_t choice = 64;
    bool pchoice = false;
    float best_ms = 0.f;
    bool first = true;
    for (int persist = 0; persist < (idx->weighted ? 1 : 2); persist++) {
      for (int g : {16, 32, 64}) {
        launch(g, persist);  // warm
        check(hipEventRecord(e0, st));
        for (int r = 0; r < 3; r++) launch(g, persist);
        check(hipEventRecord(e1, st));
        check(hipEventSynchronize(e1));
        float ms = 0.f;
        check(hipEventElapsedTime(&ms, e0, e1));
        if (first || ms < best_ms) {
          best_ms = ms;
          choice = g;
          pchoice = persist != 0;
          first = false;
        }
      }
    }
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tune.qgroup = choice;
      if (!idx->weighted) g_tune.qpersist = pchoice ? 1 : 0;
    }
    if (best) *best = choice;
    return PLL_OK;
  });
}

int pll_autotune_build(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *order,
                       int32_t t_bp, uint32_t flags, void *stream, int64_t *best) {
  if (flags & (PLL_PLAIN | PLL_PARENTS)) return PLL_E_INVAL;
  // coordinate descent, one knob at a time from the current settings, two
  // passes over the knobs; every candidate is one whole build (the labels
  // never depend on the knobs)
  struct Knob {
    const char *name;
    std::vector<int64_t> cands;
  };
  const std::vector<Knob> knobs = {
      {"xgroup", {8, 16, 32}},
      {"chunk", {128, 256, 512}},
      {"window_work", {64000000, 128000000, 256000000}},
      {"sort_level", {1 << 18, 1 << 20, 1 << 22}},
  };
  std::map<std::string, int64_t> chosen;
  // two passes: a knob's best value can move once the others have moved
  for (int pass = 0; pass < 2; pass++)
  for (const Knob &k : knobs) {
    const int64_t start = pll_get_tuning(k.name);
    int64_t pick = start;
    double pick_s = 0;
    bool first = true;
    for (int64_t c : k.cands) {
      if (pll_set_tuning(k.name, c) != PLL_OK) continue;
      pll_index *ix = nullptr;
      const auto t0 = Clock::now();
      const int rc = pll_build(n, row_ptr, col, order, t_bp, flags, stream, &ix);
      const double secs = ns_since(t0) * 1e-9;
      pll_free(ix);
      if (rc != PLL_OK) {
        pll_set_tuning(k.name, start);
        return rc;
      }
      if (first || secs < pick_s) {
        pick = c;
        pick_s = secs;
        first = false;
      }
    }
    pll_set_tuning(k.name, pick);
    chosen[k.name] = pick;
  }
  if (best) {
    best[0] = chosen["xgroup"];
    best[1] = chosen["chunk"];
    best[2] = chosen["window_work"];
    best[3] = chosen["sort_level"];
  }
  return PLL_OK;
}

int pll_sync(const pll_index *idx, void *stream) {
  if (!idx) return PLL_E_INVAL;
  hipStream_t st = (hipStream_t)stream;
  return guarded([&] {
    int32_t herr = 0;
    check(hipMemcpyAsync(&herr, idx->err.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    check(hipMemsetAsync(idx->err.p, 0, sizeof(int32_t), st));
    check(hipStreamSynchronize(st));
    return herr ? PLL_E_INVAL : PLL_OK;
  });
}

int pll_export_sizes(const pll_index *idx, int32_t graph, int64_t *n, int64_t *entries,
                     int32_t *t_bp) {
  if (!idx || graph < 0 || graph >= idx->G) return PLL_E_INVAL;
  if (n) *n = idx->vtx_off[graph + 1] - idx->vtx_off[graph];
  if (entries) *entries = idx->g_entries.empty() ? 0 : idx->g_entries[graph];
  if (t_bp) *t_bp = idx->t;
  return PLL_OK;
}

int pll_query_path(const pll_index *idx, const int32_t *pairs, int64_t q, int32_t max_len,
                   int32_t *paths, int32_t *lens, uint32_t flags, void *stream) {
  if (!idx || q < 0 || max_len < 0) return PLL_E_INVAL;
  if (!idx->parents) return PLL_E_UNSUPPORTED;
  if (q == 0) return PLL_OK;
  if (!pairs || !lens || (max_len > 0 && !paths)) return PLL_E_INVAL;
  hipStream_t st = (hipStream_t)stream;
  const AllocStream alloc_stream(st);
  if (!(flags & PLL_DEVICE_PTRS)) {
    for (int64_t i = 0; i < 2 * q; i++)
      if (pairs[i] < 0 || pairs[i] >= idx->n) return PLL_E_INVAL;
    return guarded([&] {
      const size_t cells = (size_t)q * (size_t)max_len;
      DBuf<int32_t> dp((size_t)(2 * q)), dpath(std::max<size_t>(cells, 1)), dlen((size_t)q);
      h2d(dp.p, pairs, (size_t)(2 * q), st);
      // rows the kernel leaves alone come back unchanged
      if (cells) h2d(dpath.p, paths, cells, st);
      if (idx->weighted)
        check(launch_wquery_path(idx->view(), dp.p, q, max_len, dpath.p, dlen.p, nullptr, st));
      else
        check(launch_query_path(idx->view(), dp.p, q, max_len, dpath.p, dlen.p, nullptr, st));
      d2h(lens, dlen.p, (size_t)q, st);
      if (cells) d2h(paths, dpath.p, cells, st);
      check(hipStreamSynchronize(st));
      return PLL_OK;
    });
  }
  return guarded([&] {
    int32_t *err = nullptr;
    check(hipMallocAsync((void **)&err, sizeof(int32_t), st));
    check(hipMemsetAsync(err, 0, sizeof(int32_t), st));
    check(launch_validate_pairs(pairs, q, idx->n, err, st));
    if (idx->weighted)
      check(launch_wquery_path(idx->view(), pairs, q, max_len, paths, lens, err, st));
    else
      check(launch_query_path(idx->view(), pairs, q, max_len, paths, lens, err, st));
    int32_t herr = 0;
    if (flags & PLL_SYNC) {
      check(hipMemcpyAsync(&herr, err, sizeof(int32_t), hipMemcpyDeviceToHost, st));
      check(hipFreeAsync(err, st));
      check(hipStreamSynchronize(st));
      return herr ? PLL_E_INVAL : PLL_OK;
    }
    check(launch_or_flag(err, idx->err.p, st));
    check(hipFreeAsync(err, st));
    return PLL_OK;
  });
}

int pll_export_in(const pll_index *idx, int32_t graph, int64_t *entries, int64_t *off,
                  uint32_t *hub, uint8_t *dist) {
  if (!idx || graph < 0 || graph >= idx->G) return PLL_E_INVAL;
  if (!idx->directed || idx->weighted) return PLL_E_UNSUPPORTED;
  return guarded([&] {
    const int64_t g0 = idx->vtx_off[graph];
    const int64_t ng = idx->vtx_off[graph + 1] - g0;
    hipStream_t st = nullptr;
    std::vector<int64_t> hio((size_t)idx->n + 1);
    if (idx->n) d2h(hio.data(), idx->ioff.p, (size_t)idx->n + 1, st);
    check(hipStreamSynchronize(st));
    std::vector<int64_t> rows((size_t)ng), oo((size_t)ng + 1, 0);
    for (int64_t l = 0; l < ng; l++) {
      rows[l] = idx->grank(graph, l);
      oo[l + 1] = oo[l] + hio[rows[l] + 1] - 1 - hio[rows[l]];
    }
    const int64_t ne = oo[ng];
    if (entries) *entries = ne;
    if (off) std::memcpy(off, oo.data(), oo.size() * sizeof(int64_t));
    if (ne == 0 || (!hub && !dist)) return PLL_OK;
    DBuf<int64_t> drows((size_t)ng), doo((size_t)ng + 1);
    h2d(drows.p, rows.data(), (size_t)ng, st);
    h2d(doo.p, oo.data(), (size_t)ng + 1, st);
    DBuf<uint32_t> oh((size_t)ne);
    DBuf<uint8_t> od((size_t)ne);
    check(launch_gather_labels(drows.p, ng, idx->ioff.p, idx->ihub.p, idx->idist.p, idx->lrank.p,
                               doo.p, oh.p, od.p, st));
    if (hub) d2h(hub, oh.p, (size_t)ne, st);
    if (dist) d2h(dist, od.p, (size_t)ne, st);
    check(hipStreamSynchronize(st));
    return PLL_OK;
  });
}

int pll_export_parents(const pll_index *idx, int32_t graph, uint32_t *par) {
  if (!idx || graph < 0 || graph >= idx->G || !par) return PLL_E_INVAL;
  if (!idx->parents) return PLL_E_UNSUPPORTED;
  return guarded([&] {
    const int64_t g0 = idx->vtx_off[graph];
    const int64_t ng = idx->vtx_off[graph + 1] - g0;
    hipStream_t st = nullptr;
    std::vector<int64_t> rows((size_t)ng), oo((size_t)ng + 1, 0);
    for (int64_t l = 0; l < ng; l++) {
      rows[l] = idx->grank(graph, l);
      oo[l + 1] = oo[l] + idx->hoff[rows[l] + 1] - 1 - idx->hoff[rows[l]];
    }
    const int64_t ne = oo[ng];
    if (ne == 0) return PLL_OK;
    DBuf<int64_t> drows((size_t)ng), doo((size_t)ng + 1);
    h2d(drows.p, rows.data(), (size_t)ng, st);
    h2d(doo.p, oo.data(), (size_t)ng + 1, st);
    DBuf<uint32_t> op((size_t)ne);
    DBuf<uint8_t> od((size_t)ne);
    // same gather as the hubs: parents are global ranks too
    check(launch_gather_labels(drows.p, ng, idx->off.p, idx->par.p, idx->dist.p, idx->lrank.p,
                               doo.p, op.p, od.p, st));
    d2h(par, op.p, (size_t)ne, st);
    check(hipStreamSynchronize(st));
    return PLL_OK;
  });
}

int pll_export_in_parents(const pll_index *idx, int32_t graph, uint32_t *par) {
  if (!idx || graph < 0 || graph >= idx->G || !par) return PLL_E_INVAL;
  if (!idx->parents || !idx->directed || idx->weighted) return PLL_E_UNSUPPORTED;
  return guarded([&] {
    const int64_t ng = idx->vtx_off[graph + 1] - idx->vtx_off[graph];
    hipStream_t st = nullptr;
    std::vector<int64_t> hio((size_t)idx->n + 1);
    if (idx->n) d2h(hio.data(), idx->ioff.p, (size_t)idx->n + 1, st);
    check(hipStreamSynchronize(st));
    std::vector<int64_t> rows((size_t)ng), oo((size_t)ng + 1, 0);
    for (int64_t l = 0; l < ng; l++) {
      rows[l] = idx->grank(graph, l);
      oo[l + 1] = oo[l] + hio[rows[l] + 1] - 1 - hio[rows[l]];
    }
    const int64_t ne = oo[ng];
    if (ne == 0) return PLL_OK;
    DBuf<int64_t> drows((size_t)ng), doo((size_t)ng + 1);
    h2d(drows.p, rows.data(), (size_t)ng, st);
    h2d(doo.p, oo.data(), (size_t)ng + 1, st);
    DBuf<uint32_t> op((size_t)ne);
    DBuf<uint8_t> od((size_t)ne);
    // same gather as the hubs: parents are global ranks too
    check(launch_gather_labels(drows.p, ng, idx->ioff.p, idx->ipar.p, idx->idist.p, idx->lrank.p,
                               doo.p, op.p, od.p, st));
    d2h(par, op.p, (size_t)ne, st);
    check(hipStreamSynchronize(st));
    return PLL_OK;
  });
}

int pll_export(const pll_index *idx, int32_t graph, int64_t *off, uint32_t *hub, uint8_t *dist,
               uint8_t *bp_d, uint64_t *bp_m1, uint64_t *bp_0, int32_t *rank) {
  if (!idx || graph < 0 || graph >= idx->G) return PLL_E_INVAL;
  if (idx->weighted) return PLL_E_UNSUPPORTED;
  return guarded([&] {
    const int32_t t = idx->t, tp = idx->tpad;
    const int64_t g0 = idx->vtx_off[graph];
    const int64_t ng = idx->vtx_off[graph + 1] - g0;
    hipStream_t st = nullptr;
    // the graph's rows (global ranks) in local rank order, and output offsets
    std::vector<int64_t> rows((size_t)ng), oo((size_t)ng + 1, 0);
    for (int64_t l = 0; l < ng; l++) {
      rows[l] = idx->grank(graph, l);
      oo[l + 1] = oo[l] + idx->hoff[rows[l] + 1] - 1 - idx->hoff[rows[l]];
    }
    const int64_t ne = oo[ng];
    if (off) std::memcpy(off, oo.data(), oo.size() * sizeof(int64_t));
    if (ng == 0) return PLL_OK;
    DBuf<int64_t> drows((size_t)ng), doo((size_t)ng + 1);
    h2d(drows.p, rows.data(), (size_t)ng, st);
    h2d(doo.p, oo.data(), (size_t)ng + 1, st);
    if ((hub || dist) && ne > 0) {
      DBuf<uint32_t> oh((size_t)ne);
      DBuf<uint8_t> od((size_t)ne);
      check(launch_gather_labels(drows.p, ng, idx->off.p, idx->hub.p, idx->dist.p, idx->lrank.p,
                                 doo.p, oh.p, od.p, st));
      if (hub) d2h(hub, oh.p, (size_t)ne, st);
      if (dist) d2h(dist, od.p, (size_t)ne, st);
      check(hipStreamSynchronize(st));
    }
    if (t > 0 && (bp_d || bp_m1 || bp_0)) {
      const size_t nb = (size_t)ng * t;
      DBuf<uint8_t> obd(nb);
      DBuf<uint64_t> om1(nb), om0(nb);
      check(launch_gather_bp(drows.p, ng, t, tp, idx->bpd.p, idx->bpm.p, obd.p, om1.p, om0.p, st));
      if (bp_d) d2h(bp_d, obd.p, nb, st);
      if (bp_m1) d2h(bp_m1, om1.p, nb, st);
      if (bp_0) d2h(bp_0, om0.p, nb, st);
      check(hipStreamSynchronize(st));
    }
    if (rank) {
      DBuf<int32_t> orank((size_t)ng);
      check(launch_gather_rank(g0, ng, idx->rank.p, idx->lrank.p, orank.p, st));
      d2h(rank, orank.p, (size_t)ng, st);
      check(hipStreamSynchronize(st));
    }
    return PLL_OK;
  });
}

int pll_stats(const pll_index *idx, int32_t graph, int64_t *counters, int32_t ncounters) {
  if (!idx || graph < 0 || graph >= idx->G || !counters || ncounters < 0) return PLL_E_INVAL;
  for (int32_t i = 0; i < ncounters && i < PLL_NSTATS; i++) counters[i] = idx->stats[i];
  return PLL_OK;
}

int64_t pll_level_trace(const pll_index *idx, int64_t *rows, int64_t max_rows) {
  if (!idx || max_rows < 0 || (max_rows > 0 && !rows)) return PLL_E_INVAL;
  const int64_t nrows = (int64_t)(idx->level_trace.size() / kTraceCols);
  const int64_t k = std::min(nrows, max_rows);
  if (k > 0) std::memcpy(rows, idx->level_trace.data(), (size_t)k * kTraceCols * sizeof(int64_t));
  return nrows;
}

void pll_free(pll_index *idx) {
  if (!idx) return;
  idx->detach_streams();
  delete idx;
}

const char *pll_strerror(int code) {
  switch (code) {
    case PLL_OK: return "ok";
    case PLL_E_INVAL: return "invalid argument";
    case PLL_E_NOMEM: return "out of memory";
    case PLL_E_RANGE: return "a distance does not fit in 8 bits (255 or more)";
    case PLL_E_DEVICE: return "HIP device error";
    case PLL_E_UNSUPPORTED: return "unsupported request";
    default: return "unknown error";
  }
}

static int set_tuning_locked(const std::string &k, int64_t value, int64_t &trim_to);

int pll_set_tuning(const char *key, int64_t value) {
  if (!key) return PLL_E_INVAL;
  int64_t trim_to = -1;
  int rc;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    rc = set_tuning_locked(std::string(key), value, trim_to);
  }
  if (rc == PLL_OK && trim_to >= 0) cache_trim((size_t)trim_to << 20);
  return rc;
}

static int set_tuning_locked(const std::string &k, int64_t value, int64_t &trim_to) {
  auto pow2_in = [](int64_t v, int64_t lo, int64_t hi) {
    return v >= lo && v <= hi && (v & (v - 1)) == 0;
  };
  if (k == "window") {
    if (value < 1 || value > kMaxWindow) return PLL_E_INVAL;
    g_tune.window = (int)value;
  } else if (k == "window_work") {
    if (value < 0 || value > (1ll << 40)) return PLL_E_INVAL;
    g_tune.window_work = value;
  } else if (k == "list_cap") {
    if (value < 0) return PLL_E_INVAL;
    g_tune.list_cap = value;
  } else if (k == "table_cap") {
    if (value < 0) return PLL_E_INVAL;
    g_tune.table_cap = value;
  } else if (k == "window_mem_mb") {
    if (value < 1 || value > (1ll << 22)) return PLL_E_INVAL;
    g_tune.window_mem_mb = value;
  } else if (k == "group") {
    if (value != 0 && !pow2_in(value, 4, 64)) return PLL_E_INVAL;
    g_tune.group = (int)value;
  } else if (k == "xgroup") {
    if (!pow2_in(value, 4, 64)) return PLL_E_INVAL;
    g_tune.xgroup = (int)value;
  } else if (k == "wgroup") {
    if (!pow2_in(value, 4, 64)) return PLL_E_INVAL;
    g_tune.wgroup = (int)value;
  } else if (k == "landmarks") {
    if (value < 0 || value > 1) return PLL_E_INVAL;
    g_tune.landmarks = (int)value;
  } else if (k == "live_adjacency") {
    if (value < 0 || value > 1) return PLL_E_INVAL;
    g_tune.live_adjacency = (int)value;
  } else if (k == "expand_prune") {
    if (value < 0 || value > 1) return PLL_E_INVAL;
    g_tune.expand_prune = (int)value;
  } else if (k == "qpersist") {
    if (value < 0 || value > 1) return PLL_E_INVAL;
    g_tune.qpersist = (int)value;
  } else if (k == "root_sort") {
    if (value < 0 || value > 2) return PLL_E_INVAL;
    g_tune.root_sort = (int)value;
  } else if (k == "sort_level") {
    if (value < 0) return PLL_E_INVAL;
    g_tune.sort_level = value;
  } else if (k == "sort_scan") {
    if (value < 0) return PLL_E_INVAL;
    g_tune.sort_scan = value;
  } else if (k == "pool_keep_mb") {
    if (value < 0 || value > (1ll << 22)) return PLL_E_INVAL;
    g_tune.pool_keep_mb = value;
    trim_to = value;
  } else if (k == "wwork") {
    if (value < 0 || value > (1ll << 40)) return PLL_E_INVAL;
    g_tune.wwork = value;
  } else if (k == "chunk") {
    if (value < 64 || value > (1 << 20)) return PLL_E_INVAL;
    g_tune.chunk = (int)value;
  } else if (k == "qgroup") {
    if (!pow2_in(value, 16, 64)) return PLL_E_INVAL;
    g_tune.qgroup = (int)value;
  } else if (k == "levels_per_sync") {
    if (value < 1 || value > 64) return PLL_E_INVAL;
    g_tune.levels_per_sync = (int)value;
  } else if (k == "profile") {
    if (value < 0 || value > 1) return PLL_E_INVAL;
    g_tune.profile = (int)value;
  } else if (k == "serve_coalesce") {
    if (value < 0 || value > 1) return PLL_E_INVAL;
    g_tune.serve_coalesce = (int)value;
  } else if (k == "bp_chunk") {
    if (value < 1 || value > (1 << 20)) return PLL_E_INVAL;
    g_tune.bp_chunk = (int)value;
  } else if (k == "whole_n") {
    if (value < 0 || value > kGMaxN) return PLL_E_INVAL;
    g_tune.whole_n = value;
  } else if (k == "packed_rows") {
    if (value < 0 || value > 1) return PLL_E_INVAL;
    g_tune.packed_rows = (int)value;
  } else if (k == "whole_pool") {
    if (value < 1 || value > (1 << 20)) return PLL_E_INVAL;
    g_tune.whole_pool = value;
  } else {
    return PLL_E_INVAL;
  }
  return PLL_OK;
}

int64_t pll_get_tuning(const char *key) {
  if (!key) return PLL_E_INVAL;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const std::string k(key);
  if (k == "window") return g_tune.window;
  if (k == "window_work") return g_tune.window_work;
  if (k == "window_mem_mb") return g_tune.window_mem_mb;
  if (k == "list_cap") return g_tune.list_cap;
  if (k == "table_cap") return g_tune.table_cap;
  if (k == "group") return g_tune.group;
  if (k == "xgroup") return g_tune.xgroup;
  if (k == "wgroup") return g_tune.wgroup;
  if (k == "wwork") return g_tune.wwork;
  if (k == "pool_keep_mb") return g_tune.pool_keep_mb;
  if (k == "landmarks") return g_tune.landmarks;
  if (k == "live_adjacency") return g_tune.live_adjacency;
  if (k == "expand_prune") return g_tune.expand_prune;
  if (k == "root_sort") return g_tune.root_sort;
  if (k == "qpersist") return g_tune.qpersist;
  if (k == "sort_level") return g_tune.sort_level;
  if (k == "sort_scan") return g_tune.sort_scan;
  if (k == "chunk") return g_tune.chunk;
  if (k == "qgroup") return g_tune.qgroup;
  if (k == "levels_per_sync") return g_tune.levels_per_sync;
  if (k == "profile") return g_tune.profile;
  if (k == "bp_chunk") return g_tune.bp_chunk;
  if (k == "serve_coalesce") return g_tune.serve_coalesce;
  if (k == "whole_n") return g_tune.whole_n;
  if (k == "whole_pool") return g_tune.whole_pool;
  if (k == "packed_rows") return g_tune.packed_rows;
  return PLL_E_INVAL;
}

}  // extern "C"
