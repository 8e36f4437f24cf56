// Internal declarations of the gfx950 Pruned Landmark Labeling library:
// device-side helpers, the device data structures and the kernel launchers.
// Nothing here is part of the public ABI (include/pll.h).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>

#include "pll.h"

namespace pll {

constexpr uint8_t kInf8 = 255;           // "infinity" in 8-bit distances
constexpr uint32_t kSentinel = 0xFFFFFFFFu;  // hub of the storage-only sentinel
constexpr int kWave = 64;                // CDNA wavefront width
constexpr int kMaxLevels = 256;          // BFS levels 0..254 are storable
constexpr int kMaxWindow = 16384;        // concurrent roots (bits per vertex mask)
constexpr int kLandmarks = 16;           // landmark rows of builds without bit-parallel labels

// ---------------------------------------------------------------------------
// Wave helpers (64-wide wavefronts).

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ uint64_t lanes_below_mask() {
  int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Wave-aggregated append: every active lane with pred gets a distinct slot
// in [*ctr, *ctr + count), with one atomic per wave.  Returns -1 for lanes
// without pred.
__device__ __forceinline__ int64_t wave_append(bool pred, unsigned long long *ctr) {
  uint64_t m = __ballot(pred);
  if (m == 0) return -1;
  int leader = __ffsll((unsigned long long)m) - 1;
  unsigned long long base = 0;
  if (lane_id() == leader) base = atomicAdd(ctr, (unsigned long long)__popcll(m));
  base = __shfl(base, leader);
  if (!pred) return -1;
  return (int64_t)(base + (unsigned long long)__popcll(m & lanes_below_mask()));
}

// Wave-aggregated reservation of v >= 0 slots per lane at *ctr, one atomic
// per wave; returns this lane's first slot.  All 64 lanes must call it
// together (converged code).
__device__ __forceinline__ unsigned long long wave_reserve(unsigned long long v,
                                                           unsigned long long *ctr) {
  long long x = (long long)v;  // inclusive prefix sum over the lanes
  for (int o = 1; o < kWave; o <<= 1) {
    const long long y = __shfl_up(x, o);
    if (lane_id() >= o) x += y;
  }
  const unsigned long long tot = (unsigned long long)__shfl(x, kWave - 1);
  unsigned long long base = 0;
  if (lane_id() == 0 && tot) base = atomicAdd(ctr, tot);
  base = __shfl(base, 0);
  return base + (unsigned long long)x - v;
}

// Wave-private staging of (a, b) pairs in LDS, written out to a global
// list with one atomic reservation per flush.  Every method must be called
// by all 64 lanes of the wave together (converged code): the fill count is
// then the same in every lane.
template <int CAP>
struct WaveStage {
  int32_t *a, *b;  // this wave's LDS arrays, CAP entries each
  int32_t *c;      // optional third array (null: not staged)
  int n;           // entries staged (wave-uniform)
  __device__ __forceinline__ void init(int32_t *aa, int32_t *bb, int32_t *cc = nullptr) {
    a = aa;
    b = bb;
    c = cc;
    n = 0;
  }
  // stage (va, vb[, vc]) from each lane with pred; flush first if it might
  // not fit
  template <typename F>
  __device__ __forceinline__ void push(bool pred, int32_t va, int32_t vb, F &&flush,
                                       int32_t vc = 0) {
    const uint64_t m = __ballot(pred);
    if (!m) return;
    if (n + kWave > CAP) {
      flush(*this);
      n = 0;
    }
    if (pred) {
      const int pos = n + __popcll(m & lanes_below_mask());
      a[pos] = va;
      b[pos] = vb;
      if (c) c[pos] = vc;
    }
    n += __popcll(m);
  }
  // reserve n slots at *ctr; returns the base (same in every lane) after
  // making the staged entries visible to the whole wave
  __device__ __forceinline__ unsigned long long reserve(unsigned long long *ctr) {
    __threadfence_block();
    unsigned long long base = 0;
    if (lane_id() == 0) base = atomicAdd(ctr, (unsigned long long)n);
    return __shfl(base, 0);
  }
};

// End of a staged kernel, block-wide: one reservation at *ctr for what all
// waves of the block still hold, in place of one per wave (see kCtrLine).
// Every thread of the block must call it, in block-uniform control flow.
// s_n: LDS [waves per block]; s_base: LDS.  Returns this wave's base.
template <int CAP>
__device__ __forceinline__ unsigned long long block_reserve(const WaveStage<CAP> &sg,
                                                            unsigned long long *ctr,
                                                            int32_t *s_n,
                                                            unsigned long long *s_base) {
  const int wv = threadIdx.x / kWave, nwv = blockDim.x / kWave;
  if (lane_id() == 0) s_n[wv] = sg.n;
  __syncthreads();  // also makes every lane's staged entries visible
  if (threadIdx.x == 0) {
    int32_t tot = 0;
    for (int i = 0; i < nwv; i++) tot += s_n[i];
    *s_base = tot ? atomicAdd(ctr, (unsigned long long)tot) : 0ull;
  }
  __syncthreads();
  unsigned long long b = *s_base;
  for (int i = 0; i < wv; i++) b += (unsigned long long)s_n[i];
  return b;
}

// Kernel launch that, given timing events, has the dispatch itself record
// them at the kernel's start and end (no marker packets between kernels).
#define PLL_LAUNCH_TIMED(K, gd, bd, st, e0, e1, ...)                    \
  do {                                                                 \
    if (e0)                                                            \
      hipExtLaunchKernelGGL(K, gd, bd, 0, st, e0, e1, 0, __VA_ARGS__); \
    else                                                               \
      hipLaunchKernelGGL(K, gd, bd, 0, st, __VA_ARGS__);               \
  } while (0)

// Groups of G consecutive lanes inside a wave.
template <int G>
struct Group {
  static_assert(G == 4 || G == 8 || G == 16 || G == 32 || G == 64, "group size");
  __device__ __forceinline__ static int rank() { return lane_id() & (G - 1); }
  __device__ __forceinline__ static int base() { return lane_id() & ~(G - 1); }
  __device__ __forceinline__ static uint64_t mask() {
    return G == 64 ? ~0ull : (((1ull << G) - 1) << base());
  }
  // true on every lane of the group if pred holds on any active lane of it
  __device__ __forceinline__ static bool any(bool pred) {
    return (__ballot(pred) & mask()) != 0;
  }
  __device__ __forceinline__ static uint64_t or_reduce(uint64_t v) {
#pragma unroll
    for (int o = 1; o < G; o <<= 1) v |= __shfl_xor(v, o, G);
    return v;
  }
  __device__ __forceinline__ static unsigned long long sum_reduce(unsigned long long v) {
#pragma unroll
    for (int o = 1; o < G; o <<= 1) v += __shfl_xor(v, o, G);
    return v;
  }
  __device__ __forceinline__ static int64_t max_reduce64(int64_t v) {
#pragma unroll
    for (int o = 1; o < G; o <<= 1) {
      int64_t w = __shfl_xor(v, o, G);
      v = w > v ? w : v;
    }
    return v;
  }
  __device__ __forceinline__ static int min_reduce(int v) {
#pragma unroll
    for (int o = 1; o < G; o <<= 1) {
      int w = __shfl_xor(v, o, G);
      v = w < v ? w : v;
    }
    return v;
  }
};

// Agent-scope relaxed atomic load/store (bypass the non-coherent vector L1).
template <typename T>
__device__ __forceinline__ T ld_acquire_agent(const T *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_relaxed_agent(T *p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Distance through one bit-parallel slot (Section 5.3): d_s + d_t, minus 2
// if S^{-1}(s) and S^{-1}(t) meet, else minus 1 if S^{0}(s) meets S^{-1}(t)
// or S^{-1}(s) meets S^{0}(t).
__device__ __forceinline__ int bp_pair_dist(int ds, uint64_t m1s, uint64_t m0s, int dt,
                                            uint64_t m1t, uint64_t m0t) {
  int td = ds + dt;
  if (m1s & m1t)
    td -= 2;
  else if ((m0s & m1t) | (m1s & m0t))
    td -= 1;
  return td;
}

// ---------------------------------------------------------------------------
// Device data structures.

// Graph in rank space: vertex r is the vertex of rank r; neighbour lists
// hold ranks.
struct DGraph {
  int32_t n;
  int32_t nwords;      // (n + 31) / 32
  const int64_t *row;  // [n+1]
  const int32_t *col;  // [row[n]]
};

// Bit-parallel labels, vertex-major: for vertex v and slot i, the distance
// d[v*tpad+i] (rows padded to a multiple of 16 bytes with 255, so a lane can
// read 16 slots at once) and the two sets of the slot side by side in one
// 16-byte pair: m[2*(v*t+i)] = S^{-1}, m[2*(v*t+i)+1] = S^{0}.
struct DBp {
  int32_t t, tpad;
  const uint8_t *d;
  const uint64_t *m;
  const uint64_t *z;  // [n] slots whose S^{-1} is non-empty (bit per slot)
  // optional (tpad a multiple of 32): the distances again in 4 bits, tpad/2
  // bytes per vertex; byte k holds slot k in its low nibble and slot
  // k + tpad/2 in its high nibble, each min(d, 15) (15: 15 or more, or
  // unreachable).  Read by the expansion's distance-row prune, which only
  // needs to know whether d_k + d_x <= D.
  const uint4 *q = nullptr;
};
// The same, writable, plus per-vertex "found at the next level" slot bits
// used while the bit-parallel BFS runs.
struct DBpW {
  int32_t t, tpad;
  uint8_t *d;
  uint64_t *m;
  uint64_t *found;
};
__host__ __device__ inline int32_t bp_pad(int32_t t) { return (t + 15) & ~15; }

// Device-wide atomics that fall on one cache line are carried out one at a
// time (about 12 ns apiece on MI355X, returning or not), so counters that
// many waves update each get a line of their own, and kernels sum per block
// before they add.
constexpr int kCtrLine = 128;
struct alignas(kCtrLine) LineCtr {
  unsigned long long v;
};

// Per-level control block of a level-synchronous frontier whose levels are
// stored one after another: level L occupies [base[L], base[L] + cnt[L]).
struct LevelCtl {
  unsigned long long cnt[kMaxLevels + 2];
  unsigned long long base[kMaxLevels + 2];
  unsigned long long hcnt[kMaxLevels + 2];  // heavy expansion tasks per level
  unsigned long long hcnt2[kMaxLevels + 2]; // second task list (bit-parallel E1)
  unsigned long long cmark[kMaxLevels + 2]; // first candidate found at each level
  // each counter below sits on a cache line of its own (kCtrLine)
  alignas(kCtrLine) unsigned long long ccnt;       // candidate labels of the window
  alignas(kCtrLine) unsigned long long httotal;    // entries of the window's root tables
  alignas(kCtrLine) unsigned long long visited;    // (root, vertex) entries tested
  alignas(kCtrLine) unsigned long long ntests;     // ... that reached the normal-label test
  alignas(kCtrLine) unsigned long long lscanned;   // label entries read by those tests
  alignas(kCtrLine) unsigned long long labeled;    // entries labeled (candidates)
  alignas(kCtrLine) unsigned long long edges;      // adjacency entries expanded inline
  alignas(kCtrLine) unsigned long long hedges;     // adjacency entries expanded as tasks
  alignas(kCtrLine) unsigned long long bp_direct;  // reached neighbours pruned by distances alone
  alignas(kCtrLine) unsigned long long bp_sets;    // entries whose test read slot sets
  alignas(kCtrLine) unsigned long long bp_checks;  // slot-set pairs read
  alignas(kCtrLine) unsigned long long earlier;    // neighbours ranked before the window
  alignas(kCtrLine) unsigned long long xclaims;    // neighbours claimed by k_win_expand
  alignas(kCtrLine) unsigned long long hdirect;    // bp_direct's share of k_win_heavy
  alignas(kCtrLine) unsigned long long hearlier;   // earlier's share of k_win_heavy
  alignas(kCtrLine) int32_t flags;
  int32_t pad;
};

enum : int32_t {
  kFlagOvfFrontier = 1,
  kFlagOvfHeavy = 2,
  kFlagOvfCand = 4,
  kFlagRange = 8,  // a vertex at distance 255 would be labeled (or reached, BP)
  kFlagOvfHash = 16,  // the root tables need more room than allocated
  kOverflowFlags = kFlagOvfFrontier | kFlagOvfHeavy | kFlagOvfCand | kFlagOvfHash,
  kFlagOvfPool = 32,  // a whole-graph build ran out of label pool
};

// Whole small graphs of a batch, one workgroup per graph (graphs.hip): the
// largest graph such a workgroup takes (its T array, visited bits and BFS
// queue live in LDS), and the control block of one launch.
constexpr int32_t kGMaxN = 16384;
struct GraphCtl {
  alignas(kCtrLine) int32_t cursor;  // next graph of the list
  alignas(kCtrLine) int32_t flags;   // kFlagRange | kFlagOvfPool
  alignas(kCtrLine) unsigned long long visited;  // (root, vertex) entries tested
  unsigned long long tests;     // ... that reached the normal-label test
  unsigned long long scanned;   // label entries read by those tests
  unsigned long long labeled;   // entries added
  unsigned long long edges;     // adjacency entries expanded
};

// Growing label store used during the build: label of rank r lives at
// hub/dist[off[r] .. off[r]+len[r]) inside a pool; cap[r] slots reserved.
// hdr[r] repeats what a prune test of r reads first, in one 16-byte
// record: x, y = the bit-parallel mask z[r] (slots whose sets are not both
// empty), z = off[r] / 16 (slots are reserved in multiples of 16 entries),
// w = len[r].
struct DStore {
  int64_t *off;
  int32_t *len;
  int32_t *cap;
  uint32_t *hub;
  uint8_t *dist;
  unsigned long long *top;  // pool bump pointer (device)
  int64_t pool_cap;
  uint4 *hdr;
};

// Frontier and task buffers shared by both BFS phases.
struct DFrontier {
  int32_t *slot;  // root slot (window-relative) or bit-parallel slot
  int32_t *v;     // vertex rank
  int64_t cap;
  int32_t *hslot, *hv, *hchunk;  // heavy tasks: chunks of long adjacency lists
  int64_t hcap;
  int32_t *h2slot, *h2v, *h2chunk;
  LevelCtl *ctl;
};

// State of one window of concurrently processed roots [s, s + W).
struct DWindow {
  int32_t s, W, words;  // W roots; words: mask row stride (wd row stride words*64);
                        // only the first (W+63)/64 words are in use
  uint32_t *vis;        // [W][nwords] visited bits per root slot
  uint64_t *ht;         // hash tables of the roots' labels (hub, distance)
  int64_t *htoff;       // [W+1] table j at [htoff[j], htoff[j+1]), size 2^x or 0
  int64_t htcap;        // entries available at ht
  uint64_t *sig;        // [W][4] 256-bit hub signature of each root's label
  uint8_t *wd;          // [n][words*64] distance from window root j (valid
                        // where the vertex's cmask bit j is set)
  uint64_t *cmask;      // [n][words] window roots that labeled the vertex
  uint64_t *kmask;      // [n][words] ... and whose label survived cleaning
  uint64_t *csum;       // [n][4] bit i: word i of the vertex's cmask row is non-zero
  int32_t *cu;          // candidate vertex
  int32_t *cj;          // candidate root slot
  uint8_t *cd;          // candidate distance
  uint8_t *cdes;        // 1 if this candidate commits its vertex's row
  int64_t ccap;
  const uint8_t *used;  // [n] 1 for bit-parallel roots and neighbours
};

// One BFS level of a window, grouped by root: the prune tests run root by
// root, each root's label table and bit-parallel row staged in LDS.  rc0 /
// rc1 count the entries of each window root on the levels of even / odd
// index (the expansion that makes a level adds its claims), roff / toff are
// their exclusive scans over entries and over tasks of at most kTaskEntries
// entries (roff[W] = entries, toff[W] = tasks), rfill the scatter cursors,
// and sv the level's vertices in root order.
constexpr int kTaskEntries = 1024;
struct DRootSort {
  uint32_t *rc0, *rc1;  // [W]
  uint32_t *rfill;      // [W]
  int64_t *roff;        // [W+1]
  int64_t *toff;        // [W+1]
  int32_t *sv;          // [cap]
  int64_t cap;
};

// ---------------------------------------------------------------------------
// Weighted graphs (pruned Dijkstra searches, Section 6).

constexpr uint32_t kWInf = 0xFFFFFFFFu;  // "infinity" in 32-bit distances
constexpr int kWLand = 16;               // landmark hubs of the relaxation filter

// Weighted graph in rank space: weight wt[e] belongs to edge col[e].
struct DWGraph {
  int32_t n;
  const int64_t *row;
  const int32_t *col;
  const uint32_t *wt;
};

// Growing weighted label store: label of rank r at ent[off[r] ..
// off[r]+len[r]), each entry hub << 32 | distance (so entries sort by hub).
struct DWStore {
  int64_t *off;
  int32_t *len;
  int32_t *cap;
  uint64_t *ent;
  unsigned long long *top;  // pool bump pointer (device)
  int64_t pool_cap;
  uint32_t *par;  // parent of each entry's vertex in the hub's search tree (null: not kept)
};

// Control block of one weighted window (device).
struct WCtl {  // one cache line per counter (kCtrLine)
  LineCtr fcnt[2];                                 // entries of the two frontier lists
  alignas(kCtrLine) unsigned long long tcnt;       // touched (root slot, vertex) entries
  alignas(kCtrLine) unsigned long long ccnt;       // candidate labels
  alignas(kCtrLine) unsigned long long httotal;    // entries of the window's root tables
  alignas(kCtrLine) unsigned long long survivors;
  alignas(kCtrLine) unsigned long long tests;      // entries that ran the prune test
  alignas(kCtrLine) unsigned long long scanned;    // label entries read by prune tests
  alignas(kCtrLine) unsigned long long edges;      // edges relaxed
  alignas(kCtrLine) unsigned long long improved;   // tentative distances lowered
  alignas(kCtrLine) unsigned long long processed;  // frontier entries processed
  alignas(kCtrLine) unsigned long long filtered;   // relaxations skipped by the landmark bound
  alignas(kCtrLine) unsigned long long checked;    // relaxations checked against it
  alignas(kCtrLine) int32_t flags;
  int32_t pad;
};
enum : int32_t {
  kWOvfFrontier = 1,
  kWOvfTouched = 2,
  kWOvfCand = 4,
  kWOvfHash = 16,
};

// Per-window state of the weighted searches of roots [s, s+W) on one side
// (an undirected graph has one side; a digraph a forward and a reverse one).
// Entry (j, u) stands for vertex u in the search of root s+j; td and fl are
// dense [W][n].
struct DWWindow {
  int32_t s, W, n, words;  // words: 64-bit mask words per vertex, (W+63)/64
  uint32_t *td;            // tentative distance, kWInf if not reached (no parents)
  uint64_t *tdp;           // with parents: distance << 32 | parent rank, ~0 if not
                           // reached (then td is not used)
  uint32_t *cp;            // candidate parents (with parents, else null)
  uint8_t *fl;             // flag bits (weighted.hip), padded to 4 bytes
  uint64_t *ht;            // root tables: hub -> distance of L(s+j)
  int64_t *htoff;          // [W+1]
  int64_t htcap;
  uint64_t *sig;           // [W][4]: 256-bit hub signature of each root's label
  uint64_t *lm;            // [n][words]: roots whose search labeled the vertex
  uint64_t *km;            // [n][words]: ... whose label survived cleaning
  uint64_t *lsum;          // [n]: bit q set if word q of the lm row is non-zero
  int32_t *fj0, *fu0, *fj1, *fu1;  // the two frontier lists
  int64_t fcap;
  int32_t *tj, *tu;        // touched entries
  int64_t tcap;
  int32_t *cj, *cu;        // candidates: root slot, vertex, distance
  uint32_t *cd;
  uint8_t *cdes;           // 1 if the candidate commits its vertex's row
  int64_t ccap;
  WCtl *ctl;
  // relaxation filter (null: off): 16-bit distances (65535 = that far or
  // unreachable) between the kWLand landmark hubs and every vertex,
  // vertex-major, [n][kWLand]: lroot gives the root's side of a hub path,
  // lvert the reached vertex's side; lskip[u] = entries of landmark hubs at
  // the head of u's label in this side's store
  const uint16_t *lroot;
  const uint16_t *lvert;
  const uint8_t *lskip;
};

// ---------------------------------------------------------------------------
// Launchers (return hipError_t of the launch).

hipError_t launch_validate_graph(int32_t n, const int32_t *row, const int32_t *col,
                                 const int32_t *order, const int32_t *gid,
                                 const int64_t *vtx_off, uint32_t *seen, int32_t *err,
                                 hipStream_t st);
hipError_t launch_fill_gid(const int64_t *vtx_off, int32_t G, int32_t *gid, hipStream_t st);
hipError_t launch_batch_rank(int32_t N, const int32_t *gid, const int64_t *vtx_off,
                             const int32_t *order, const int64_t *lbase, const int32_t *gpos,
                             const int64_t *gblk, int32_t *rank, int32_t *gorder,
                             int32_t *lrank, int32_t *rgid,
                             hipStream_t st);
hipError_t launch_iota_rank(const int32_t *order, int32_t *rank, int32_t n, hipStream_t st);
hipError_t launch_degrees(const int32_t *in_row, const int32_t *order, int64_t *deg, int32_t n,
                          hipStream_t st);
hipError_t launch_relabel_cols(const int32_t *in_row, const int32_t *in_col, const int32_t *order,
                               const int32_t *rank, const int64_t *row, int32_t *col, int32_t n,
                               hipStream_t st);
// exclusive scan of int64 in[0..n) into out[0..n], out[n] = total; tmp must
// hold scan_tmp_elems(n) int64
int64_t scan_tmp_elems(int64_t n);
hipError_t launch_exclusive_scan(const int64_t *in, int64_t *out, int64_t n, int64_t *tmp,
                                 hipStream_t st);

// In-edges of the rank-space graph: irow int64[n+1], icol int32[row[n]];
// work int64[n+1], tmp scan_tmp_elems(n+1) int64; with wt, iwt[row[n]] gets
// the weight of each in-edge.
hipError_t launch_transpose(const int64_t *row, const int32_t *col, int32_t n, int64_t *irow,
                            int32_t *icol, int64_t *work, int64_t *tmp, hipStream_t st,
                            const uint32_t *wt = nullptr, uint32_t *iwt = nullptr);
hipError_t launch_bp_select(DGraph g, int32_t G, int32_t t, const int64_t *vtx_off,
                            const int64_t *lbase, const int32_t *gpos, const int64_t *gblk,
                            const int32_t *lrank,
                            uint32_t *used_bits, uint32_t *tmp_bits, uint8_t *used_bytes,
                            int32_t *root, int32_t *nsel, int32_t *sel, hipStream_t st);
// bit-parallel BFS: work items = (vertex, chunk of its adjacency list)
hipError_t launch_bpv_items_count(DGraph g, int chunk, int64_t *cnt, int64_t *ioff, int64_t *tmp,
                                  hipStream_t st);
hipError_t launch_bpv_items_fill(DGraph g, const int64_t *ioff, int32_t *it_v, int32_t *it_c,
                                 hipStream_t st);
// slot records: root[s], nsel[s], sel[s*64..] for s = graph * t + slot
hipError_t launch_bpv_init(int32_t nrec, int32_t t, DBpW b, const int32_t *root,
                           const int32_t *nsel, const int32_t *sel, hipStream_t st);
hipError_t launch_bpv_level(DGraph g, DBpW b, const int32_t *it_v, const int32_t *it_c,
                            int64_t nitems, int chunk, int L, unsigned long long *cnt,
                            int32_t *flags, hipStream_t st);
hipError_t launch_bpv_finish(int64_t total, uint64_t *m, hipStream_t st);
hipError_t launch_bpv_nonempty(int32_t n, int32_t t, const uint64_t *m, uint64_t *z,
                               hipStream_t st);
// DBp::q from the 8-bit rows d ([n][tpad], tpad a multiple of 32): q holds
// n * tpad / 32 uint4
hipError_t launch_bp_pack(const uint8_t *d, int32_t n, int32_t tpad, uint4 *q, hipStream_t st);

hipError_t launch_win_reset_ctl(LevelCtl *ctl, hipStream_t st);
// sizes: int64[nroots + 1]; scan_tmp: scan_tmp_elems(nroots + 1) int64
hipError_t launch_win_init(DGraph g, DWindow w, DStore s, DFrontier f, int32_t nroots,
                           int64_t *sizes, int64_t *scan_tmp, hipStream_t st);
// ev0/ev1 (may be null): recorded around the level kernel itself.  bp: the
// bit-parallel labels of the prune test; rb / vb: distance rows of the
// expansion-time prune, root side and reached-vertex side (the bit-parallel
// rows for an undirected graph with t > 0; landmark rows otherwise, or
// tpad = 0 for none).
// s: the store labeled by this side's searches; rst: the store the roots'
// labels come from (s itself for an undirected graph).
// skip_below: neighbours ranked below it are left unvisited (the window
// start; 0 visits every neighbour, as the paper's algorithm does).
// ev0 / ev1 and ev2 / ev3 (optional): start and end of the test kernel and
// of the expansion kernel, recorded by their dispatches.
hipError_t launch_win_level(DGraph g, DBp bp, DBp rb, DBp vb, DStore s, DStore rst, DWindow w,
                            DFrontier f, DRootSort rs, int d, int group, int xgroup, int chunk,
                            int32_t skip_below, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1,
                            hipEvent_t ev2, hipEvent_t ev3);
// Landmark rows out uint8[n][kLandmarks] of a window whose searches pruned
// nothing (W >= kLandmarks): distance from its j-th root to every vertex,
// 255 if not reached.  Run before the window's commit clears its masks.
hipError_t launch_win_landmarks(DWindow w, int32_t n, uint8_t *out, hipStream_t st);
// nrow[n+1] / ncol[<= g's entries]: g without the neighbours ranked below s
// and with empty rows below s (cnt: n scratch values; scan_tmp as for
// launch_exclusive_scan).  wt / nwt (optional): edge weights, carried along.
hipError_t launch_live_adjacency(DGraph g, int32_t s, int64_t *nrow, int32_t *ncol, int64_t *cnt,
                                 int64_t *scan_tmp, hipStream_t st, const uint32_t *wt = nullptr,
                                 uint32_t *nwt = nullptr);
hipError_t launch_win_reset(DGraph g, DWindow w, DStore s, DFrontier f, int32_t nroots,
                            int64_t nvisited, hipStream_t st);
hipError_t launch_win_abort(DGraph g, DWindow w, int64_t ncand, hipStream_t st);
hipError_t launch_win_clean(DWindow w, DWindow o, int64_t ncand, hipStream_t st);
hipError_t launch_win_commit(DWindow w, DStore s, int64_t ncand, hipStream_t st);
// Pruned phase of whole graphs: graph i of the list owns the global ranks
// [gbase[i], gbase[i] + gn[i]), gn[i] <= kGMaxN, listed largest first; the
// list's workgroups label them in s, which must hold no entries of them
// yet.  ctl must be zeroed before the launch; afterwards its flags hold
// kFlagRange (a vertex at distance 255 would be labeled) or kFlagOvfPool
// (the pool is too small: the labels of the listed graphs are then
// incomplete and must be cleared before a retry).
// qp (optional, pairs = null for none): graph i's pairs are
// pairs[range[2i] .. range[2i+1]) (vertex ids, rank maps them to ranks),
// answered into out at the same index once the graph's labels are done.
struct GraphPairs {
  const int32_t *pairs;
  const int64_t *range;
  const int32_t *rank;
  uint8_t *out;
};
hipError_t launch_graph_pruned(DGraph g, DBp bp, const uint8_t *used, DStore s,
                               const int64_t *gbase, const int32_t *gn, int32_t ngraphs,
                               GraphCtl *ctl, GraphPairs qp, int32_t grid, hipStream_t st);
hipError_t launch_final_count(const int32_t *len, int64_t *cnt, int32_t n, hipStream_t st);
// hdr of an empty store (z: the bit-parallel masks, or null for none)
hipError_t launch_store_hdr(DStore s, const uint64_t *z, int32_t n, hipStream_t st);
hipError_t launch_final_copy(DStore s, const int64_t *foff, uint32_t *fhub, uint8_t *fdist,
                             int32_t n, hipStream_t st);
// Parents of the final labels (shortest paths, Section 6): for every entry
// (h, d) of u with d >= 1, the lowest-ranked p with an edge p -> u (row u of
// `pred`) whose label holds (h, d - 1); u itself for d = 0.  Sentinels get
// kSentinel.  Work items: chunks of a vertex's predecessors; cnt[u] = items
// of u (launch_tree_count), ioff = its exclusive scan (n + 1 values, nitems
// in total), items: int32[nitems] scratch.
hipError_t launch_tree_count(DGraph pred, int64_t *cnt, int32_t n, hipStream_t st);
hipError_t launch_tree_parents(DGraph pred, const int64_t *foff, const uint32_t *fhub,
                               const uint8_t *fdist, uint32_t *fpar, int32_t n,
                               const int64_t *ioff, int32_t *items, int64_t nitems,
                               hipStream_t st);

// Queries: ranks of ids, bit-parallel labels, final CSR labels with sentinel.
struct DIndex {
  int32_t n;
  int32_t t, tpad;
  const int32_t *rank;
  const int32_t *rgid;  // graph of each rank (batches), or null for one graph
  const uint8_t *bpd;
  const uint64_t *bpm;  // interleaved (S^{-1}, S^{0}) pairs
  const int64_t *off;
  const uint32_t *hub;
  const uint8_t *dist;
  // labels of the target side of a query: the same arrays for an
  // undirected graph, L_IN for a directed one (off/hub/dist are L_OUT)
  const int64_t *toff;
  const uint32_t *thub;
  const uint8_t *tdist;
  // kept by builds with PLL_PARENTS (else null): parent of each entry's
  // vertex in the hub's BFS tree, the rank-space graph, rank -> id
  const uint32_t *par;
  const uint32_t *tpar;  // parents of the target-side labels (L_IN of a digraph)
  const int64_t *grow;
  const int32_t *gcol;
  const int32_t *ord;
  // weighted index: packed entries hub << 32 | distance at off (source
  // side) and toff (target side), each label closed by ~0
  const uint64_t *went;
  const uint64_t *twent;
};
hipError_t launch_validate_pairs(const int32_t *pairs, int64_t q, int32_t n, int32_t *err,
                                 hipStream_t st);
hipError_t launch_or_flag(const int32_t *src, int32_t *dst, hipStream_t st);
// cursor (device, optional): use the persistent batched form with it as
// the shared work cursor
hipError_t launch_query(DIndex ix, const int32_t *pairs, int64_t q, uint8_t *out,
                        const int32_t *err, bool plain, int qgroup, hipStream_t st,
                        unsigned long long *cursor = nullptr);
// *flag = 0 by a kernel (graph-capturable, unlike a memset)
hipError_t launch_zero_flag(int32_t *flag, hipStream_t st);
// Persistent batched queries: groups take chunks of pairs from *cursor
// (device, zeroed by a kernel first, so the launch may be captured in a
// graph).
hipError_t launch_query_persist(DIndex ix, const int32_t *pairs, int64_t q, uint8_t *out,
                                const int32_t *err, int qgroup, unsigned long long *cursor,
                                hipStream_t st);

// export of one graph (rows = its global ranks in local rank order)
hipError_t launch_invert_rank(const int32_t *rank, int32_t *ord, int32_t n, hipStream_t st);
// Shortest paths of q pairs (ids): row i of paths (maxlen ids) and lens[i]
// (D+1; 0 unreachable; -(D+1) if maxlen is too small; INT32_MIN if the
// index is inconsistent).  err as launch_query.
hipError_t launch_query_path(DIndex ix, const int32_t *pairs, int64_t q, int32_t maxlen,
                             int32_t *paths, int32_t *lens, const int32_t *err, hipStream_t st);
hipError_t launch_gather_labels(const int64_t *rows, int64_t m, const int64_t *src_off,
                                const uint32_t *hub, const uint8_t *dist, const int32_t *lrank,
                                const int64_t *out_off, uint32_t *out_hub, uint8_t *out_dist,
                                hipStream_t st);
hipError_t launch_gather_bp(const int64_t *rows, int64_t m, int32_t t, int32_t tpad,
                            const uint8_t *bpd, const uint64_t *bpm, uint8_t *out_d,
                            uint64_t *out_m1, uint64_t *out_m0, hipStream_t st);
hipError_t launch_gather_rank(int64_t g0, int64_t ng, const int32_t *rank, const int32_t *lrank,
                              int32_t *out, hipStream_t st);

// Weighted graphs (weighted.hip).
hipError_t launch_validate_weights(const uint32_t *w, int64_t nnz, int32_t *err, hipStream_t st);
hipError_t launch_relabel_weights(const int32_t *in_row, const uint32_t *in_w, const int32_t *order,
                                  const int64_t *row, uint32_t *wt, int32_t n, hipStream_t st);
hipError_t launch_ww_reset_ctl(WCtl *ctl, hipStream_t st);
hipError_t launch_ww_zero_list(WCtl *ctl, int list, hipStream_t st);
// sizes: int64[W + 1]; scan_tmp: scan_tmp_elems(W + 1) int64
hipError_t launch_ww_init(DWStore tabsrc, DWWindow w, int64_t *sizes, int64_t *scan_tmp,
                          hipStream_t st);
hipError_t launch_ww_step(DWGraph g, DWStore s, DWWindow w, int cur, int group, hipStream_t st,
                          hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
hipError_t launch_ww_collect(DWWindow w, hipStream_t st);
hipError_t launch_ww_clean(DWWindow w, DWWindow o, hipStream_t st);
hipError_t launch_ww_commit(DWWindow w, DWStore s, hipStream_t st);
hipError_t launch_ww_reset(DWWindow w, hipStream_t st);
// out uint16[n][kWLand] <- the first kWLand distance rows of w (W >= kWLand),
// saturated at 65535; skip[v] <- label entries of v with a hub < kWLand
hipError_t launch_ww_landmarks(DWWindow w, uint16_t *out, hipStream_t st);
hipError_t launch_ww_lskip(DWStore s, int32_t n, uint8_t *skip, hipStream_t st);
hipError_t launch_wfinal_count(const int32_t *len, int64_t *cnt, int32_t n, hipStream_t st);
hipError_t launch_wfinal_copy(DWStore s, const int64_t *foff, uint64_t *fent, uint32_t *fpar,
                              int32_t n, hipStream_t st);
// Shortest paths of a weighted index built with parents (lens = vertices on
// the path; 0 unreachable; -(vertices) if maxlen is too small).
hipError_t launch_wquery_path(DIndex ix, const int32_t *pairs, int64_t q, int32_t maxlen,
                              int32_t *paths, int32_t *lens, const int32_t *err, hipStream_t st);
// out[i] = min(d(s, t), kWInf) over the packed weighted labels of ix
hipError_t launch_wquery(DIndex ix, const int32_t *pairs, int64_t q, uint32_t *out,
                         const int32_t *err, bool plain, int qgroup, hipStream_t st);

}  // namespace pll
