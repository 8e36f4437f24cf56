// Pruned BFSs (Algorithms 1 and 2, Section 4.2) run as windows of
// concurrent roots, then cleaned back to the sequential result.
//
// The paper runs one pruned BFS per vertex in rank order; root k prunes with
// every label made by roots before k.  Here a window of roots [s, s+W) is run
// concurrently and each prunes with the labels of roots before s only (plus
// the bit-parallel labels).  Fewer labels prune less, so the window produces
// a superset of the sequential labels ("candidates"), all at exact distances
// (a candidate reached late would have met a pruning hub on the way).  A
// candidate (k, d) of vertex u is then dropped iff some window root j < k
// holds candidates for both u and v_k with d(j,u) + d(j,v_k) <= d: the
// lowest-ranked vertex on the shortest v_k-u paths is such a j whenever the
// sequential algorithm would have pruned u, and no j < k can reach the sum d
// otherwise (it would lie on a shortest path and have pruned u).  The
// survivors are the labels of the sequential algorithm exactly; W = 1 is the
// paper's algorithm with nothing to clean.
//
// Per window: init (stage each root's label into its row of T, Section
// 4.5.1 "Querying"), one level kernel per BFS level over the (root, vertex)
// frontier of all roots together, cleaning, and an in-order commit into the
// growing label store.  Visited bits and T are cleared afterwards from the
// frontier lists and the roots' labels, never by a full sweep (Section
// 4.5.1, "Initialization").
#include "pll_internal.h"

namespace pll {

namespace {

constexpr int kBlock = 256;

// The root's label for the normal-label test (the role of the paper's
// array T, Section 4.5.1 "Querying"): an open-addressing table per window
// root mapping hub -> distance, sized to a power of two >= 4 |L(k)|, so a
// lookup costs about one probe.  All tables of a window take a few MB and
// stay in cache, where a dense T would take n bytes per root and every
// lookup would be a random HBM read.  An entry packs hub (low 32 bits) and
// distance (next 8); kEmpty marks a free slot (no hub is 0xFFFFFFFF).
constexpr uint64_t kEmpty = ~0ull;

__device__ __forceinline__ uint32_t ht_hash(uint32_t h) {
  uint32_t x = h * 0x85EBCA6Bu;
  return x ^ (x >> 16);
}

struct RootTable {
  const uint64_t *p;
  uint32_t mask;  // size - 1; size 0 means an empty label
  bool empty;
  // distance from the root to hub h, or 255 if h is not in L(k)
  __device__ __forceinline__ int get(uint32_t h) const {
    if (empty) return kInf8;
    uint32_t slot = ht_hash(h) & mask;
    for (;;) {
      const uint64_t e = p[slot];
      if ((uint32_t)e == h) return (int)((e >> 32) & 0xFFu);
      if (e == kEmpty) return kInf8;
      slot = (slot + 1) & mask;
    }
  }
};
__device__ __forceinline__ RootTable root_table(const DWindow &w, int32_t j) {
  const int64_t a = w.htoff[j], b = w.htoff[j + 1];
  return RootTable{w.ht + a, (uint32_t)(b - a - 1), b == a};
}

__global__ void k_win_reset_ctl(LevelCtl *ctl) {
  unsigned long long *p = reinterpret_cast<unsigned long long *>(ctl);
  const int words = (int)(sizeof(LevelCtl) / sizeof(unsigned long long));
  for (int i = threadIdx.x; i < words; i += blockDim.x) p[i] = 0;
}

// Hub signature bit (0..255) of a root's label: multiplicative hashing.
__device__ __forceinline__ uint32_t sig_bit(uint32_t h) { return (h * 2654435761u) >> 24; }

// Table size of each window root (0 for an empty label or a root that runs
// no BFS), for the exclusive scan that places the tables; sizes[W] = 0.
__global__ void k_win_ht_size(DWindow w, DStore st, int64_t *sizes) {
  const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j > w.W) return;
  int64_t sz = 0;
  if (j < w.W && !w.used[w.s + j]) {
    const int32_t len = st.len[w.s + j];
    if (len > 0) {
      sz = 8;
      while (sz < 4 * (int64_t)len) sz <<= 1;
    }
  }
  sizes[j] = sz;
}

// Wave j (of the grid): root k = s + j.  Build the root's table of L(k)
// and the 256-bit signature of its hubs, mark k visited, put (j, k) on
// level 0 and label it: (k, 0) becomes a candidate of L(k) without a test.  Bit-parallel roots and neighbours run no pruned BFS (they would
// prune themselves at distance 0).  The first wave publishes the tables'
// total size and flags a window whose tables do not fit (it is then run
// again after the host grows the table area).
constexpr int kInitBlock = 1024;  // 16 roots per block share one list reservation

__global__ void __launch_bounds__(kInitBlock) k_win_init(DGraph g, DWindow w, DStore st,
                                                         DFrontier f) {
  __shared__ unsigned int s_n;
  __shared__ unsigned long long s_base, s_cbase;
  if (threadIdx.x == 0) s_n = 0;
  __syncthreads();
  const int32_t j = (int32_t)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave);
  const int lane = lane_id();
  const int32_t k = w.s + j;
  const int64_t total = w.htoff[w.W];
  if (j == 0 && lane == 0) {
    f.ctl->httotal = (unsigned long long)total;
    if (total > w.htcap) atomicOr(&f.ctl->flags, kFlagOvfHash);
  }
  const bool live = j < w.W && !w.used[k];
  if (j < w.W && !live && lane < 4) w.sig[4 * (int64_t)j + lane] = 0ull;
  unsigned int local = 0;
  if (live) {
    const int64_t a = w.htoff[j], sz = w.htoff[j + 1] - a;
    const bool fits = total <= w.htcap;
    if (fits)
      for (int64_t e = lane; e < sz; e += kWave) w.ht[a + e] = kEmpty;
    __threadfence_block();  // the wave's clears land before its inserts
    const int64_t o = st.off[k];
    const int32_t len = st.len[k];
    uint64_t sg[4] = {0ull, 0ull, 0ull, 0ull};
    for (int32_t e = lane; e < len; e += kWave) {
      const uint32_t h = st.hub[o + e];
      const uint32_t b = sig_bit(h);
#pragma unroll
      for (int q = 0; q < 4; q++) sg[q] |= (uint32_t)q == (b >> 6) ? 1ull << (b & 63) : 0ull;
      if (!fits) continue;
      const unsigned long long ent = ((unsigned long long)st.dist[o + e] << 32) | h;
      uint32_t slot = ht_hash(h) & (uint32_t)(sz - 1);
      while (atomicCAS((unsigned long long *)&w.ht[a + slot], (unsigned long long)kEmpty, ent) !=
             (unsigned long long)kEmpty)
        slot = (slot + 1) & (uint32_t)(sz - 1);
    }
#pragma unroll
    for (int q = 0; q < 4; q++) sg[q] = Group<kWave>::or_reduce(sg[q]);
    if (lane < 4)
      w.sig[4 * (int64_t)j + lane] = lane == 0 ? sg[0] : lane == 1 ? sg[1] : lane == 2 ? sg[2] : sg[3];
    if (lane == 0) {
      atomicOr(&w.vis[(int64_t)j * g.nwords + (k >> 5)], 1u << (k & 31));
      // level 0 is decided here: (k, 0) is never pruned, since every hub
      // already in L(k) lies at a positive distance from k and the
      // bit-parallel slots that could give 0 belong to used vertices
      w.wd[(int64_t)k * (w.words * 64) + j] = 0;
      atomicOr((unsigned long long *)&w.cmask[(int64_t)k * w.words + (j >> 6)], 1ull << (j & 63));
      atomicOr((unsigned long long *)&w.csum[4 * (int64_t)k + (j >> 12)], 1ull << ((j >> 6) & 63));
      local = atomicAdd(&s_n, 1u);
    }
  }
  // one reservation per block on the level-0 list and on the candidate
  // list: a device-wide counter takes its atomics one at a time
  __syncthreads();
  if (threadIdx.x == 0 && s_n) {
    LevelCtl *ctl = f.ctl;
    s_base = atomicAdd(&ctl->cnt[0], (unsigned long long)s_n);
    s_cbase = atomicAdd(&ctl->ccnt, (unsigned long long)s_n);
    atomicAdd(&ctl->visited, (unsigned long long)s_n);
    atomicAdd(&ctl->labeled, (unsigned long long)s_n);
  }
  __syncthreads();
  if (live && lane == 0) {
    const unsigned long long p = s_base + local;
    f.slot[p] = j;
    f.v[p] = k;
    const unsigned long long c = s_cbase + local;
    if (c < (unsigned long long)w.ccap) {
      w.cu[c] = k;
      w.cj[c] = j;
      w.cd[c] = 0;
    } else {
      atomicOr(&f.ctl->flags, kFlagOvfCand);
    }
  }
}

// Full prune test of one vertex by one lane (used only for the rare vertex
// at distance 255, to decide whether the build must fail).
__device__ bool prune_test_serial(DBp bp, DStore st, RootTable Tj, int32_t k, int32_t u,
                                  int d) {
  for (int32_t i = 0; i < bp.t; i++) {
    const int dk = bp.d[(int64_t)k * bp.tpad + i], du = bp.d[(int64_t)u * bp.tpad + i];
    if (dk == kInf8 || du == kInf8) continue;
    const uint64_t *mk = bp.m + 2 * ((int64_t)k * bp.t + i);
    const uint64_t *mu = bp.m + 2 * ((int64_t)u * bp.t + i);
    if (bp_pair_dist(dk, mk[0], mk[1], du, mu[0], mu[1]) <= d) return true;
  }
  const int64_t o = st.off[u];
  const int32_t len = st.len[u];
  for (int32_t e = 0; e < len; e++) {
    const int th = Tj.get(st.hub[o + e]);
    if (th != kInf8 && st.dist[o + e] + th <= d) return true;
  }
  return false;
}

// Bit-parallel prune test of (root k, vertex u, distance d) by a group of G
// lanes: does some slot give QUERY_BP(k, u) <= d (Section 5.3)?  A slot's
// estimate is d_k + d_u minus 0, 1 or 2, so the distance bytes decide most
// slots alone: d_k + d_u <= d prunes outright ("direct"), d_k + d_u - 2 > d
// never does.  Only the slots in between read their (S^{-1}, S^{0}) pairs,
// G slots per round, the slots that prune with -1 or -2 first (they succeed
// more often than the -2-only ones), stopping at the first round that
// prunes.  Distance rows are read 16 slots per lane.
// Byte-wise sums of two distance-row words, two bytes at a time in 16-bit
// fields: `hit` gets a bit where a + c <= D (K1 = (D+1) * 0x00010001; 255
// never counts there since 255 + c > 254 >= D), n2 / n1 the 4-bit masks (bit
// = byte) of the bytes with a + c == D + 1 / D + 2 (K2 = (D+2) * 0x00010001),
// both distances finite.
__device__ __forceinline__ void swar_word(uint32_t aw, uint32_t bw, uint32_t K1, uint32_t K2,
                                          uint32_t &hit, uint32_t &n1, uint32_t &n2) {
  uint32_t z1[2], z2[2];
#pragma unroll
  for (int h = 0; h < 2; h++) {  // h = 0: bytes 0 and 2, h = 1: bytes 1 and 3
    const uint32_t a = (aw >> (8 * h)) & 0x00FF00FFu;
    const uint32_t c = (bw >> (8 * h)) & 0x00FF00FFu;
    uint32_t sum = a + c;
    hit |= ~((sum | 0x80008000u) - K1) & 0x80008000u;
    const uint32_t inf = (((a + 0x00010001u) | (c + 0x00010001u)) >> 8) & 0x00010001u;
    sum |= inf * 0x1FFu;  // 255 in either byte: the field is >= 511
    const uint32_t x1 = sum ^ K1, x2 = sum ^ K2;
    z1[h] = ~((x1 | 0x80008000u) - 0x00010001u) & 0x80008000u;
    z2[h] = ~((x2 | 0x80008000u) - 0x00010001u) & 0x80008000u;
  }
  n2 = ((z1[0] >> 15) & 1u) | ((z1[1] >> 14) & 2u) | ((z1[0] >> 29) & 4u) | ((z1[1] >> 28) & 8u);
  n1 = ((z2[0] >> 15) & 1u) | ((z2[1] >> 14) & 2u) | ((z2[0] >> 29) & 4u) | ((z2[1] >> 28) & 8u);
}

// per-lane counts stay far below 2^32 within one launch; 32-bit keeps them
// to one register each (the wave sums are 64-bit)
struct BpTally {
  uint32_t direct = 0, sets = 0, checks = 0;
};

// zk, zu: bp.z[k] and bp.z[u] (read by the caller together with its other
// loads).
// krow / kpairs: the root's distance row (bp.tpad bytes) and its t set pairs,
// staged in LDS by the caller.
template <int G>
__device__ __forceinline__ bool bp_prunes(const DBp &bp, const uint4 *krow,
                                          const ulonglong2 *kpairs, int32_t u, int d,
                                          uint64_t zk, uint64_t zu, BpTally &tally) {
  const int gr = Group<G>::rank();
  const int nv = bp.tpad >> 4;
  bool direct = false;
  uint64_t need1 = 0, need2 = 0;  // slots where only -2 helps / where -1 or -2 helps
  if (gr < nv) {
    const uint4 a = krow[gr];
    const uint4 b = reinterpret_cast<const uint4 *>(bp.d + (int64_t)u * bp.tpad)[gr];
    const uint32_t aw[4] = {a.x, a.y, a.z, a.w}, bw[4] = {b.x, b.y, b.z, b.w};
    const uint32_t K1 = (uint32_t)(d + 1) * 0x00010001u, K2 = (uint32_t)(d + 2) * 0x00010001u;
    uint32_t hit = 0;
#pragma unroll
    for (int q = 0; q < 4; q++) {
      uint32_t n1, n2;
      swar_word(aw[q], bw[q], K1, K2, hit, n1, n2);
      need1 |= (uint64_t)n1 << (gr * 16 + q * 4);
      need2 |= (uint64_t)n2 << (gr * 16 + q * 4);
    }
    direct = hit != 0;
  }
  if (Group<G>::any(direct)) {
    if (gr == 0) tally.direct++;
    return true;
  }
  need1 = Group<G>::or_reduce(need1);
  need2 = Group<G>::or_reduce(need2);
  if (!(need1 | need2)) return false;
  // -2 needs S^{-1} non-empty on both sides; -1 (with S^0 on one side)
  // needs it on at least one
  need1 &= zk & zu;
  need2 &= zk | zu;
  if (!(need1 | need2)) return false;
  if (gr == 0) tally.sets++;
  const ulonglong2 *pk = kpairs;
  const ulonglong2 *pu = reinterpret_cast<const ulonglong2 *>(bp.m) + (int64_t)u * bp.t;
  // one slot per lane per round, stopping at the first round that prunes
  // (measured: fewer pair reads than dealing 16 slots per round)
  uint64_t rest2 = need2, rest1 = need1;
  while (rest2 | rest1) {
    // deal the next G slots of the queue (need2 first) to the lanes
    int mine = -1;
    bool mine2 = false;
#pragma unroll
    for (int r = 0; r < G; r++) {
      int i = -1;
      bool is2 = false;
      if (rest2) {
        i = __ffsll((unsigned long long)rest2) - 1;
        rest2 &= rest2 - 1;
        is2 = true;
      } else if (rest1) {
        i = __ffsll((unsigned long long)rest1) - 1;
        rest1 &= rest1 - 1;
      }
      if (r == gr) {
        mine = i;
        mine2 = is2;
      }
    }
    bool pr = false;
    if (mine >= 0) {
      tally.checks++;  // one slot pair per lane
      const ulonglong2 mk = pk[mine], mu = pu[mine];
      pr = (mk.x & mu.x) != 0 || (mine2 && ((mk.y & mu.x) | (mk.x & mu.y)) != 0);
    }
    if (Group<G>::any(pr)) return true;
  }
  return false;
}
template <int G>
__device__ __forceinline__ bool label_prunes(const DStore &st, RootTable Tj, ulonglong2 s01,
                                             ulonglong2 s23, int64_t o, int32_t len, int d) {
  constexpr int U = 4;
  constexpr uint32_t kNoHub = 0xFFFFFFFFu;
  const int gr = Group<G>::rank();
  if (len == 0 || Tj.empty) return false;
  const uint32_t *hp = st.hub + o;
  const uint8_t *dp = st.dist + o;
  for (int32_t base = 0; base < len; base += G * U) {
    uint32_t hh[U];
#pragma unroll
    for (int i = 0; i < U; i++) {
      const int32_t e = base + i * G + gr;
      hh[i] = e < len ? hp[e] : kNoHub;
    }
    uint32_t slot[U];
    bool want[U];
#pragma unroll
    for (int i = 0; i < U; i++) {
      const uint32_t b = sig_bit(hh[i]);
      const uint64_t wd = (b & 128) ? ((b & 64) ? s23.y : s23.x) : ((b & 64) ? s01.y : s01.x);
      want[i] = hh[i] != kNoHub && ((wd >> (b & 63)) & 1ull);
      slot[i] = ht_hash(hh[i]) & Tj.mask;
    }
    uint64_t ent[U];
#pragma unroll
    for (int i = 0; i < U; i++) ent[i] = want[i] ? Tj.p[slot[i]] : kEmpty;
    bool hit = false;
#pragma unroll
    for (int i = 0; i < U; i++) {
      if (!want[i]) continue;
      // finish the probe sequence (rarely more than one slot at load <= 1/4)
      uint64_t e = ent[i];
      uint32_t sl = slot[i];
      while ((uint32_t)e != hh[i] && e != kEmpty) {
        sl = (sl + 1) & Tj.mask;
        e = Tj.p[sl];
      }
      if (e != kEmpty) {
        const int32_t idx = base + i * G + gr;
        hit |= (int)dp[idx] + (int)((e >> 32) & 0xFFu) <= d;
      }
    }
    if (Group<G>::any(hit)) return true;
  }
  return false;
}

// The root's table in LDS: buckets of four 32-bit slots (one 16-byte LDS
// read), each slot hub << 8 | distance (hub ranks below 2^24 - 1) or
// kEmpty32.  A hub goes to the first free slot of bucket hash(h), or of the
// next bucket when all four are taken, so a lookup that meets a bucket with
// a free slot is done.  Buckets: a power of two >= |L(k)| (one entry per
// bucket on average), at most kLdsSlots / 4, so roots with labels of up to
// kLdsSlots / 4 entries; longer labels, or graphs of 2^24 - 1 or more
// vertices, use the window's table in global memory.
constexpr int kLdsSlots = 4096;
constexpr uint32_t kEmpty32 = 0xFFFFFFFFu;

// Bucket of hub h in the LDS table.  Hub ranks there are below 2^24 - 1, so
// a 24-bit multiply (a full-rate instruction, unlike the 32-bit one) mixes
// them; the table is small (at most 1024 buckets), and the shift brings the
// product's well-mixed middle bits down.
__device__ __forceinline__ uint32_t lds_hash(uint32_t h) {
  const uint32_t x = __umul24(h, 0x9E3779u);
  return x ^ (x >> 13);
}

// Distance of hub h in one bucket q, or 255: a slot holds h << 8 | dist, so
// slot ^ (h << 8) is the distance exactly when the hubs match and at least
// 256 otherwise (an empty slot included, hub ranks being below 2^24 - 1).
__device__ __forceinline__ int lds_bucket_dist(const uint4 q, uint32_t hk) {
  const uint32_t a = min(min(q.x ^ hk, q.y ^ hk), q.z ^ hk);
  return (int)min(min(a, q.w ^ hk), 255u);
}

// distance of hub h in the LDS table from bucket b on, 255 if absent
// (stored distances are at most 254): a bucket with a free slot ends the
// probe
__device__ __forceinline__ int lds_lookup_from(const uint4 *tab, uint32_t bmask, uint32_t h,
                                               uint32_t b) {
  const uint32_t hk = h << 8;
  for (;;) {
    const uint4 q = tab[b];
    const int dist = lds_bucket_dist(q, hk);
    if (dist != kInf8 || q.w == kEmpty32) return dist;
    b = (b + 1) & bmask;
  }
}

// Normal-label test against the LDS table: as label_prunes, without the
// signature (an LDS probe is cheaper than the signature's registers).
// Labels in the build's store start at multiples of 16 entries (pool slots
// are reserved in multiples of 16) and a slot's capacity is a multiple of
// 16, so a lane reads 4 consecutive entries at once -- 16 bytes of hubs and
// 4 bytes of distances, both issued before any probe -- and a quad that
// runs past the label's end stays inside its slot (those entries are
// masked out).  The four first buckets are read together; a hub absent
// from a full bucket (rare: one entry per bucket on average) continues into
// the next buckets.
template <int G>
__device__ __forceinline__ bool label_prunes_lds(const DStore &st, const uint4 *tab,
                                                 uint32_t bmask, int64_t o, int32_t len, int d) {
  const int gr = Group<G>::rank();
  if (len == 0) return false;
  const uint4 *hq = reinterpret_cast<const uint4 *>(st.hub + o);
  const uint32_t *dq = reinterpret_cast<const uint32_t *>(st.dist + o);
  const int32_t nq = (len + 3) >> 2;  // quads of entries
  uint4 h = gr < nq ? hq[gr] : make_uint4(0u, 0u, 0u, 0u);
  uint32_t dd = gr < nq ? dq[gr] : 0u;
  for (int32_t q0 = 0; q0 < nq; q0 += G) {
    // the next step's quads are loaded while this step probes the table
    const int32_t qn = q0 + G + gr;
    const uint4 hn = qn < nq ? hq[qn] : make_uint4(0u, 0u, 0u, 0u);
    const uint32_t dn = qn < nq ? dq[qn] : 0u;
    const int32_t e0 = (q0 + gr) * 4;
    const uint32_t hv[4] = {h.x, h.y, h.z, h.w};
    uint32_t b[4];
    uint4 q[4];
#pragma unroll
    for (int i = 0; i < 4; i++) b[i] = lds_hash(hv[i]) & bmask;
#pragma unroll
    for (int i = 0; i < 4; i++) q[i] = tab[b[i]];
    bool hit = false;
#pragma unroll
    for (int i = 0; i < 4; i++) {
      if (e0 + i >= len) continue;
      int dist = lds_bucket_dist(q[i], hv[i] << 8);
      if (dist == kInf8 && q[i].w != kEmpty32)
        dist = lds_lookup_from(tab, bmask, hv[i], (b[i] + 1) & bmask);
      hit |= (int)((dd >> (8 * i)) & 0xFFu) + dist <= d;
    }
    if (Group<G>::any(hit)) return true;
    h = hn;
    dd = dn;
  }
  return false;
}

// One BFS level of every root of the window, in two kernels (plus one for
// long adjacency lists).
//
// k_win_test: a group of G lanes takes one (root slot j, vertex u) entry at
// distance d and runs the bit-parallel test, then the normal-label test
// against column j of T.  If neither prunes, u gets the candidate label
// (k, d).  The work per entry is short, so many entries are in flight.
//
// k_win_expand: the candidates of this level reach their neighbours at
// d+1, a group per candidate with lanes over the adjacency list (long
// lists: the first `chunk` entries here, the rest as tasks for whole waves
// in k_win_heavy).  A neighbour not yet visited by the root whose distance
// row already prunes it at d+1 (some bit-parallel root on a shortest path)
// is left unvisited: it would be pruned at any later level too, and other
// parents test it again.  The others are claimed and go to level d+1.
constexpr int kStage = 256;                 // staged entries per wave
constexpr int kWavesPerBlock = kBlock / kWave;

// The root's distance row (up to 64 slots) held in registers.
struct RootRow {
  uint4 v[4];
  int nv;
  __device__ __forceinline__ void load(const DBp &bp, int32_t k) {
    nv = bp.tpad >> 4;
    const uint4 *p = reinterpret_cast<const uint4 *>(bp.d + (int64_t)k * bp.tpad);
#pragma unroll
    for (int q = 0; q < 4; q++) v[q] = q < nv ? p[q] : make_uint4(~0u, ~0u, ~0u, ~0u);
  }
  // Is d_k + d_x <= D for some slot?  Byte sums are formed two at a time in
  // 16-bit fields (at most 510) and compared with D+1 by one subtraction per
  // field; 255 (unreachable, padding) never counts: 255 + anything > 254 >= D.
  __device__ __forceinline__ static void sum_hits(uint4 a, uint4 b, uint32_t K, uint32_t &hit) {
    const uint32_t aw[4] = {a.x, a.y, a.z, a.w}, bw[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
    for (int y = 0; y < 4; y++) {
      const uint32_t se = (aw[y] & 0x00FF00FFu) + (bw[y] & 0x00FF00FFu);
      const uint32_t so = ((aw[y] >> 8) & 0x00FF00FFu) + ((bw[y] >> 8) & 0x00FF00FFu);
      hit |= ~((se | 0x80008000u) - K) & 0x80008000u;
      hit |= ~((so | 0x80008000u) - K) & 0x80008000u;
    }
  }
  // the 4-bit row's low (hi = false) or high nibbles as bytes; a nibble of
  // 15 (15 or more, or unreachable) becomes 255, which never counts
  __device__ __forceinline__ static uint4 unpack(uint4 b, bool hi) {
    const uint32_t w[4] = {b.x, b.y, b.z, b.w};
    uint32_t o[4];
#pragma unroll
    for (int y = 0; y < 4; y++) {
      const uint32_t c = (hi ? w[y] >> 4 : w[y]) & 0x0F0F0F0Fu;
      o[y] = c | ((((c + 0x01010101u) >> 4) & 0x01010101u) * 0xF0u);
    }
    return make_uint4(o[0], o[1], o[2], o[3]);
  }
  // P: the reached vertex's row from the 4-bit copy bp.q (then tpad is 32
  // or 64)
  template <bool P>
  __device__ __forceinline__ bool direct(const DBp &bp, int32_t x, int D) const {
    const uint32_t K = (uint32_t)(D + 1) * 0x00010001u;
    if constexpr (P) {
      // half the bytes: slot k and slot k + tpad/2 share a byte
      uint32_t hit = 0;
      if (nv == 4) {
        const uint4 *p = bp.q + (int64_t)x * 2;
        const uint4 b0 = p[0], b1 = p[1];
        sum_hits(v[0], unpack(b0, false), K, hit);
        sum_hits(v[2], unpack(b0, true), K, hit);
        sum_hits(v[1], unpack(b1, false), K, hit);
        sum_hits(v[3], unpack(b1, true), K, hit);
      } else {
        const uint4 b0 = bp.q[x];
        sum_hits(v[0], unpack(b0, false), K, hit);
        sum_hits(v[1], unpack(b0, true), K, hit);
      }
      return hit != 0;
    } else {
    const uint4 *p = reinterpret_cast<const uint4 *>(bp.d + (int64_t)x * bp.tpad);
    uint32_t hit = 0;
#pragma unroll
    for (int q = 0; q < 4; q++) {
      if (q >= nv) break;
      const uint4 b = p[q];
      const uint32_t aw[4] = {v[q].x, v[q].y, v[q].z, v[q].w}, bw[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
      for (int y = 0; y < 4; y++) {
        const uint32_t se = (aw[y] & 0x00FF00FFu) + (bw[y] & 0x00FF00FFu);
        const uint32_t so = ((aw[y] >> 8) & 0x00FF00FFu) + ((bw[y] >> 8) & 0x00FF00FFu);
        hit |= ~((se | 0x80008000u) - K) & 0x80008000u;
        hit |= ~((so | 0x80008000u) - K) & 0x80008000u;
      }
    }
    return hit != 0;
    }
  }
};

// k_win_test_flat: the prune tests of level d straight from the frontier, a
// group of G lanes per entry (j, u), the root's label read through the
// window's global table and its bit-parallel row from memory.  For short
// labels this costs less than grouping the level by root; long labels go
// through k_win_test below.
// Groups of 8 or more lanes serve long label scans, which want every wave
// the CU can hold (measured: R-MAT 18 with t_bp = 0 builds 13% faster at 8
// waves per SIMD, a few registers spilled); 4-lane groups keep all their
// registers (short scans, many tests per wave).
template <int G>
constexpr int kTestWavesPerSimd = G >= 8 ? 8 : 1;

template <int G>
__global__ void __launch_bounds__(kBlock, kTestWavesPerSimd<G>) k_win_test_flat(DGraph g, DBp bp,
                                                                              DStore st,
                                                                              DWindow w,
                                                                              DFrontier f,
                                                                              int d) {
  __shared__ int32_t s_a[kWavesPerBlock][kStage];
  __shared__ int32_t s_b[kWavesPerBlock][kStage];
  __shared__ int32_t s_n[kWavesPerBlock];
  __shared__ unsigned long long s_base, s_sum[6];
  __shared__ bool s_go;
  LevelCtl *ctl = f.ctl;
  const unsigned long long beg = ctl->base[d], cnt = ctl->cnt[d];
  const unsigned long long nbase = beg + cnt;
  if (blockIdx.x == 0 && threadIdx.x == 0) ctl->base[d + 1] = nbase;
  // the roots (level 0) were labeled by k_win_init;
  // after an overflow the window is redone; never read past the buffer.
  // One thread decides for the block (the flags may change meanwhile).
  if (threadIdx.x < 6) s_sum[threadIdx.x] = 0;
  if (threadIdx.x == 0)
    s_go = !(d == 0 || cnt == 0 || (ctl->flags & kOverflowFlags) ||
             nbase > (unsigned long long)f.cap);
  __syncthreads();
  if (!s_go) return;
  const int gr = Group<G>::rank();
  constexpr int kPerWave = kWave / G;
  const int wv = threadIdx.x / kWave;
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  WaveStage<kStage> stage;
  stage.init(s_a[wv], s_b[wv]);
  // candidates (u, j): write them at list slots from c0
  auto write_out = [&](WaveStage<kStage> &sg, unsigned long long c0) {
    for (int i = lane_id(); i < sg.n; i += kWave) {
      const unsigned long long c = c0 + i;
      if (c < (unsigned long long)w.ccap) {
        w.cu[c] = sg.a[i];
        w.cj[c] = sg.b[i];
        w.cd[c] = (uint8_t)d;
      } else {
        atomicOr(&ctl->flags, kFlagOvfCand);
      }
    }
  };
  auto flush = [&](WaveStage<kStage> &sg) { write_out(sg, sg.reserve(&ctl->ccnt)); };
  uint32_t c_visit = 0, c_test = 0, c_scan = 0, c_lab = 0;
  BpTally tally;
  // the wave steps through the level in lockstep, kPerWave entries at a time
  for (int64_t base = wid * kPerWave; base < (int64_t)cnt; base += nw * kPerWave) {
    const int64_t p = base + lane_id() / G;
    bool labeled = false;
    int32_t u = 0, j = 0;
    if (p < (int64_t)cnt) {
      j = f.slot[beg + p];
      u = f.v[beg + p];
      if (gr == 0) c_visit++;
      // everything both tests may read that depends only on (j, u) is
      // loaded now, so the loads are in flight together
      const uint64_t zk = bp.t ? bp.z[w.s + j] : 0ull;
      const uint4 hd = st.hdr[u];
      const uint64_t zu = (uint64_t)hd.y << 32 | hd.x;
      const int64_t lo = (int64_t)hd.z << 4;
      const int32_t llen = (int32_t)hd.w;
      const RootTable Tj = root_table(w, j);
      const ulonglong2 *sg = reinterpret_cast<const ulonglong2 *>(w.sig + 4 * (int64_t)j);
      const ulonglong2 s01 = sg[0], s23 = sg[1];
      // bit-parallel labels first (Section 5.4)
      const int32_t k = w.s + j;
      bool pr = bp_prunes<G>(
          bp, reinterpret_cast<const uint4 *>(bp.d + (int64_t)k * bp.tpad),
          reinterpret_cast<const ulonglong2 *>(bp.m) + (int64_t)k * bp.t, u, d, zk, zu, tally);
      if (!pr) {
        pr = label_prunes<G>(st, Tj, s01, s23, lo, llen, d);
        if (gr == 0) {
          c_test++;
          c_scan += (uint32_t)llen;
        }
      }
      labeled = !pr && gr == 0;
      if (labeled) {
        c_lab++;
        w.wd[(int64_t)u * (w.words * 64) + j] = (uint8_t)d;
        atomicOr((unsigned long long *)&w.cmask[(int64_t)u * w.words + (j >> 6)],
                 1ull << (j & 63));
        atomicOr((unsigned long long *)&w.csum[4 * (int64_t)u + (j >> 12)],
                 1ull << ((j >> 6) & 63));
      }
    }
    stage.push(labeled, u, j, flush);
  }
  write_out(stage, block_reserve(stage, &ctl->ccnt, s_n, &s_base));
  const unsigned long long sums[6] = {
      Group<kWave>::sum_reduce(c_visit),     Group<kWave>::sum_reduce(c_test),
      Group<kWave>::sum_reduce(c_scan),      Group<kWave>::sum_reduce(c_lab),
      Group<kWave>::sum_reduce(tally.sets), Group<kWave>::sum_reduce(tally.checks)};
  if (lane_id() == 0)
    for (int q = 0; q < 6; q++)
      if (sums[q]) atomicAdd(&s_sum[q], sums[q]);
  __syncthreads();
  // one thread per counter, each counter on its own line
  if (threadIdx.x < 6 && s_sum[threadIdx.x]) {
    unsigned long long *dst[6] = {&ctl->visited, &ctl->ntests, &ctl->lscanned,
                                  &ctl->labeled, &ctl->bp_sets, &ctl->bp_checks};
    atomicAdd(dst[threadIdx.x], s_sum[threadIdx.x]);
  }
}

// Level d of the window, grouped by root (DRootSort).  k_root_scan (one
// block) publishes where level d+1 will start, clears the counts the
// expansion of level d is about to make, and for d >= 1 turns the counts of
// level d into entry offsets per root and tasks of at most kTaskEntries
// entries; k_root_scatter copies the level's vertices to their root's run.
constexpr int kScanThreads = 1024;

__global__ void __launch_bounds__(kScanThreads) k_root_scan(DRootSort rs, LevelCtl *ctl,
                                                            int32_t W, int d) {
  __shared__ int64_t s_e[kScanThreads], s_t[kScanThreads];
  if (threadIdx.x == 0) ctl->base[d + 1] = ctl->base[d] + ctl->cnt[d];
  const uint32_t *rc = (d & 1) ? rs.rc1 : rs.rc0;
  uint32_t *rnext = (d & 1) ? rs.rc0 : rs.rc1;
  const int per = (W + kScanThreads - 1) / kScanThreads;
  const int j0 = (int)threadIdx.x * per;
  int64_t se = 0, stk = 0;
  for (int i = 0; i < per; i++) {
    const int j = j0 + i;
    if (j >= W) break;
    const uint32_t c = d > 0 ? rc[j] : 0u;
    se += c;
    stk += (c + kTaskEntries - 1) / kTaskEntries;
    rnext[j] = 0u;
    rs.rfill[j] = 0u;
  }
  s_e[threadIdx.x] = se;
  s_t[threadIdx.x] = stk;
  __syncthreads();
  for (int o = 1; o < kScanThreads; o <<= 1) {  // inclusive scan of both sums
    const int64_t ae = threadIdx.x >= (unsigned)o ? s_e[threadIdx.x - o] : 0;
    const int64_t at = threadIdx.x >= (unsigned)o ? s_t[threadIdx.x - o] : 0;
    __syncthreads();
    s_e[threadIdx.x] += ae;
    s_t[threadIdx.x] += at;
    __syncthreads();
  }
  if (d == 0) return;
  int64_t re = s_e[threadIdx.x] - se, rt = s_t[threadIdx.x] - stk;
  for (int i = 0; i < per; i++) {
    const int j = j0 + i;
    if (j >= W) break;
    const uint32_t c = rc[j];
    rs.roff[j] = re;
    rs.toff[j] = rt;
    re += c;
    rt += (c + kTaskEntries - 1) / kTaskEntries;
  }
  if (threadIdx.x == kScanThreads - 1) {
    rs.roff[W] = s_e[kScanThreads - 1];
    rs.toff[W] = s_t[kScanThreads - 1];
  }
}

// One lane per entry of level d.  A wave sorts its 64 (root, lane) keys
// with a bitonic network in registers, so lanes of one root become
// neighbours; the first lane of each root's run reserves the run's places
// with one atomic, all runs at once, and every entry goes to its root's
// run in lane order.
__global__ void __launch_bounds__(kBlock) k_root_scatter(DRootSort rs, DFrontier f, int d) {
  LevelCtl *ctl = f.ctl;
  const unsigned long long beg = ctl->base[d], cnt = ctl->cnt[d];
  if (d == 0 || cnt == 0 || (ctl->flags & kOverflowFlags) ||
      beg + cnt > (unsigned long long)f.cap || cnt > (unsigned long long)rs.cap)
    return;
  const int lane = lane_id();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t nloop = ((int64_t)cnt + stride - 1) / stride;
  for (int64_t it = 0; it < nloop; it++) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x + it * stride;
    const bool valid = p < (int64_t)cnt;
    // key: root slot << 6 | lane (distinct; no entry sorts past INT32_MAX)
    int32_t key = valid ? (f.slot[beg + p] << 6) | lane : INT32_MAX;
    const int32_t v = valid ? f.v[beg + p] : 0;
#pragma unroll
    for (int k = 2; k <= kWave; k <<= 1) {
#pragma unroll
      for (int s = k >> 1; s > 0; s >>= 1) {
        const int32_t o = __shfl_xor(key, s);
        // ascending where lane & k is 0 (k = 64: everywhere); the lower
        // lane of a pair keeps the smaller key in an ascending run
        const bool asc = (lane & k) == 0, lower = (lane & s) == 0;
        key = (lower == asc) ? (o < key ? o : key) : (o > key ? o : key);
      }
    }
    const bool real = key != INT32_MAX;
    const int32_t j = key >> 6, src = key & (kWave - 1);
    const int32_t jprev = __shfl_up(j, 1);
    const bool first = real && (lane == 0 || jprev != j);
    const uint64_t starts = __ballot(first);
    const uint64_t reals = __ballot(real);
    // run of this lane: from the last start at or below it to the next start
    const uint64_t below = starts & (lane == kWave - 1 ? ~0ull : ((2ull << lane) - 1));
    const int r0 = below ? 63 - __clzll((long long)below) : 0;
    uint32_t b = 0;
    if (first) {
      const uint64_t after = starts & ~((2ull << lane) - 1 | (lane == kWave - 1 ? ~0ull : 0ull));
      const int r1 = after ? __ffsll((unsigned long long)after) - 1 : kWave;
      const int r1r = __popcll(reals) < r1 ? __popcll(reals) : r1;  // invalid lanes sort last
      b = atomicAdd(&rs.rfill[j], (uint32_t)(r1r - lane));
    }
    b = __shfl(b, r0);
    const int32_t vv = __shfl(v, src);
    if (real) {
      const int64_t q = rs.roff[j] + b + (lane - r0);
      rs.sv[q] = vv;
    }
  }
}

// k_win_test: the prune tests of level d, one task (a run of at most
// kTaskEntries entries of one root k = s + j) per block at a time.  The
// block first stages the root's data in LDS -- its label as a hash table
// (the role of the paper's T, Section 4.5.1 "Querying") and its
// bit-parallel distance row and set pairs -- then a group of G lanes per
// entry (j, u) runs the bit-parallel test and the normal-label test of u at
// distance d.  If neither prunes, u gets the candidate label (k, d).
constexpr int kTStage = 128;  // staged candidates per wave
// block of the root-grouped test kernel (measured: 512 threads beat 128 and
// 256 on R-MAT 22 and on the 256-graph batch)
constexpr int kTBlock = 512;
constexpr int kTWaves = kTBlock / kWave;

// st: the store of the labels being tested (L(u)); rst: the store the
// roots' labels come from (the same for an undirected graph; the other
// side's for a digraph).
template <int G>
__global__ void __launch_bounds__(kTBlock, 5) k_win_test(DGraph g, DBp bp, DStore st, DStore rst,
                                                     DWindow w, DFrontier f, DRootSort rs,
                                                     int d) {
  __shared__ uint4 s_ht[kLdsSlots / 4];
  __shared__ uint4 s_krow[4];
  __shared__ ulonglong2 s_kpairs[64];
  __shared__ int32_t s_a[kTWaves][kTStage];
  __shared__ int32_t s_b[kTWaves][kTStage];
  __shared__ int32_t s_n[kTWaves];
  __shared__ int32_t s_qu[kTWaves][32], s_ql[kTWaves][32];
  __shared__ int64_t s_qo[kTWaves][32];
  __shared__ unsigned long long s_base, s_sum[6];
  __shared__ int64_t s_task[3];
  __shared__ bool s_go;
  LevelCtl *ctl = f.ctl;
  const unsigned long long beg = ctl->base[d], cnt = ctl->cnt[d];
  if (threadIdx.x < 6) s_sum[threadIdx.x] = 0;
  // the roots (level 0) were labeled by k_win_init; after an overflow the
  // window is redone.  One thread decides for the block.
  if (threadIdx.x == 0)
    s_go = !(d == 0 || cnt == 0 || (ctl->flags & kOverflowFlags) ||
             beg + cnt > (unsigned long long)f.cap || cnt > (unsigned long long)rs.cap);
  __syncthreads();
  if (!s_go) return;
  const int64_t ntasks = rs.toff[w.W];
  const int gr = Group<G>::rank();
  constexpr int kGA = 4, kPerA = kWave / kGA, kPerB = kWave / G;
  const int wv = threadIdx.x / kWave;
  WaveStage<kTStage> stage;
  stage.init(s_a[wv], s_b[wv]);
  // candidates (u, j): write them at list slots from c0
  auto write_out = [&](WaveStage<kTStage> &sg, unsigned long long c0) {
    for (int i = lane_id(); i < sg.n; i += kWave) {
      const unsigned long long c = c0 + i;
      if (c < (unsigned long long)w.ccap) {
        w.cu[c] = sg.a[i];
        w.cj[c] = sg.b[i];
        w.cd[c] = (uint8_t)d;
      } else {
        atomicOr(&ctl->flags, kFlagOvfCand);
      }
    }
  };
  auto flush = [&](WaveStage<kTStage> &sg) { write_out(sg, sg.reserve(&ctl->ccnt)); };
  const bool small_ranks = g.n < (1 << 24) - 1;
  uint32_t c_visit = 0, c_test = 0, c_scan = 0, c_lab = 0;
  BpTally tally;
  for (int64_t t = blockIdx.x; t < ntasks; t += gridDim.x) {
    if (threadIdx.x == 0) {
      // the root of task t: the last j with toff[j] <= t
      int32_t lo = 0, hi = w.W;
      while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (rs.toff[mid] <= t) lo = mid;
        else hi = mid;
      }
      const int64_t a0 = rs.roff[lo] + (t - rs.toff[lo]) * (int64_t)kTaskEntries;
      const int64_t a1 = rs.roff[lo + 1] < a0 + kTaskEntries ? rs.roff[lo + 1] : a0 + kTaskEntries;
      s_task[0] = lo;
      s_task[1] = a0;
      s_task[2] = a1;
    }
    __syncthreads();  // also: every lane is done with the previous task's LDS
    const int32_t j = (int32_t)s_task[0];
    const int64_t t0 = s_task[1], t1 = s_task[2];
    const int32_t k = w.s + j;
    const int32_t klen = rst.len[k];
    const bool in_lds = small_ranks && klen <= kLdsSlots / 4;
    uint32_t bmask = 0;
    if (in_lds) {
      uint32_t nb = 4;
      while (nb < (uint32_t)klen) nb <<= 1;
      bmask = nb - 1;
      for (uint32_t i = threadIdx.x; i < nb; i += blockDim.x)
        s_ht[i] = make_uint4(kEmpty32, kEmpty32, kEmpty32, kEmpty32);
    }
    if (bp.t) {
      if (threadIdx.x < (unsigned)(bp.tpad >> 4))
        s_krow[threadIdx.x] = reinterpret_cast<const uint4 *>(bp.d + (int64_t)k * bp.tpad)[threadIdx.x];
      if (threadIdx.x < (unsigned)bp.t)
        s_kpairs[threadIdx.x] =
            reinterpret_cast<const ulonglong2 *>(bp.m)[(int64_t)k * bp.t + threadIdx.x];
    }
    __syncthreads();
    if (in_lds) {
      const int64_t ko = rst.off[k];
      for (int32_t e = threadIdx.x; e < klen; e += blockDim.x) {
        const uint32_t h = rst.hub[ko + e];
        const uint32_t ent = (h << 8) | (uint32_t)rst.dist[ko + e];
        uint32_t *slots = reinterpret_cast<uint32_t *>(s_ht);
        // first free slot of the bucket, else of the next one
        for (uint32_t b = lds_hash(h) & bmask, q = 0;; q++) {
          if (q == 4) {
            q = 0;
            b = (b + 1) & bmask;
          }
          if (atomicCAS(&slots[4 * b + q], kEmpty32, ent) == kEmpty32) break;
        }
      }
    }
    __syncthreads();
    const uint64_t zk = bp.t ? bp.z[k] : 0ull;
    const RootTable Tj = root_table(w, j);
    const ulonglong2 *sg = reinterpret_cast<const ulonglong2 *>(w.sig + 4 * (int64_t)j);
    // Phase A, kGA lanes per entry (16 entries per wave): the bit-parallel
    // test; survivors wait in the wave's LDS queue.  Phase B, G lanes per
    // entry: the normal-label test of kPerB queued entries at a time.
    int qn = 0;  // queued entries (wave-uniform)
    int32_t *qu = s_qu[wv], *ql = s_ql[wv];
    int64_t *qo = s_qo[wv];
    auto phase_b = [&](int nb) {
      const int e = lane_id() / G;
      bool labeled = false;
      int32_t u = 0;
      if (e < nb) {
        u = qu[qn - nb + e];
        const int64_t lo = qo[qn - nb + e];
        const int32_t llen = ql[qn - nb + e];
        const bool pr = in_lds ? label_prunes_lds<G>(st, s_ht, bmask, lo, llen, d)
                               : label_prunes<G>(st, Tj, sg[0], sg[1], lo, llen, d);
        if (gr == 0) {
          c_test++;
          c_scan += (uint32_t)llen;
        }
        labeled = !pr && gr == 0;
        if (labeled) {
          c_lab++;
          w.wd[(int64_t)u * (w.words * 64) + j] = (uint8_t)d;
          atomicOr((unsigned long long *)&w.cmask[(int64_t)u * w.words + (j >> 6)],
                   1ull << (j & 63));
          atomicOr((unsigned long long *)&w.csum[4 * (int64_t)u + (j >> 12)],
                   1ull << ((j >> 6) & 63));
        }
      }
      stage.push(labeled, u, j, flush);
    };
    for (int64_t b0 = t0 + wv * kPerA; b0 < t1; b0 += kTWaves * kPerA) {
      const int64_t p = b0 + lane_id() / kGA;
      const int gra = lane_id() & (kGA - 1);
      bool survive = false;
      int32_t u = 0, ulen = 0;
      int64_t uoff = 0;
      if (p < t1) {
        u = rs.sv[p];
        // u's bit-parallel mask and label place in one load, in flight
        // with its bit-parallel row
        const uint4 hd = st.hdr[u];
        uoff = (int64_t)hd.z << 4;
        ulen = (int32_t)hd.w;
        if (gra == 0) c_visit++;
        // bit-parallel labels first (Section 5.4)
        survive = true;
        if (bp.t) {
          const uint64_t zu = (uint64_t)hd.y << 32 | hd.x;
          survive = !bp_prunes<kGA>(bp, s_krow, s_kpairs, u, d, zk, zu, tally);
        }
      }
      const uint64_t m = __ballot(survive && gra == 0);
      if (survive && gra == 0) {
        const int pos = qn + __popcll(m & lanes_below_mask());
        qu[pos] = u;
        qo[pos] = uoff;
        ql[pos] = ulen;
      }
      qn += __popcll(m);
      __threadfence_block();  // the queue entries are visible to the whole wave
      while (qn >= kPerB) {
        phase_b(kPerB);
        qn -= kPerB;
      }
    }
    while (qn > 0) {
      const int nb = qn < kPerB ? qn : kPerB;
      phase_b(nb);
      qn -= nb;
    }
  }
  write_out(stage, block_reserve(stage, &ctl->ccnt, s_n, &s_base));
  const unsigned long long sums[6] = {
      Group<kWave>::sum_reduce(c_visit),     Group<kWave>::sum_reduce(c_test),
      Group<kWave>::sum_reduce(c_scan),      Group<kWave>::sum_reduce(c_lab),
      Group<kWave>::sum_reduce(tally.sets), Group<kWave>::sum_reduce(tally.checks)};
  if (lane_id() == 0)
    for (int q = 0; q < 6; q++)
      if (sums[q]) atomicAdd(&s_sum[q], sums[q]);
  __syncthreads();
  // one thread per counter, each counter on its own line
  if (threadIdx.x < 6 && s_sum[threadIdx.x]) {
    unsigned long long *dst[6] = {&ctl->visited, &ctl->ntests, &ctl->lscanned,
                                  &ctl->labeled, &ctl->bp_sets, &ctl->bp_checks};
    atomicAdd(dst[threadIdx.x], s_sum[threadIdx.x]);
  }
}

// Entries (j, x) of level d+1: reserve slots and write them.
struct FrontierFlush {
  LevelCtl *ctl;
  DFrontier f;
  unsigned long long nbase;
  int d;
  __device__ void operator()(WaveStage<kStage> &sg) const {
    write_out(sg, sg.reserve(&ctl->cnt[d + 1]));
  }
  // the staged entries go to level d+1 from its slot q0 on
  __device__ void write_out(const WaveStage<kStage> &sg, unsigned long long q0) const {
    for (int i = lane_id(); i < sg.n; i += kWave) {
      const unsigned long long q = nbase + q0 + i;
      if (q < (unsigned long long)f.cap) {
        f.slot[q] = sg.a[i];
        f.v[q] = sg.b[i];
      } else {
        atomicOr(&ctl->flags, kFlagOvfFrontier);
      }
    }
  }
};

// One adjacency entry x of a candidate of root k (slot j) at level d: true
// if x is claimed for level d+1, false if its distance row prunes it
// (counted in `direct`) or it was visited already.  The distance rows (t
// bytes per vertex) mostly stay in cache while a root's visited bits are
// spread over W·n/8 bytes, so the row test goes first and most edges never
// touch the visited bits.
//
// A neighbour ranked before the window (x < s) was a root itself, or a
// bit-parallel root or neighbour: the committed labels already give its exact
// distance from every later root (Section 4.2; Section 5.3 for the
// bit-parallel ones), so the test at any level would prune it.  It is left
// unvisited before any memory is read (counted in `earlier`).
template <bool P>
__device__ __forceinline__ bool reach(const DBp &vb, const RootRow &rr, uint32_t *vs, int32_t x,
                                      int d, int32_t s, uint32_t &direct, uint32_t &earlier) {
  if (x < s) {  // s: the window start, or 0 when this skip is switched off
    earlier++;
    return false;
  }
  if (rr.template direct<P>(vb, x, d + 1)) {
    direct++;
    return false;
  }
  const uint32_t bit = 1u << (x & 31);
  if (vs[x >> 5] & bit) return false;
  return !(atomicOr(&vs[x >> 5], bit) & bit);
}

template <int G, bool P>
__global__ void __launch_bounds__(kBlock, P ? 4 : 1) k_win_expand(DGraph g, DBp bp, DBp rb, DBp vb,
                                                       DStore st, DWindow w, DFrontier f,
                                                       DRootSort rs, int d, int chunk,
                                                       int32_t skip_below) {
  __shared__ int32_t s_a[kWavesPerBlock][kStage];
  __shared__ int32_t s_b[kWavesPerBlock][kStage];
  __shared__ int32_t s_n[kWavesPerBlock];
  __shared__ unsigned long long s_base, s_sum[4];
  __shared__ bool s_go;
  LevelCtl *ctl = f.ctl;
  const unsigned long long cbeg = ctl->cmark[d], cend0 = ctl->ccnt;
  if (blockIdx.x == 0 && threadIdx.x == 0) ctl->cmark[d + 1] = cend0;
  const unsigned long long cend = cend0 < (unsigned long long)w.ccap ? cend0 : w.ccap;
  // one thread decides for the block (the flags may change meanwhile)
  if (threadIdx.x < 4) s_sum[threadIdx.x] = 0;
  if (threadIdx.x == 0) s_go = !(cend <= cbeg || (ctl->flags & kOverflowFlags));
  __syncthreads();
  if (!s_go) return;
  const unsigned long long nbase = ctl->base[d + 1];
  const int gr = Group<G>::rank();
  constexpr int kPerWave = kWave / G;
  const int wv = threadIdx.x / kWave;
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  const int64_t ncand = (int64_t)(cend - cbeg);
  WaveStage<kStage> stage;
  stage.init(s_a[wv], s_b[wv]);
  const FrontierFlush flush{ctl, f, nbase, d};
  uint32_t *rnext = ((d + 1) & 1) ? rs.rc1 : rs.rc0;  // null: the next level is not sorted
  uint32_t c_edge = 0, c_direct = 0, c_earlier = 0, c_claim = 0;
  for (int64_t base = wid * kPerWave; base < ncand; base += nw * kPerWave) {
    const int64_t c = (int64_t)cbeg + base + lane_id() / G;
    const bool act = c < (int64_t)cend;
    int32_t u = 0, j = 0;
    int64_t e0 = 0, deg = 0, lim = 0;
    RootRow rr;
    rr.nv = 0;
    if (act) {
      u = w.cu[c];
      j = w.cj[c];
      e0 = g.row[u];
      deg = g.row[u + 1] - e0;
      lim = deg < chunk ? deg : chunk;
      if (gr == 0) c_edge += (uint32_t)lim;
      rr.load(rb, w.s + j);
    }
    uint32_t *vs = w.vis + (int64_t)j * g.nwords;
    const int64_t wl = Group<kWave>::max_reduce64(lim);
    uint32_t mine = 0;  // this candidate's claims, counted toward its root's run
    for (int64_t e = 0; e < wl; e += G) {
      const int64_t idx = e + gr;
      bool claimed = false;
      int32_t x = 0;
      if (idx < lim) {
        x = g.col[e0 + idx];
        claimed = reach<P>(vb, rr, vs, x, d, skip_below, c_direct, c_earlier);
        mine += claimed ? 1u : 0u;
      }
      stage.push(claimed, j, x, flush);
    }
    c_claim += mine;
    const unsigned long long gclaims = Group<G>::sum_reduce(mine);
    if (rnext && gr == 0 && gclaims) atomicAdd(&rnext[j], (uint32_t)gclaims);
    // chunks of long lists become heavy tasks (one reservation per wave)
    const int64_t extra = act && deg > lim ? (deg - lim + chunk - 1) / chunk : 0;
    unsigned long long tb =
        wave_reserve(gr == 0 ? (unsigned long long)extra : 0ull, &ctl->hcnt[d]);
    tb = __shfl(tb, Group<G>::base());
    if (extra > 0) {
      for (int64_t q = gr; q < extra; q += G) {
        if ((int64_t)tb + q < f.hcap) {
          f.hslot[tb + q] = j;
          f.hv[tb + q] = u;
          f.hchunk[tb + q] = (int32_t)q;
        } else {
          atomicOr(&ctl->flags, kFlagOvfHeavy);
        }
      }
    }
  }
  flush.write_out(stage, block_reserve(stage, &ctl->cnt[d + 1], s_n, &s_base));
  const unsigned long long w_edge = Group<kWave>::sum_reduce(c_edge);
  const unsigned long long w_direct = Group<kWave>::sum_reduce(c_direct);
  const unsigned long long w_earlier = Group<kWave>::sum_reduce(c_earlier);
  const unsigned long long w_claim = Group<kWave>::sum_reduce(c_claim);
  if (lane_id() == 0 && w_edge) atomicAdd(&s_sum[0], w_edge);
  if (lane_id() == 0 && w_direct) atomicAdd(&s_sum[1], w_direct);
  if (lane_id() == 0 && w_earlier) atomicAdd(&s_sum[2], w_earlier);
  if (lane_id() == 0 && w_claim) atomicAdd(&s_sum[3], w_claim);
  __syncthreads();
  if (threadIdx.x == 0 && s_sum[0]) atomicAdd(&ctl->edges, s_sum[0]);
  if (threadIdx.x == 1 && s_sum[1]) atomicAdd(&ctl->bp_direct, s_sum[1]);
  if (threadIdx.x == 2 && s_sum[2]) atomicAdd(&ctl->earlier, s_sum[2]);
  if (threadIdx.x == 3 && s_sum[3]) atomicAdd(&ctl->xclaims, s_sum[3]);
}

// In place of the expansion at level 254: the neighbours would sit at
// distance 255, which 8-bit labels cannot store, so every unvisited one must
// be pruned there, else the window (or, for one root, the build) fails with
// the range flag.
__global__ void __launch_bounds__(kBlock) k_win_range(DGraph g, DBp bp, DStore st, DWindow w,
                                                      DFrontier f, int d) {
  LevelCtl *ctl = f.ctl;
  const unsigned long long cbeg = ctl->cmark[d], cend0 = ctl->ccnt;
  if (blockIdx.x == 0 && threadIdx.x == 0) ctl->cmark[d + 1] = cend0;
  const unsigned long long cend = cend0 < (unsigned long long)w.ccap ? cend0 : w.ccap;
  if (cend <= cbeg || (ctl->flags & kOverflowFlags)) return;
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t c = (int64_t)cbeg + wid; c < (int64_t)cend; c += nw) {
    const int32_t u = w.cu[c], j = w.cj[c];
    const int64_t e0 = g.row[u], deg = g.row[u + 1] - e0;
    const uint32_t *vs = w.vis + (int64_t)j * g.nwords;
    const RootTable Tj = root_table(w, j);
    for (int64_t e = lane_id(); e < deg; e += kWave) {
      const int32_t x = g.col[e0 + e];
      if ((vs[x >> 5] >> (x & 31)) & 1u) continue;
      if (!prune_test_serial(bp, st, Tj, w.s + j, x, d + 1)) atomicOr(&ctl->flags, kFlagRange);
    }
  }
}

template <bool P>
__global__ void __launch_bounds__(kBlock) k_win_heavy(DGraph g, DBp rb, DBp vb, DWindow w,
                                                      DFrontier f, DRootSort rs, int d, int chunk,
                                                      int lim_inline, int32_t skip_below) {
  __shared__ int32_t s_a[kWavesPerBlock][kStage];
  __shared__ int32_t s_b[kWavesPerBlock][kStage];
  LevelCtl *ctl = f.ctl;
  const unsigned long long ntask = ctl->hcnt[d];
  if (ntask == 0 || (ctl->flags & kOverflowFlags)) return;
  const int64_t ntasks = (int64_t)ntask < f.hcap ? (int64_t)ntask : f.hcap;
  const unsigned long long nbase = ctl->base[d] + ctl->cnt[d];
  const int wv = threadIdx.x / kWave;
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  WaveStage<kStage> stage;
  stage.init(s_a[wv], s_b[wv]);
  const FrontierFlush flush{ctl, f, nbase, d};
  uint32_t *rnext = ((d + 1) & 1) ? rs.rc1 : rs.rc0;
  unsigned long long c_edge = 0;  // the same in every lane (whole-wave tasks)
  uint32_t c_direct = 0, c_earlier = 0;
  for (int64_t tk = wid; tk < ntasks; tk += nw) {
    const int32_t j = f.hslot[tk], u = f.hv[tk], c = f.hchunk[tk];
    const int64_t e0 = g.row[u], e1 = g.row[u + 1];
    const int64_t a = e0 + lim_inline + (int64_t)c * chunk;
    const int64_t b = a + chunk < e1 ? a + chunk : e1;
    uint32_t *vs = w.vis + (int64_t)j * g.nwords;
    RootRow rr;
    rr.load(rb, w.s + j);
    c_edge += (unsigned long long)(b - a);
    uint32_t mine = 0;
    for (int64_t e0b = a; e0b < b; e0b += kWave) {
      const int64_t e = e0b + lane_id();
      bool claimed = false;
      int32_t x = 0;
      if (e < b) {
        x = g.col[e];
        claimed = reach<P>(vb, rr, vs, x, d, skip_below, c_direct, c_earlier);
        mine += claimed ? 1u : 0u;
      }
      stage.push(claimed, j, x, flush);
    }
    const unsigned long long tclaims = Group<kWave>::sum_reduce(mine);
    if (rnext && lane_id() == 0 && tclaims) atomicAdd(&rnext[j], (uint32_t)tclaims);
  }
  if (stage.n) flush(stage);
  const unsigned long long w_direct = Group<kWave>::sum_reduce(c_direct);
  const unsigned long long w_earlier = Group<kWave>::sum_reduce(c_earlier);
  if (lane_id() == 0 && c_edge) atomicAdd(&ctl->hedges, c_edge);
  if (lane_id() == 0 && w_direct) atomicAdd(&ctl->hdirect, w_direct);
  if (lane_id() == 0 && w_earlier) atomicAdd(&ctl->hearlier, w_earlier);
}

// Landmark rows (see launch_win_landmarks): out[u * 16 + j] = d(root j, u)
// for the first 16 roots of a window that pruned nothing, 255 if the root
// did not reach u.
__global__ void __launch_bounds__(kBlock) k_win_landmarks(DWindow w, int32_t n, uint8_t *out) {
  const int64_t total = (int64_t)n * kLandmarks;
  const int64_t stride = (int64_t)w.words * 64;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t u = i / kLandmarks, j = i % kLandmarks;
    const bool hit = (w.cmask[u * w.words] >> j) & 1ull;
    out[i] = hit ? w.wd[u * stride + j] : kInf8;
  }
}

// Clear visited words of every (slot, vertex) ever put on a level.
__global__ void __launch_bounds__(kBlock) k_win_reset_vis(DGraph g, DWindow w, DFrontier f,
                                                          int64_t nvisited) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nvisited;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t j = f.slot[p], x = f.v[p];
    w.vis[(int64_t)j * g.nwords + (x >> 5)] = 0u;
  }
}


// Mask rows of a vertex hold one bit per window root; csum (4 words per
// vertex) marks which 64-bit words of the row are non-zero, so the passes
// below visit only those words (a vertex is labeled by few roots of a
// window, and rows are up to 256 words long).
__device__ __forceinline__ void csum_load(const DWindow &w, int32_t u, uint64_t sm[4]) {
  const ulonglong2 *p = reinterpret_cast<const ulonglong2 *>(w.csum + 4 * (int64_t)u);
  const ulonglong2 a = p[0], b = p[1];
  sm[0] = a.x;
  sm[1] = a.y;
  sm[2] = b.x;
  sm[3] = b.y;
}

// Drop the window's candidates (a window is re-run smaller after an
// overflow), in two passes: every candidate clears its own mask word, then
// (all words cleared) the summaries.
__global__ void __launch_bounds__(kBlock) k_win_abort(DWindow w, int64_t ncand) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncand;
       c += (int64_t)gridDim.x * blockDim.x)
    w.cmask[(int64_t)w.cu[c] * w.words + (w.cj[c] >> 6)] = 0ull;
}

__global__ void __launch_bounds__(kBlock) k_win_abort_sum(DWindow w, int64_t ncand) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncand;
       c += (int64_t)gridDim.x * blockDim.x) {
    ulonglong2 *p = reinterpret_cast<ulonglong2 *>(w.csum + 4 * (int64_t)w.cu[c]);
    p[0] = make_ulonglong2(0ull, 0ull);
    p[1] = make_ulonglong2(0ull, 0ull);
  }
}

// Cleaning: candidate (k = s+j, d) of u survives iff no window root j' < j
// labeled both u and v_k with d(j',u) + d(j',v_k) <= d.  Also marks one
// candidate per vertex (the lowest j) to commit the vertex's row.  `o` is
// the window whose candidates give the v_k side: the same window for an
// undirected graph; for a directed one the search in the other direction
// (a forward candidate (k, d(k,u)) is dropped by j' with d(k,j') from the
// reverse search and d(j',u) from the forward one, and vice versa).
__global__ void __launch_bounds__(kBlock) k_win_clean(DWindow w, DWindow o, int64_t ncand) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncand;
       c += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = w.cu[c], j = w.cj[c];
    const int d = w.cd[c];
    const int32_t k = w.s + j;
    const uint64_t *cu_row = w.cmask + (int64_t)u * w.words;
    const uint64_t *ck_row = o.cmask + (int64_t)k * o.words;
    const uint8_t *wu = w.wd + (int64_t)u * (w.words * 64);
    const uint8_t *wk = o.wd + (int64_t)k * (o.words * 64);
    const int jw = j >> 6, jb = j & 63;
    uint64_t su[4], sk[4];
    csum_load(w, u, su);
    csum_load(o, k, sk);
    bool drop = false;
    for (int q = 0; q <= (jw >> 6) && !drop; q++) {
      uint64_t sm = su[q] & sk[q];
      if (q == (jw >> 6)) sm &= (jw & 63) == 63 ? ~0ull : ((2ull << (jw & 63)) - 1);
      while (sm && !drop) {
        const int i = q * 64 + __ffsll((unsigned long long)sm) - 1;
        sm &= sm - 1;
        uint64_t m = cu_row[i] & ck_row[i];
        if (i == jw) m &= jb ? (~0ull >> (64 - jb)) : 0ull;
        while (m) {
          const int b = __ffsll((unsigned long long)m) - 1;
          m &= m - 1;
          const int jj = i * 64 + b;
          if ((int)wu[jj] + (int)wk[jj] <= d) {
            drop = true;
            break;
          }
        }
      }
    }
    if (!drop)
      atomicOr((unsigned long long *)&w.kmask[(int64_t)u * w.words + jw], 1ull << jb);
    int low = -1;
    for (int q = 0; q < 4 && low < 0; q++) {
      if (su[q]) {
        const int i = q * 64 + __ffsll((unsigned long long)su[q]) - 1;
        low = i * 64 + __ffsll((unsigned long long)cu_row[i]) - 1;
      }
    }
    w.cdes[c] = (low == j) ? 1 : 0;
  }
}

// Commit, in three passes so that no thread walks a whole row serially.
// Pass 1, one lane per touched vertex (its designated candidate): count the
// surviving labels, grow the vertex's pool slot when full (the copy of the
// old entries is done by the whole wave), publish the new length and clear
// the vertex's candidate mask.
__global__ void __launch_bounds__(kBlock) k_win_commit_alloc(DWindow w, DStore st,
                                                             int64_t ncand) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nloop = (ncand + stride - 1) / stride;
  for (int64_t it = 0; it < nloop; it++) {
    const int64_t c = t0 + it * stride;
    bool reloc = false, mine = false;
    int32_t u = 0, len = 0, need = 0;
    int64_t oo = 0, no = 0, nc = 0;
    if (c < ncand && w.cdes[c]) {
      mine = true;
      u = w.cu[c];
      const uint64_t *krow = w.kmask + (int64_t)u * w.words;
      uint64_t *crow = w.cmask + (int64_t)u * w.words;
      uint64_t su[4];
      csum_load(w, u, su);
      int32_t total = 0;
      for (int q = 0; q < 4; q++) {
        uint64_t sm = su[q];
        while (sm) {
          const int i = q * 64 + __ffsll((unsigned long long)sm) - 1;
          sm &= sm - 1;
          total += __popcll(krow[i]);
          crow[i] = 0ull;
        }
      }
      len = st.len[u];
      need = len + total;
      if (total > 0 && need > st.cap[u]) {
        nc = 2 * (int64_t)need;
        if (nc < 16) nc = 16;
        nc = (nc + 15) & ~(int64_t)15;
        oo = st.off[u];
        reloc = true;
      }
      st.len[u] = need;
    }
    no = (int64_t)wave_reserve((unsigned long long)nc, st.top);
    uint64_t m = __ballot(reloc);
    while (m) {
      const int l = __ffsll((unsigned long long)m) - 1;
      m &= m - 1;
      const int32_t ln = __shfl(len, l);
      const int64_t so = __shfl(oo, l), dn = __shfl(no, l);
      for (int32_t e = lane_id(); e < ln; e += kWave) {
        st.hub[dn + e] = st.hub[so + e];
        st.dist[dn + e] = st.dist[so + e];
      }
    }
    if (reloc) {
      st.off[u] = no;
      st.cap[u] = (int32_t)nc;
    }
    // the test kernels' copy of the place and length (one 8-byte store)
    if (mine) {
      const uint64_t o16 = (uint64_t)((reloc ? no : st.off[u]) >> 4);
      reinterpret_cast<uint64_t *>(st.hdr + u)[1] = o16 | ((uint64_t)(uint32_t)need << 32);
    }
  }
}

// Pass 2, one thread per candidate: a survivor writes (root rank, distance)
// at its place among the vertex's new labels, in root order, so labels stay
// sorted by hub rank (Section 4.5.1).
__global__ void __launch_bounds__(kBlock) k_win_commit_write(DWindow w, DStore st,
                                                             int64_t ncand) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncand;
       c += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = w.cu[c], j = w.cj[c];
    const int jw = j >> 6, jb = j & 63;
    const uint64_t *krow = w.kmask + (int64_t)u * w.words;
    const uint64_t kw = krow[jw];
    if ((kw >> jb) & 1ull) {
      int32_t above = __popcll(jb == 63 ? 0ull : (kw >> (jb + 1)));
      uint64_t su[4];
      csum_load(w, u, su);
      for (int q = jw >> 6; q < 4; q++) {
        uint64_t sm = su[q];
        if (q == (jw >> 6)) sm &= (jw & 63) == 63 ? 0ull : (~0ull << ((jw & 63) + 1));
        while (sm) {
          const int i = q * 64 + __ffsll((unsigned long long)sm) - 1;
          sm &= sm - 1;
          above += __popcll(krow[i]);
        }
      }
      const int64_t o = st.off[u] + st.len[u] - 1 - above;
      st.hub[o] = (uint32_t)(w.s + j);
      st.dist[o] = w.cd[c];
    }
  }
}

// Pass 3, one thread per touched vertex: clear its survivor mask and the
// summary.
__global__ void __launch_bounds__(kBlock) k_win_commit_clear(DWindow w, int64_t ncand) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncand;
       c += (int64_t)gridDim.x * blockDim.x) {
    if (!w.cdes[c]) continue;
    const int32_t u = w.cu[c];
    uint64_t *krow = w.kmask + (int64_t)u * w.words;
    uint64_t su[4];
    csum_load(w, u, su);
    for (int q = 0; q < 4; q++) {
      uint64_t sm = su[q];
      while (sm) {
        const int i = q * 64 + __ffsll((unsigned long long)sm) - 1;
        sm &= sm - 1;
        krow[i] = 0ull;
      }
    }
    ulonglong2 *p = reinterpret_cast<ulonglong2 *>(w.csum + 4 * (int64_t)u);
    p[0] = make_ulonglong2(0ull, 0ull);
    p[1] = make_ulonglong2(0ull, 0ull);
  }
}

// hdr of an empty store: the bit-parallel masks, place 0, length 0
__global__ void k_store_hdr(uint4 *hdr, const uint64_t *z, int32_t n) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t m = z ? z[r] : 0ull;
    hdr[r] = make_uint4((uint32_t)m, (uint32_t)(m >> 32), 0u, 0u);
  }
}

__global__ void k_final_count(const int32_t *len, int64_t *cnt, int32_t n) {
  const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) cnt[r] = (int64_t)len[r] + 1;  // + sentinel
}

// One wave per vertex: copy its label into the final CSR and close it with
// the storage-only sentinel (Section 4.5.2).
__global__ void __launch_bounds__(kBlock) k_final_copy(DStore st, const int64_t *foff,
                                                       uint32_t *fhub, uint8_t *fdist,
                                                       int32_t n) {
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t r = wid; r < n; r += nw) {
    const int64_t o = st.off[r], fo = foff[r];
    const int32_t len = st.len[r];
    for (int32_t e = lane_id(); e < len; e += kWave) {
      fhub[fo + e] = st.hub[o + e];
      fdist[fo + e] = st.dist[o + e];
    }
    if (lane_id() == 0) {
      fhub[fo + len] = kSentinel;
      fdist[fo + len] = kInf8;
    }
  }
}

unsigned grid_for(int64_t items, int per_block, int64_t cap) {
  int64_t b = (items + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

}  // namespace

hipError_t launch_win_reset_ctl(LevelCtl *ctl, hipStream_t st) {
  hipLaunchKernelGGL(k_win_reset_ctl, dim3(1), dim3(256), 0, st, ctl);
  return hipGetLastError();
}

hipError_t launch_win_init(DGraph g, DWindow w, DStore s, DFrontier f, int32_t nroots,
                           int64_t *sizes, int64_t *scan_tmp, hipStream_t st) {
  if (nroots <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_win_ht_size, dim3((nroots + 1 + 255) / 256), dim3(256), 0, st, w, s, sizes);
  hipError_t e = launch_exclusive_scan(sizes, w.htoff, (int64_t)nroots, scan_tmp, st);
  if (e != hipSuccess) return e;
  constexpr int kInitWaves = kInitBlock / kWave;
  hipLaunchKernelGGL(k_win_init, dim3((nroots + kInitWaves - 1) / kInitWaves), dim3(kInitBlock), 0,
                     st, g, w, s, f);
  return hipGetLastError();
}

hipError_t launch_win_level(DGraph g, DBp bp, DBp rb, DBp vb, DStore s, DStore rst, DWindow w,
                            DFrontier f, DRootSort rs, int d, int group, int xgroup, int chunk,
                            int32_t skip_below, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1,
                            hipEvent_t ev2, hipEvent_t ev3) {
  const int blocks = 2048;
  const dim3 gd(blocks), bd(kBlock);
  // at level 0 the test kernels return at once (the roots are labeled by
  // k_win_init); they still run so that their timing events stay paired
  if (!rs.rc0) {
    switch (group) {
      case 4: PLL_LAUNCH_TIMED(k_win_test_flat<4>, gd, bd, st, ev0, ev1, g, bp, s, w, f, d); break;
      case 8: PLL_LAUNCH_TIMED(k_win_test_flat<8>, gd, bd, st, ev0, ev1, g, bp, s, w, f, d); break;
      case 16: PLL_LAUNCH_TIMED(k_win_test_flat<16>, gd, bd, st, ev0, ev1, g, bp, s, w, f, d); break;
      case 32: PLL_LAUNCH_TIMED(k_win_test_flat<32>, gd, bd, st, ev0, ev1, g, bp, s, w, f, d); break;
      default: PLL_LAUNCH_TIMED(k_win_test_flat<64>, gd, bd, st, ev0, ev1, g, bp, s, w, f, d); break;
    }
  } else {
  hipLaunchKernelGGL(k_root_scan, dim3(1), dim3(kScanThreads), 0, st, rs, f.ctl, w.W, d);
  if (d > 0) hipLaunchKernelGGL(k_root_scatter, gd, bd, 0, st, rs, f, d);
  const dim3 gt(blocks * kBlock / kTBlock), bt(kTBlock);
  switch (group) {
    case 4: PLL_LAUNCH_TIMED(k_win_test<4>, gt, bt, st, ev0, ev1, g, bp, s, rst, w, f, rs, d); break;
    case 8: PLL_LAUNCH_TIMED(k_win_test<8>, gt, bt, st, ev0, ev1, g, bp, s, rst, w, f, rs, d); break;
    case 16: PLL_LAUNCH_TIMED(k_win_test<16>, gt, bt, st, ev0, ev1, g, bp, s, rst, w, f, rs, d); break;
    case 32: PLL_LAUNCH_TIMED(k_win_test<32>, gt, bt, st, ev0, ev1, g, bp, s, rst, w, f, rs, d); break;
    default: PLL_LAUNCH_TIMED(k_win_test<64>, gt, bt, st, ev0, ev1, g, bp, s, rst, w, f, rs, d); break;
  }
  }
  if (d + 1 >= (int)kInf8) {
    PLL_LAUNCH_TIMED(k_win_range, gd, bd, st, ev2, ev3, g, bp, s, w, f, d);
    return hipGetLastError();
  }
  // the 4-bit rows when the caller made them (tpad 32 or 64)
  const bool packed = vb.q && (vb.tpad == 32 || vb.tpad == 64);
#define PLL_EXPAND(GG)                                                                       \
  do {                                                                                       \
    if (packed)                                                                              \
      PLL_LAUNCH_TIMED((k_win_expand<GG, true>), gd, bd, st, ev2, ev3, g, bp, rb, vb, s, w, f, \
                       rs, d, chunk, skip_below);                                            \
    else                                                                                     \
      PLL_LAUNCH_TIMED((k_win_expand<GG, false>), gd, bd, st, ev2, ev3, g, bp, rb, vb, s, w,   \
                       f, rs, d, chunk, skip_below);                                         \
  } while (0)
  switch (xgroup) {
    case 4: PLL_EXPAND(4); break;
    case 8: PLL_EXPAND(8); break;
    case 16: PLL_EXPAND(16); break;
    case 32: PLL_EXPAND(32); break;
    default: PLL_EXPAND(64); break;
  }
#undef PLL_EXPAND
  if (packed)
    hipLaunchKernelGGL(k_win_heavy<true>, gd, bd, 0, st, g, rb, vb, w, f, rs, d, chunk, chunk,
                       skip_below);
  else
    hipLaunchKernelGGL(k_win_heavy<false>, gd, bd, 0, st, g, rb, vb, w, f, rs, d, chunk, chunk,
                       skip_below);
  return hipGetLastError();
}

// Live adjacency: g's rows without the neighbours ranked below s (which
// the expansion skips anyway, see reach), and empty rows for the vertices
// below s (never expanded again: they are never visited).  One wave per
// row; the fill keeps each row's order.
__global__ void __launch_bounds__(kBlock) k_live_count(DGraph g, int32_t s, int64_t *cnt) {
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t r = wave; r < g.n; r += nwaves) {
    int64_t c = 0;
    if (r >= s)
      for (int64_t e = g.row[r] + lane_id(); e < g.row[r + 1]; e += kWave) c += g.col[e] >= s;
    c = (int64_t)Group<kWave>::sum_reduce((unsigned long long)c);
    if (lane_id() == 0) cnt[r] = c;
  }
}

__global__ void __launch_bounds__(kBlock) k_live_fill(DGraph g, int32_t s, const int64_t *nrow,
                                                      int32_t *ncol, const uint32_t *wt,
                                                      uint32_t *nwt) {
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t r = wave; r < g.n; r += nwaves) {
    if (r < s) continue;
    int64_t o = nrow[r];
    const int64_t b = g.row[r + 1];
    for (int64_t e0 = g.row[r]; e0 < b; e0 += kWave) {
      const int64_t e = e0 + lane_id();
      const int32_t x = e < b ? g.col[e] : -1;
      const bool keep = x >= s;
      const uint64_t m = __ballot(keep);
      if (keep) {
        const int64_t q = o + __popcll(m & lanes_below_mask());
        ncol[q] = x;
        if (wt) nwt[q] = wt[e];  // a weighted graph keeps each edge's weight
      }
      o += __popcll(m);
    }
  }
}

hipError_t launch_live_adjacency(DGraph g, int32_t s, int64_t *nrow, int32_t *ncol, int64_t *cnt,
                                 int64_t *scan_tmp, hipStream_t st, const uint32_t *wt,
                                 uint32_t *nwt) {
  if (g.n <= 0) return hipSuccess;
  const unsigned blocks = grid_for((int64_t)g.n * kWave, kBlock, 8192);
  hipLaunchKernelGGL(k_live_count, dim3(blocks), dim3(kBlock), 0, st, g, s, cnt);
  hipError_t e = launch_exclusive_scan(cnt, nrow, (int64_t)g.n, scan_tmp, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_live_fill, dim3(blocks), dim3(kBlock), 0, st, g, s, nrow, ncol, wt, nwt);
  return hipGetLastError();
}

hipError_t launch_win_landmarks(DWindow w, int32_t n, uint8_t *out, hipStream_t st) {
  if (n <= 0 || w.W < kLandmarks) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_win_landmarks, dim3(grid_for((int64_t)n * kLandmarks, kBlock, 8192)),
                     dim3(kBlock), 0, st, w, n, out);
  return hipGetLastError();
}

hipError_t launch_win_reset(DGraph g, DWindow w, DStore s, DFrontier f, int32_t nroots,
                            int64_t nvisited, hipStream_t st) {
  if (nvisited > 0)
    hipLaunchKernelGGL(k_win_reset_vis, dim3(grid_for(nvisited, kBlock, 8192)), dim3(kBlock), 0,
                       st, g, w, f, nvisited);
  return hipGetLastError();
}

hipError_t launch_win_abort(DGraph /*g*/, DWindow w, int64_t ncand, hipStream_t st) {
  if (ncand > 0) {
    const unsigned blocks = grid_for(ncand, kBlock, 8192);
    hipLaunchKernelGGL(k_win_abort, dim3(blocks), dim3(kBlock), 0, st, w, ncand);
    hipLaunchKernelGGL(k_win_abort_sum, dim3(blocks), dim3(kBlock), 0, st, w, ncand);
  }
  return hipGetLastError();
}

hipError_t launch_win_clean(DWindow w, DWindow o, int64_t ncand, hipStream_t st) {
  if (ncand > 0)
    hipLaunchKernelGGL(k_win_clean, dim3(grid_for(ncand, kBlock, 8192)), dim3(kBlock), 0, st, w, o,
                       ncand);
  return hipGetLastError();
}

hipError_t launch_win_commit(DWindow w, DStore s, int64_t ncand, hipStream_t st) {
  if (ncand <= 0) return hipSuccess;
  const unsigned blocks = grid_for(ncand, kBlock, 8192);
  hipLaunchKernelGGL(k_win_commit_alloc, dim3(blocks), dim3(kBlock), 0, st, w, s, ncand);
  hipLaunchKernelGGL(k_win_commit_write, dim3(blocks), dim3(kBlock), 0, st, w, s, ncand);
  hipLaunchKernelGGL(k_win_commit_clear, dim3(blocks), dim3(kBlock), 0, st, w, ncand);
  return hipGetLastError();
}

hipError_t launch_final_count(const int32_t *len, int64_t *cnt, int32_t n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_final_count, dim3((n + 255) / 256), dim3(256), 0, st, len, cnt, n);
  return hipGetLastError();
}

hipError_t launch_store_hdr(DStore s, const uint64_t *z, int32_t n, hipStream_t st) {
  if (n > 0)
    hipLaunchKernelGGL(k_store_hdr, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, s.hdr, z, n);
  return hipGetLastError();
}

hipError_t launch_final_copy(DStore s, const int64_t *foff, uint32_t *fhub, uint8_t *fdist,
                             int32_t n, hipStream_t st) {
  if (n > 0)
    hipLaunchKernelGGL(k_final_copy, dim3(grid_for((int64_t)n * kWave, kBlock, 8192)),
                       dim3(kBlock), 0, st, s, foff, fhub, fdist, n);
  return hipGetLastError();
}

}  // namespace pll
