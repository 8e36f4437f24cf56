// Weighted graphs (Section 6, "Weighted Graphs"): every root runs a pruned
// Dijkstra search instead of a pruned BFS; there are no bit-parallel labels
// and distances are 32-bit.
//
// A window of roots [s, s+W) runs concurrently, each search pruning with the
// labels of roots before s, exactly as the unweighted windows do; the
// cleaning argument there only uses shortest-path distances, so it carries
// over unchanged (a candidate (k, d) of u is dropped iff a window root j < k
// labeled both u and v_k with d(j,u) + d(j,v_k) <= d).
//
// One search on the GPU is label-correcting instead of settling vertices in
// distance order: steps over a frontier of (root slot, vertex) entries whose
// tentative distance dropped.  An entry is tested against the root's table
// with its current distance; if it is not pruned it is marked labeled and
// relaxes its edges (atomicMin on the tentative distances), and every entry
// whose distance drops joins the next frontier.  The distances only fall and
// the test only gets easier to pass as they fall, so "labeled" never has to
// be undone, and at the fixpoint the labeled entries and their distances are
// those of the pruned Dijkstra search: a vertex pruned at its final
// distance relaxed nothing after it was reached at that distance, and every
// vertex not pruned at its final distance was tested at it.
//
// Entry flags (one byte per entry, updated through 32-bit atomics): Q0/Q1
// "in frontier list 0/1", TOUCHED "on the touched list" (for the reset and
// the candidates), LABELED.  A step reading list c clears Q_c of what it
// reads and sets Q_{1-c} of what it queues, so an entry is on each list at
// most once and no improvement is lost: one made during a step is always
// seen by a later step (the entry is queued for the next one, or already
// is).
//
// Relaxation filter.  The first window's searches run with no committed
// labels, so for its first kWLand roots h they are complete Dijkstra
// searches and their distance rows are exact: d(h, v) for every v.  For any
// later window, QUERY(root, v) over the committed labels equals the minimum
// of d(root, h) + d(h, v) over all committed hubs h (the property behind
// Theorem 4.1), so it is at most lb = min over those kWLand hubs.  An edge
// that would give v a distance nd >= lb can only make v pruned at nd, and
// a pruned vertex does nothing, so the relaxation is skipped before its
// random read of td: the rows are kept vertex-major as 16-bit distances
// (kWLand of them = 32 bytes per vertex, cache resident), a distance of
// 65535 or more stored as 65535 and then left out of the minimum (the bound
// only gets weaker, so it stays safe).  For a digraph the forward search
// uses d(root -> h) from the reverse rows and d(h -> v) from the forward
// rows, and the reverse search the other way round.  The same bound makes
// the landmark hubs useless in the prune test of a later window (an entry
// is only reached below it), so a test at a distance below 65535 skips the
// label entries of hubs below kWLand.
#include <climits>

#include "pll_internal.h"

namespace pll {

namespace {

constexpr int kBlock = 256;
constexpr unsigned kGrid = 2048;
constexpr int kWStage = 256;  // staged list entries per wave
constexpr uint64_t kEmptyW = ~0ull;

constexpr uint32_t kQ0 = 1, kQ1 = 2, kTouched = 4, kLabeled = 8;

__device__ __forceinline__ uint32_t qbit(int list) { return list ? kQ1 : kQ0; }

// Byte flags through the aligned 32-bit word that holds them; return the
// byte's old value.
__device__ __forceinline__ uint32_t fl_or(uint8_t *fl, int64_t idx, uint32_t bits) {
  uint32_t *w = reinterpret_cast<uint32_t *>(fl + (idx & ~(int64_t)3));
  const int sh = (int)(idx & 3) * 8;
  return (atomicOr(w, bits << sh) >> sh) & 0xFFu;
}
__device__ __forceinline__ uint32_t fl_clear(uint8_t *fl, int64_t idx, uint32_t bits) {
  uint32_t *w = reinterpret_cast<uint32_t *>(fl + (idx & ~(int64_t)3));
  const int sh = (int)(idx & 3) * 8;
  return (atomicAnd(w, ~(bits << sh)) >> sh) & 0xFFu;
}

// The root's label as an open-addressing table hub -> distance (the role of
// the array T of Section 4.5.1): entry = distance << 32 | hub, kEmptyW free,
// size a power of two >= 4 |L(root)|.
__device__ __forceinline__ uint32_t wt_hash(uint32_t h) {
  const uint32_t x = h * 0x9E3779B1u;
  return x ^ (x >> 15);
}

struct WRootTable {
  const uint64_t *p;
  uint32_t mask;
  bool empty;
  __device__ __forceinline__ uint32_t get(uint32_t h) const {
    if (empty) return kWInf;
    uint32_t slot = wt_hash(h) & mask;
    for (;;) {
      const uint64_t e = p[slot];
      if ((uint32_t)e == h) return (uint32_t)(e >> 32);
      if (e == kEmptyW) return kWInf;
      slot = (slot + 1) & mask;
    }
  }
};

__device__ __forceinline__ WRootTable wroot_table(const DWWindow &w, int32_t j) {
  const int64_t a = w.htoff[j], b = w.htoff[j + 1];
  return WRootTable{w.ht + a, (uint32_t)(b - a - 1), b == a};
}

// Hub signature bit (0..255) of a root's label: a label entry whose hub's
// bit is clear in the root's 256-bit signature cannot be in the root's
// table, so it is not probed.
__device__ __forceinline__ uint32_t wsig_bit(uint32_t h) { return (h * 2654435761u) >> 24; }

// The prune test of entry (root table T, vertex u) at distance d: does some
// hub of L(u) (from entry b0 on) give T[h] + d(h, u) <= d?  G lanes, U
// entries per lane per round, signature check before each probe; adds the
// entries read to *scanned (lane 0).
// o, len: L(u)'s place in the store; s01, s23: the root's signature (read
// by the caller together with its other loads).
template <int G>
__device__ __forceinline__ bool wlabel_prunes(const DWStore &s, const WRootTable &T,
                                              ulonglong2 s01, ulonglong2 s23, int64_t o,
                                              int32_t len, uint32_t d, int32_t b0,
                                              uint32_t *scanned) {
  constexpr int U = 2;
  const int gr = Group<G>::rank();
  if (T.empty || len <= b0) return false;
  for (int32_t base = b0; base < len; base += G * U) {
    if (gr == 0) *scanned += (uint32_t)(len - base < G * U ? len - base : G * U);
    uint64_t ent[U];
#pragma unroll
    for (int i = 0; i < U; i++) {
      const int32_t e = base + i * G + gr;
      ent[i] = e < len ? s.ent[o + e] : kEmptyW;
    }
    uint32_t hh[U], slot[U];
    bool want[U];
#pragma unroll
    for (int i = 0; i < U; i++) {
      hh[i] = (uint32_t)(ent[i] >> 32);
      const uint32_t b = wsig_bit(hh[i]);
      const uint64_t wd = (b & 128) ? ((b & 64) ? s23.y : s23.x) : ((b & 64) ? s01.y : s01.x);
      want[i] = ent[i] != kEmptyW && ((wd >> (b & 63)) & 1ull);
      slot[i] = wt_hash(hh[i]) & T.mask;
    }
    uint64_t te[U];
#pragma unroll
    for (int i = 0; i < U; i++) te[i] = want[i] ? T.p[slot[i]] : kEmptyW;
    bool hit = false;
#pragma unroll
    for (int i = 0; i < U; i++) {
      if (!want[i]) continue;
      // finish the probe sequence (rarely more than one slot at load <= 1/4)
      uint64_t e = te[i];
      uint32_t sl = slot[i];
      while ((uint32_t)e != hh[i] && e != kEmptyW) {
        sl = (sl + 1) & T.mask;
        e = T.p[sl];
      }
      if (e != kEmptyW) hit |= (ent[i] & 0xFFFFFFFFull) + (e >> 32) <= (uint64_t)d;
    }
    if (Group<G>::any(hit)) return true;
  }
  return false;
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
  return Group<kWave>::sum_reduce(v);
}

// Tentative distance of entry idx: td, or the high half of tdp when parents
// are kept (tdp = distance << 32 | parent, so one 64-bit atomic minimum
// keeps distance and parent consistent: the smallest distance wins and,
// among equal distances, the lowest-ranked parent).
__device__ __forceinline__ uint32_t wdist(const DWWindow &w, int64_t idx) {
  return w.tdp ? (uint32_t)(w.tdp[idx] >> 32) : w.td[idx];
}

__global__ void k_validate_weights(const uint32_t *w, int64_t nnz, int32_t *err) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nnz;
       i += (int64_t)gridDim.x * blockDim.x)
    if (w[i] == 0) atomicOr(err, 1);
}

// One wave per rank-space row: the weights of vertex order[r]'s row, in the
// row's order (the column copy maps the neighbours the same way).
__global__ void __launch_bounds__(kBlock) k_relabel_weights(const int32_t *in_row,
                                                            const uint32_t *in_w,
                                                            const int32_t *order,
                                                            const int64_t *row, uint32_t *wt,
                                                            int32_t n) {
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t r = wave; r < n; r += nwaves) {
    const int32_t v = order[r];
    const int64_t a = in_row[v], b = in_row[v + 1], o = row[r];
    for (int64_t e = a + lane_id(); e < b; e += kWave) wt[o + (e - a)] = in_w[e];
  }
}

__global__ void k_ww_reset_ctl(WCtl *ctl) {
  unsigned long long *p = reinterpret_cast<unsigned long long *>(ctl);
  const int words = (int)(sizeof(WCtl) / sizeof(unsigned long long));
  for (int i = threadIdx.x; i < words; i += blockDim.x) p[i] = 0;
}

__global__ void k_ww_zero_list(WCtl *ctl, int list) {
  if (threadIdx.x == 0) ctl->fcnt[list].v = 0;
}

__global__ void k_ww_ht_size(DWStore src, DWWindow w, int64_t *sizes) {
  const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j > w.W) return;
  int64_t sz = 0;
  if (j < w.W) {
    const int32_t len = src.len[w.s + j];
    if (len > 0) {
      sz = 8;
      while (sz < 4 * (int64_t)len) sz <<= 1;
    }
  }
  sizes[j] = sz;
}

// Wave j: root r = s + j.  Its table from L(r) in `src` (the root's own
// labels; for a digraph the opposite direction's), distance 0 at r, (j, r)
// on frontier list 0 and on the touched list.  Wave 0 publishes the list
// counts and flags tables that do not fit (the window is then re-run after
// the host grows the table area; the steps do nothing while a flag is set).
__global__ void __launch_bounds__(kBlock) k_ww_init(DWStore src, DWWindow w) {
  const int32_t j = (int32_t)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave);
  if (j >= w.W) return;
  const int lane = lane_id();
  const int32_t r = w.s + j;
  const int64_t total = w.htoff[w.W];
  const bool fits = total <= w.htcap;
  if (j == 0 && lane == 0) {
    w.ctl->httotal = (unsigned long long)total;
    if (!fits) atomicOr(&w.ctl->flags, kWOvfHash);
    w.ctl->fcnt[0].v = (unsigned long long)w.W;
    w.ctl->tcnt = (unsigned long long)w.W;
  }
  const int64_t a = w.htoff[j], sz = w.htoff[j + 1] - a;
  if (fits)
    for (int64_t e = lane; e < sz; e += kWave) w.ht[a + e] = kEmptyW;
  __threadfence_block();  // the wave's clears land before its inserts
  const int64_t o = src.off[r];
  const int32_t len = src.len[r];
  uint64_t sg[4] = {0ull, 0ull, 0ull, 0ull};
  for (int32_t e = lane; e < len; e += kWave) {
    const uint64_t ent = src.ent[o + e];
    const uint32_t h = (uint32_t)(ent >> 32);
    const uint32_t bit = wsig_bit(h);
#pragma unroll
    for (int q = 0; q < 4; q++) sg[q] |= (uint32_t)q == (bit >> 6) ? 1ull << (bit & 63) : 0ull;
    if (!fits) continue;
    const unsigned long long te = ((ent & 0xFFFFFFFFull) << 32) | h;
    uint32_t slot = wt_hash(h) & (uint32_t)(sz - 1);
    while (atomicCAS((unsigned long long *)&w.ht[a + slot], (unsigned long long)kEmptyW, te) !=
           (unsigned long long)kEmptyW)
      slot = (slot + 1) & (uint32_t)(sz - 1);
  }
#pragma unroll
  for (int q = 0; q < 4; q++) sg[q] = Group<kWave>::or_reduce(sg[q]);
  if (lane < 4)
    w.sig[4 * (int64_t)j + lane] = lane == 0 ? sg[0] : lane == 1 ? sg[1] : lane == 2 ? sg[2] : sg[3];
  if (lane == 0) {
    const int64_t idx = (int64_t)j * w.n + r;
    if (w.tdp)
      w.tdp[idx] = (uint64_t)(uint32_t)r;  // distance 0, its own parent
    else
      w.td[idx] = 0;
    fl_or(w.fl, idx, kTouched | kQ0);
    w.fj0[j] = j;
    w.fu0[j] = r;
    w.tj[j] = j;
    w.tu[j] = r;
  }
}

// One step over frontier list `cur`, G lanes per entry: the prune test
// (QUERY(root, u) over the labels committed before the window, with the
// root's table) while the entry is not labeled yet, then the relaxation of
// u's edges.  Improved entries go to list 1-cur (once) and, the first time
// they are reached, to the touched list.
// Latency bound: 8 waves per SIMD (registers capped at 64, a few spilled)
// measured 8% faster than the 4 that 100 registers allow.
template <int G>
__global__ void __launch_bounds__(kBlock, 8) k_ww_step(DWGraph g, DWStore s, DWWindow w, int cur) {
  constexpr int kWaves = kBlock / kWave;
  __shared__ int32_t s_nj[kWaves][kWStage], s_nu[kWaves][kWStage];
  __shared__ int32_t s_tj[kWaves][kWStage], s_tu[kWaves][kWStage];
  __shared__ int32_t s_n1[kWaves], s_n2[kWaves];
  // the root's 16-bit landmark distances of each entry a wave holds, read
  // by the entry's lanes while they relax its edges (held in registers they
  // would spill at 8 waves per SIMD)
  __shared__ uint4 s_rl[kWaves][kWave / G][kWLand / 8];
  __shared__ unsigned long long s_b1, s_b2, s_sum[7];
  __shared__ bool s_go;
  // one thread decides for the block (the flags may change meanwhile)
  if (threadIdx.x < 7) s_sum[threadIdx.x] = 0;
  if (threadIdx.x == 0) s_go = w.ctl->flags == 0;
  __syncthreads();
  if (!s_go) return;
  unsigned long long cnt = w.ctl->fcnt[cur].v;
  if (cnt > (unsigned long long)w.fcap) cnt = (unsigned long long)w.fcap;
  const int32_t *inj = cur ? w.fj1 : w.fj0;
  const int32_t *inu = cur ? w.fu1 : w.fu0;
  int32_t *outj = cur ? w.fj0 : w.fj1;
  int32_t *outu = cur ? w.fu0 : w.fu1;
  unsigned long long *outc = &w.ctl->fcnt[cur ^ 1].v;
  const uint32_t qc = qbit(cur), qn = qbit(cur ^ 1);
  const int gr = Group<G>::rank(), gb = Group<G>::base();
  constexpr int kPerWave = kWave / G;
  const int wv = threadIdx.x / kWave;
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  const int32_t n = w.n;
  // entries for the next frontier list and for the touched list are staged
  // per wave and written with one reservation per stage
  WaveStage<kWStage> sn, stt;
  sn.init(s_nj[wv], s_nu[wv]);
  stt.init(s_tj[wv], s_tu[wv]);
  auto write_n = [&](const WaveStage<kWStage> &sg, unsigned long long q0) {
    for (int i = lane_id(); i < sg.n; i += kWave) {
      const unsigned long long q = q0 + i;
      if (q < (unsigned long long)w.fcap) {
        outj[q] = sg.a[i];
        outu[q] = sg.b[i];
      } else {
        atomicOr(&w.ctl->flags, kWOvfFrontier);
      }
    }
  };
  auto write_t = [&](const WaveStage<kWStage> &sg, unsigned long long q0) {
    for (int i = lane_id(); i < sg.n; i += kWave) {
      const unsigned long long q = q0 + i;
      if (q < (unsigned long long)w.tcap) {
        w.tj[q] = sg.a[i];
        w.tu[q] = sg.b[i];
      } else {
        atomicOr(&w.ctl->flags, kWOvfTouched);
      }
    }
  };
  auto flush_n = [&](WaveStage<kWStage> &sg) { write_n(sg, sg.reserve(outc)); };
  auto flush_t = [&](WaveStage<kWStage> &sg) { write_t(sg, sg.reserve(&w.ctl->tcnt)); };
  // counts: labels scanned per lane, the others per wave (ballots, so they
  // stay in scalar registers); far below 2^32 within one launch, the block
  // sums are 64-bit
  uint32_t c_scanned = 0;
  uint32_t c_tests = 0, c_edges = 0, c_improved = 0, c_proc = 0, c_filtered = 0, c_checked = 0;
  const uint4 *rl = s_rl[wv][lane_id() / G];
  // the wave steps through the list in lockstep, kPerWave entries at a time
  for (int64_t base = wid * kPerWave; base < (int64_t)cnt; base += nw * kPerWave) {
    const int64_t i = base + lane_id() / G;
    int32_t j = 0, u = 0;
    uint32_t d = 0;
    int64_t a = 0, b = 0;  // u's edges to relax (none if pruned)
    bool tested = false;
    if (i < (int64_t)cnt) {
      j = inj[i];
      u = inu[i];
      const int64_t idx = (int64_t)j * n + u;
      uint32_t f = 0;
      if (gr == 0) {
        f = fl_clear(w.fl, idx, qc);
        d = w.tdp ? (uint32_t)(ld_acquire_agent(&w.tdp[idx]) >> 32) : ld_acquire_agent(&w.td[idx]);
      }
      // what the prune test may read that depends only on (j, u) is loaded
      // now, in flight with the flag and distance
      const int64_t lo = s.off[u];
      const int32_t llen = s.len[u];
      const int32_t skip = w.lroot ? (int32_t)w.lskip[u] : 0;
      const WRootTable T = wroot_table(w, j);
      const ulonglong2 *sg = reinterpret_cast<const ulonglong2 *>(w.sig + 4 * (int64_t)j);
      const ulonglong2 s01 = sg[0], s23 = sg[1];
      f = (uint32_t)__shfl((int)f, gb);
      d = (uint32_t)__shfl((int)d, gb);
      bool pr = false;
      if (!(f & kLabeled)) {
        tested = true;
        // entries of landmark hubs cannot prune here (see above): the entry
        // was reached below the 16-bit bound, and a hub left out of that
        // bound is at least 65535 away, so below 65535 none of them can
        const int32_t b0 = (w.lroot && d < 0xFFFFu) ? skip : 0;
        pr = wlabel_prunes<G>(s, T, s01, s23, lo, llen, d, b0, &c_scanned);
        if (!pr && gr == 0) fl_or(w.fl, idx, kLabeled);
      }
      if (!pr) {
        if (w.lroot && gr < kWLand / 8) {
          const uint4 *p = reinterpret_cast<const uint4 *>(w.lroot + (int64_t)(w.s + j) * kWLand);
          s_rl[wv][lane_id() / G][gr] = p[gr];
        }
        a = g.row[u];
        b = g.row[u + 1];
      }
    }
    c_proc += (uint32_t)__popcll(__ballot(i < (int64_t)cnt && gr == 0));
    c_tests += (uint32_t)__popcll(__ballot(tested && gr == 0));
    __threadfence_block();  // the landmark rows in LDS are visible to the whole wave
    const int64_t wl = Group<kWave>::max_reduce64(b - a);
    for (int64_t e0 = 0; e0 < wl; e0 += G) {
      const int64_t e = a + e0 + gr;
      bool push_n = false, push_t = false;
      int32_t v = 0;
      bool checked = false, filtered = false, lowered_any = false;
      if (e < b) {
        v = g.col[e];
        const uint64_t nd = (uint64_t)d + g.wt[e];
        bool useful = nd < (uint64_t)kWInf;
        if (useful && w.lroot) {
          checked = true;
          const uint4 *p = reinterpret_cast<const uint4 *>(w.lvert + (int64_t)v * kWLand);
          uint32_t lb = kWInf;
#pragma unroll
          for (int q = 0; q < kWLand / 8; q++) {
            const uint4 x = p[q], r = rl[q];
            const uint32_t xv[4] = {x.x, x.y, x.z, x.w}, rv[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
            for (int i = 0; i < 4; i++) {
#pragma unroll
              for (int half = 0; half < 2; half++) {
                const uint32_t a16 = (rv[i] >> (16 * half)) & 0xFFFFu;
                const uint32_t b16 = (xv[i] >> (16 * half)) & 0xFFFFu;
                const uint32_t t = (a16 == 0xFFFFu || b16 == 0xFFFFu) ? kWInf : a16 + b16;
                lb = t < lb ? t : lb;
              }
            }
          }
          if ((uint64_t)lb <= nd) {
            useful = false;
            filtered = true;
          }
        }
        if (useful) {
          const int64_t vi = (int64_t)j * n + v;
          bool lowered = false;
          if (w.tdp) {
            // distance and parent in one atomic; an equal distance with a
            // lower-ranked parent only updates the parent
            const unsigned long long key = (nd << 32) | (uint32_t)u;
            if (key < w.tdp[vi]) {
              const unsigned long long old =
                  atomicMin((unsigned long long *)&w.tdp[vi], key);
              lowered = key < old && (uint32_t)(old >> 32) > (uint32_t)nd;
            }
          } else if ((uint32_t)nd < w.td[vi]) {
            lowered = (uint32_t)nd < atomicMin(&w.td[vi], (uint32_t)nd);
          }
          if (lowered) {
            lowered_any = true;
            const uint32_t of = fl_or(w.fl, vi, kTouched | qn);
            push_t = !(of & kTouched);
            push_n = !(of & qn);
          }
        }
      }
      c_edges += (uint32_t)__popcll(__ballot(e < b));
      c_checked += (uint32_t)__popcll(__ballot(checked));
      c_filtered += (uint32_t)__popcll(__ballot(filtered));
      c_improved += (uint32_t)__popcll(__ballot(lowered_any));
      sn.push(push_n, j, v, flush_n);
      stt.push(push_t, j, v, flush_t);
    }
  }
  write_n(sn, block_reserve(sn, outc, s_n1, &s_b1));
  write_t(stt, block_reserve(stt, &w.ctl->tcnt, s_n2, &s_b2));
  const unsigned long long sums[7] = {c_checked, c_filtered, c_tests, wave_sum(c_scanned),
                                      c_edges,   c_improved, c_proc};
  if (lane_id() == 0)
    for (int q = 0; q < 7; q++)
      if (sums[q]) atomicAdd(&s_sum[q], sums[q]);
  __syncthreads();
  // one thread per counter, each counter on its own line
  if (threadIdx.x < 7 && s_sum[threadIdx.x]) {
    unsigned long long *dst[7] = {&w.ctl->checked, &w.ctl->filtered, &w.ctl->tests,
                                  &w.ctl->scanned, &w.ctl->edges,    &w.ctl->improved,
                                  &w.ctl->processed};
    atomicAdd(dst[threadIdx.x], s_sum[threadIdx.x]);
  }
}

// Labeled touched entries become candidates (root slot, vertex, final
// distance); the vertex's mask row and summary get the root's bit.
__global__ void __launch_bounds__(kBlock) k_ww_collect(DWWindow w) {
  constexpr int kWaves = kBlock / kWave;
  __shared__ int32_t s_j[kWaves][kWStage], s_u[kWaves][kWStage];
  __shared__ int32_t s_n[kWaves];
  __shared__ unsigned long long s_base;
  unsigned long long tc = w.ctl->tcnt;
  if (tc > (unsigned long long)w.tcap) tc = (unsigned long long)w.tcap;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nloop = ((int64_t)tc + stride - 1) / stride;
  // labeled entries (j, u) are staged per wave; the write-out reads their
  // final distance and parent again
  WaveStage<kWStage> sg;
  sg.init(s_j[threadIdx.x / kWave], s_u[threadIdx.x / kWave]);
  auto write_out = [&](const WaveStage<kWStage> &st, unsigned long long p0) {
    for (int i = lane_id(); i < st.n; i += kWave) {
      const unsigned long long p = p0 + i;
      const int32_t j = st.a[i], u = st.b[i];
      if (p < (unsigned long long)w.ccap) {
        const int64_t idx = (int64_t)j * w.n + u;
        w.cj[p] = j;
        w.cu[p] = u;
        w.cd[p] = wdist(w, idx);
        if (w.cp) w.cp[p] = w.tdp ? (uint32_t)w.tdp[idx] : 0u;
        atomicOr((unsigned long long *)&w.lm[(int64_t)u * w.words + (j >> 6)],
                 1ull << (j & 63));
        atomicOr((unsigned long long *)&w.lsum[u], 1ull << (j >> 6));
      } else {
        atomicOr(&w.ctl->flags, kWOvfCand);
      }
    }
  };
  auto flush = [&](WaveStage<kWStage> &st) { write_out(st, st.reserve(&w.ctl->ccnt)); };
  for (int64_t it = 0; it < nloop; it++) {  // wave-uniform trip count
    const int64_t i = t0 + it * stride;
    bool lab = false;
    int32_t j = 0, u = 0;
    if (i < (int64_t)tc) {
      j = w.tj[i];
      u = w.tu[i];
      lab = (w.fl[(int64_t)j * w.n + u] & kLabeled) != 0;
    }
    sg.push(lab, j, u, flush);
  }
  write_out(sg, block_reserve(sg, &w.ctl->ccnt, s_n, &s_base));
}

// Cleaning: candidate (k, d) of u is dropped iff a window root j < k labeled
// both u (in this side's searches) and v_k (in side o's: the same side for
// an undirected graph, the opposite direction for a digraph) with
// d(j, u) + d(j, v_k) <= d.  Survivors set their bit in the km row; the
// candidate of u's lowest window root is u's designated committer.
__global__ void __launch_bounds__(kBlock) k_ww_clean(DWWindow w, DWWindow o) {
  __shared__ unsigned long long s_keep;
  if (threadIdx.x == 0) s_keep = 0;
  __syncthreads();
  unsigned long long kept = 0;
  unsigned long long cc = w.ctl->ccnt;
  if (cc > (unsigned long long)w.ccap) cc = (unsigned long long)w.ccap;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nloop = ((int64_t)cc + stride - 1) / stride;
  const int32_t n = w.n;
  for (int64_t it = 0; it < nloop; it++) {
    const int64_t c = t0 + it * stride;
    bool keep = false;
    if (c < (int64_t)cc) {
      const int32_t k = w.cj[c], u = w.cu[c];
      const uint64_t d = w.cd[c];
      const int32_t rk = w.s + k;
      const int kw = k >> 6;
      const uint64_t *lu = w.lm + (int64_t)u * w.words;
      const uint64_t *lk = o.lm + (int64_t)rk * o.words;
      uint64_t sm = w.lsum[u] & o.lsum[rk];
      sm &= kw == 63 ? ~0ull : ((2ull << kw) - 1);
      bool drop = false;
      while (sm && !drop) {
        const int q = __ffsll((unsigned long long)sm) - 1;
        sm &= sm - 1;
        uint64_t m = lu[q] & lk[q];
        if (q == kw) m &= (1ull << (k & 63)) - 1;
        while (m) {
          const int bb = __ffsll((unsigned long long)m) - 1;
          m &= m - 1;
          const int64_t jj = (int64_t)q * 64 + bb;
          if ((uint64_t)wdist(w, jj * n + u) + wdist(o, jj * n + rk) <= d) {
            drop = true;
            break;
          }
        }
      }
      if (!drop) {
        keep = true;
        atomicOr((unsigned long long *)&w.km[(int64_t)u * w.words + kw], 1ull << (k & 63));
      }
      const int q0 = __ffsll((unsigned long long)w.lsum[u]) - 1;
      const int low = q0 * 64 + __ffsll((unsigned long long)lu[q0]) - 1;
      w.cdes[c] = low == k ? 1 : 0;
    }
    kept += keep ? 1ull : 0ull;
  }
  // one addition per block (see kCtrLine)
  kept = wave_sum(kept);
  if (lane_id() == 0 && kept) atomicAdd(&s_keep, kept);
  __syncthreads();
  if (threadIdx.x == 0 && s_keep) atomicAdd(&w.ctl->survivors, s_keep);
}

// Commit pass 1, one lane per designated candidate: count the vertex's
// survivors, grow its slot when full (the whole wave copies the old
// entries), publish the new length, clear the lm row.
__global__ void __launch_bounds__(kBlock) k_ww_commit_alloc(DWWindow w, DWStore st) {
  unsigned long long cc = w.ctl->ccnt;
  if (cc > (unsigned long long)w.ccap) cc = (unsigned long long)w.ccap;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nloop = ((int64_t)cc + stride - 1) / stride;
  for (int64_t it = 0; it < nloop; it++) {
    const int64_t c = t0 + it * stride;
    bool reloc = false;
    int32_t u = 0, len = 0;
    int64_t oo = 0, no = 0, nc = 0;
    if (c < (int64_t)cc && w.cdes[c]) {
      u = w.cu[c];
      uint64_t *lrow = w.lm + (int64_t)u * w.words;
      const uint64_t *krow = w.km + (int64_t)u * w.words;
      uint64_t sm = w.lsum[u];
      int32_t total = 0;
      while (sm) {
        const int q = __ffsll((unsigned long long)sm) - 1;
        sm &= sm - 1;
        total += __popcll(krow[q]);
        lrow[q] = 0ull;
      }
      len = st.len[u];
      const int32_t need = len + total;
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
        st.ent[dn + e] = st.ent[so + e];
        if (st.par) st.par[dn + e] = st.par[so + e];
      }
    }
    if (reloc) {
      st.off[u] = no;
      st.cap[u] = (int32_t)nc;
    }
  }
}

// Commit pass 2, one thread per candidate: a survivor writes (root rank,
// distance) at its place among the vertex's new entries, in root order, so
// labels stay sorted by hub rank.
__global__ void __launch_bounds__(kBlock) k_ww_commit_write(DWWindow w, DWStore st) {
  unsigned long long cc = w.ctl->ccnt;
  if (cc > (unsigned long long)w.ccap) cc = (unsigned long long)w.ccap;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < (int64_t)cc;
       c += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = w.cu[c], k = w.cj[c];
    const int kw = k >> 6, kb = k & 63;
    const uint64_t *krow = w.km + (int64_t)u * w.words;
    const uint64_t kword = krow[kw];
    if (!((kword >> kb) & 1ull)) continue;
    int32_t above = __popcll(kb == 63 ? 0ull : (kword >> (kb + 1)));
    uint64_t sm = w.lsum[u] & (kw == 63 ? 0ull : (~0ull << (kw + 1)));
    while (sm) {
      const int q = __ffsll((unsigned long long)sm) - 1;
      sm &= sm - 1;
      above += __popcll(krow[q]);
    }
    const int64_t o = st.off[u] + st.len[u] - 1 - above;
    st.ent[o] = ((uint64_t)(uint32_t)(w.s + k) << 32) | w.cd[c];
    if (st.par) st.par[o] = w.cp[c];
  }
}

// Commit pass 3, one thread per designated candidate: clear the km row and
// the summary.
__global__ void __launch_bounds__(kBlock) k_ww_commit_clear(DWWindow w) {
  unsigned long long cc = w.ctl->ccnt;
  if (cc > (unsigned long long)w.ccap) cc = (unsigned long long)w.ccap;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < (int64_t)cc;
       c += (int64_t)gridDim.x * blockDim.x) {
    if (!w.cdes[c]) continue;
    const int32_t u = w.cu[c];
    uint64_t *krow = w.km + (int64_t)u * w.words;
    uint64_t sm = w.lsum[u];
    while (sm) {
      const int q = __ffsll((unsigned long long)sm) - 1;
      sm &= sm - 1;
      krow[q] = 0ull;
    }
    w.lsum[u] = 0ull;
  }
}

// Touched entries back to "not reached" (never a full sweep).
__global__ void __launch_bounds__(kBlock) k_ww_reset(DWWindow w) {
  unsigned long long tc = w.ctl->tcnt;
  if (tc > (unsigned long long)w.tcap) tc = (unsigned long long)w.tcap;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)tc;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t idx = (int64_t)w.tj[i] * w.n + w.tu[i];
    if (w.tdp)
      w.tdp[idx] = ~0ull;
    else
      w.td[idx] = kWInf;
    w.fl[idx] = 0;
  }
}

// Vertex-major 16-bit copy of the first kWLand distance rows of a window:
// out[v * kWLand + h] = min(td[h][v], 65535).
__global__ void __launch_bounds__(kBlock) k_ww_landmarks(DWWindow w, uint16_t *out) {
  const int64_t total = (int64_t)w.n * kWLand;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t v = i / kWLand, h = i % kWLand;
    const uint32_t d = wdist(w, h * w.n + v);
    out[i] = (uint16_t)(d < 0xFFFFu ? d : 0xFFFFu);
  }
}

// Per vertex: how many of its first label entries have a landmark hub.
__global__ void __launch_bounds__(kBlock) k_ww_lskip(DWStore st, int32_t n, uint8_t *skip) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    const int64_t o = st.off[v];
    const int32_t len = st.len[v];
    int32_t c = 0;
    while (c < len && c < kWLand && (uint32_t)(st.ent[o + c] >> 32) < (uint32_t)kWLand) c++;
    skip[v] = (uint8_t)c;
  }
}

__global__ void k_wfinal_count(const int32_t *len, int64_t *cnt, int32_t n) {
  const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) cnt[r] = (int64_t)len[r] + 1;  // + sentinel
}

__global__ void __launch_bounds__(kBlock) k_wfinal_copy(DWStore st, const int64_t *foff,
                                                        uint64_t *fent, uint32_t *fpar,
                                                        int32_t n) {
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t r = wid; r < n; r += nw) {
    const int64_t o = st.off[r], fo = foff[r];
    const int32_t len = st.len[r];
    for (int32_t e = lane_id(); e < len; e += kWave) {
      fent[fo + e] = st.ent[o + e];
      if (fpar) fpar[fo + e] = st.par[o + e];
    }
    if (lane_id() == 0) {
      fent[fo + len] = kEmptyW;
      if (fpar) fpar[fo + len] = kSentinel;
    }
  }
}

// Queries: merge join (Section 3.3) over the packed labels, 64-bit sums.
__global__ void __launch_bounds__(kBlock) k_wquery_plain(DIndex ix, const int32_t *pairs, int64_t q,
                                                         uint32_t *out, const int32_t *err) {
  if (err && *err) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < q;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t rs = ix.rank[pairs[2 * i]], rt = ix.rank[pairs[2 * i + 1]];
    uint64_t best = kWInf;
    int64_t a = ix.off[rs], b = ix.toff[rt];
    for (;;) {
      const uint64_t ea = ix.went[a], eb = ix.twent[b];
      const uint32_t ha = (uint32_t)(ea >> 32), hb = (uint32_t)(eb >> 32);
      if (ha == hb) {
        if (ha == kSentinel) break;
        const uint64_t v = (ea & 0xFFFFFFFFull) + (eb & 0xFFFFFFFFull);
        best = v < best ? v : best;
        a++;
        b++;
      } else if (ha < hb) {
        a++;
      } else {
        b++;
      }
    }
    out[i] = (uint32_t)best;
  }
}

// G lanes per pair: chunks of G entries of both labels; each lane finds its
// source hub among the target chunk held in lanes by a halving search.
template <int G>
__global__ void __launch_bounds__(kBlock) k_wquery_group(DIndex ix, const int32_t *pairs, int64_t q,
                                                         uint32_t *out, const int32_t *err) {
  if (err && *err) return;
  const int gr = Group<G>::rank();
  const int gb = Group<G>::base();
  const int64_t gid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  const int64_t ngroups = ((int64_t)gridDim.x * blockDim.x) / G;
  for (int64_t i = gid; i < q; i += ngroups) {
    const int32_t rs = ix.rank[pairs[2 * i]], rt = ix.rank[pairs[2 * i + 1]];
    uint64_t best = kWInf;
    int64_t a = ix.off[rs], b = ix.toff[rt];
    const int64_t ea = ix.off[rs + 1], eb = ix.toff[rt + 1];
    for (;;) {
      const uint64_t xa = ix.went[a + gr < ea ? a + gr : ea - 1];
      const uint64_t xb = ix.twent[b + gr < eb ? b + gr : eb - 1];
      const uint32_t ha = (uint32_t)(xa >> 32), hb = (uint32_t)(xb >> 32);
      int lo = 0;
#pragma unroll
      for (int s = G / 2; s >= 1; s >>= 1) {
        const uint32_t hm = (uint32_t)__shfl((int)hb, gb + lo + s - 1);
        if (hm < ha) lo += s;
      }
      const uint32_t hf = (uint32_t)__shfl((int)hb, gb + lo);
      const uint32_t df = (uint32_t)__shfl((int)(uint32_t)xb, gb + lo);
      if (hf == ha && ha != kSentinel) {
        const uint64_t v = (xa & 0xFFFFFFFFull) + df;
        best = v < best ? v : best;
      }
      const uint32_t lastA = (uint32_t)__shfl((int)ha, gb + G - 1);
      const uint32_t lastB = (uint32_t)__shfl((int)hb, gb + G - 1);
      if (lastA == kSentinel && lastB == kSentinel) break;
      if (lastA <= lastB) a += G;
      if (lastB <= lastA) b += G;
    }
#pragma unroll
    for (int o = 1; o < G; o <<= 1) {
      const uint64_t v = __shfl_xor(best, o, G);
      best = v < best ? v : best;
    }
    if (gr == 0) out[i] = (uint32_t)best;
  }
}

// entry of hub h in the packed label of rank c, or -1
__device__ int64_t wfind_hub(const int64_t *off, const uint64_t *ent, int32_t c, uint32_t h) {
  int64_t lo = off[c], hi = off[c + 1] - 1;  // sentinel excluded
  const int64_t end = hi;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo) / 2;
    if ((uint32_t)(ent[mid] >> 32) < h)
      lo = mid + 1;
    else
      hi = mid;
  }
  return (lo < end && (uint32_t)(ent[lo] >> 32) == h) ? lo : -1;
}

// Vertices from rank c up the search tree of hub h (c first, h last):
// written at out[pos + dir * i] while i < room; returns the count, or -1 on
// a broken index.
__device__ int64_t wascend(const DIndex &ix, const int64_t *off, const uint64_t *ent,
                           const uint32_t *par, int32_t c, uint32_t h, int32_t *out, int64_t pos,
                           int64_t dir, int64_t room) {
  int64_t cnt = 0;
  for (;;) {
    if (out && cnt < room) out[pos + dir * cnt] = ix.ord[c];
    cnt++;
    if ((uint32_t)c == h) return cnt;
    if (cnt > ix.n) return -1;
    const int64_t e = wfind_hub(off, ent, c, h);
    if (e < 0) return -1;
    c = (int32_t)par[e];
  }
}

// Shortest paths of a weighted index kept with parents, one thread per
// pair: the best hub of the merge (first on ties), then the two search
// trees of the hub ascended (counted first, so a path that does not fit
// writes nothing).  lens = vertices on the path, 0 if unreachable,
// -(vertices) if maxlen is too small, INT32_MIN for a broken index.
__global__ void __launch_bounds__(kBlock) k_wquery_path(DIndex ix, const int32_t *pairs, int64_t q,
                                                        int32_t maxlen, int32_t *paths,
                                                        int32_t *lens, const int32_t *err) {
  if (err && *err) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < q;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t s = pairs[2 * i], t = pairs[2 * i + 1];
    const int32_t rs = ix.rank[s], rt = ix.rank[t];
    int32_t *out = paths + i * (int64_t)maxlen;
    if (rs == rt) {
      if (maxlen >= 1) out[0] = s;
      lens[i] = maxlen >= 1 ? 1 : -1;
      continue;
    }
    uint64_t best = kWInf;
    uint32_t h = kSentinel;
    int64_t a = ix.off[rs], b = ix.toff[rt];
    for (;;) {
      const uint64_t ea = ix.went[a], eb = ix.twent[b];
      const uint32_t ha = (uint32_t)(ea >> 32), hb = (uint32_t)(eb >> 32);
      if (ha == hb) {
        if (ha == kSentinel) break;
        const uint64_t v = (ea & 0xFFFFFFFFull) + (eb & 0xFFFFFFFFull);
        if (v < best) {
          best = v;
          h = ha;
        }
        a++;
        b++;
      } else if (ha < hb) {
        a++;
      } else {
        b++;
      }
    }
    if (best >= kWInf) {
      lens[i] = 0;
      continue;
    }
    const int64_t cs = wascend(ix, ix.off, ix.went, ix.par, rs, h, nullptr, 0, 1, 0);
    const int64_t ct = wascend(ix, ix.toff, ix.twent, ix.tpar, rt, h, nullptr, 0, 1, 0);
    if (cs < 0 || ct < 0) {
      lens[i] = INT32_MIN;
      continue;
    }
    const int64_t total = cs + ct - 1;
    if (total > maxlen) {
      lens[i] = (int32_t)-total;
      continue;
    }
    wascend(ix, ix.off, ix.went, ix.par, rs, h, out, 0, 1, total);
    wascend(ix, ix.toff, ix.twent, ix.tpar, rt, h, out, total - 1, -1, total);
    lens[i] = (int32_t)total;
  }
}

unsigned grid_for(int64_t items, int per_block, int64_t cap) {
  int64_t b = (items + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

}  // namespace

hipError_t launch_validate_weights(const uint32_t *w, int64_t nnz, int32_t *err, hipStream_t st) {
  if (nnz <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_validate_weights, dim3(grid_for(nnz, 256, 4096)), dim3(256), 0, st, w, nnz,
                     err);
  return hipGetLastError();
}

hipError_t launch_relabel_weights(const int32_t *in_row, const uint32_t *in_w, const int32_t *order,
                                  const int64_t *row, uint32_t *wt, int32_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_relabel_weights, dim3(grid_for((int64_t)n * kWave, kBlock, 8192)),
                     dim3(kBlock), 0, st, in_row, in_w, order, row, wt, n);
  return hipGetLastError();
}

hipError_t launch_ww_reset_ctl(WCtl *ctl, hipStream_t st) {
  hipLaunchKernelGGL(k_ww_reset_ctl, dim3(1), dim3(64), 0, st, ctl);
  return hipGetLastError();
}

hipError_t launch_ww_zero_list(WCtl *ctl, int list, hipStream_t st) {
  hipLaunchKernelGGL(k_ww_zero_list, dim3(1), dim3(64), 0, st, ctl, list);
  return hipGetLastError();
}

hipError_t launch_ww_init(DWStore tabsrc, DWWindow w, int64_t *sizes, int64_t *scan_tmp,
                          hipStream_t st) {
  if (w.W <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ww_ht_size, dim3((w.W + 1 + 255) / 256), dim3(256), 0, st, tabsrc, w,
                     sizes);
  hipError_t e = launch_exclusive_scan(sizes, w.htoff, (int64_t)w.W, scan_tmp, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_ww_init, dim3(grid_for((int64_t)w.W * kWave, kBlock, 1 << 20)),
                     dim3(kBlock), 0, st, tabsrc, w);
  return hipGetLastError();
}

hipError_t launch_ww_step(DWGraph g, DWStore s, DWWindow w, int cur, int group, hipStream_t st,
                          hipEvent_t ev0, hipEvent_t ev1) {
  switch (group) {
    case 4:
      PLL_LAUNCH_TIMED(k_ww_step<4>, dim3(kGrid), dim3(kBlock), st, ev0, ev1, g, s, w, cur);
      break;
    case 8:
      PLL_LAUNCH_TIMED(k_ww_step<8>, dim3(kGrid), dim3(kBlock), st, ev0, ev1, g, s, w, cur);
      break;
    case 32:
      PLL_LAUNCH_TIMED(k_ww_step<32>, dim3(kGrid), dim3(kBlock), st, ev0, ev1, g, s, w, cur);
      break;
    case 64:
      PLL_LAUNCH_TIMED(k_ww_step<64>, dim3(kGrid), dim3(kBlock), st, ev0, ev1, g, s, w, cur);
      break;
    default:
      PLL_LAUNCH_TIMED(k_ww_step<16>, dim3(kGrid), dim3(kBlock), st, ev0, ev1, g, s, w, cur);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_ww_collect(DWWindow w, hipStream_t st) {
  hipLaunchKernelGGL(k_ww_collect, dim3(kGrid), dim3(kBlock), 0, st, w);
  return hipGetLastError();
}

hipError_t launch_ww_clean(DWWindow w, DWWindow o, hipStream_t st) {
  hipLaunchKernelGGL(k_ww_clean, dim3(kGrid), dim3(kBlock), 0, st, w, o);
  return hipGetLastError();
}

hipError_t launch_ww_commit(DWWindow w, DWStore s, hipStream_t st) {
  hipLaunchKernelGGL(k_ww_commit_alloc, dim3(kGrid), dim3(kBlock), 0, st, w, s);
  hipLaunchKernelGGL(k_ww_commit_write, dim3(kGrid), dim3(kBlock), 0, st, w, s);
  hipLaunchKernelGGL(k_ww_commit_clear, dim3(kGrid), dim3(kBlock), 0, st, w);
  return hipGetLastError();
}

hipError_t launch_ww_reset(DWWindow w, hipStream_t st) {
  hipLaunchKernelGGL(k_ww_reset, dim3(kGrid), dim3(kBlock), 0, st, w);
  return hipGetLastError();
}

hipError_t launch_ww_landmarks(DWWindow w, uint16_t *out, hipStream_t st) {
  if (w.n <= 0 || w.W < kWLand) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_ww_landmarks, dim3(grid_for((int64_t)w.n * kWLand, kBlock, 8192)),
                     dim3(kBlock), 0, st, w, out);
  return hipGetLastError();
}

hipError_t launch_ww_lskip(DWStore s, int32_t n, uint8_t *skip, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ww_lskip, dim3(grid_for(n, kBlock, 8192)), dim3(kBlock), 0, st, s, n,
                     skip);
  return hipGetLastError();
}

hipError_t launch_wfinal_count(const int32_t *len, int64_t *cnt, int32_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_wfinal_count, dim3((n + 255) / 256), dim3(256), 0, st, len, cnt, n);
  return hipGetLastError();
}

hipError_t launch_wfinal_copy(DWStore s, const int64_t *foff, uint64_t *fent, uint32_t *fpar,
                              int32_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_wfinal_copy, dim3(grid_for((int64_t)n * kWave, kBlock, 8192)),
                     dim3(kBlock), 0, st, s, foff, fent, fpar, n);
  return hipGetLastError();
}

hipError_t launch_wquery_path(DIndex ix, const int32_t *pairs, int64_t q, int32_t maxlen,
                              int32_t *paths, int32_t *lens, const int32_t *err, hipStream_t st) {
  if (q <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_wquery_path, dim3(grid_for(q, kBlock, 16384)), dim3(kBlock), 0, st, ix,
                     pairs, q, maxlen, paths, lens, err);
  return hipGetLastError();
}

hipError_t launch_wquery(DIndex ix, const int32_t *pairs, int64_t q, uint32_t *out,
                         const int32_t *err, bool plain, int qgroup, hipStream_t st) {
  if (q <= 0) return hipSuccess;
  if (plain) {
    hipLaunchKernelGGL(k_wquery_plain, dim3(grid_for(q, 256, 65536)), dim3(256), 0, st, ix, pairs,
                       q, out, err);
    return hipGetLastError();
  }
  switch (qgroup) {
    case 16:
      hipLaunchKernelGGL(k_wquery_group<16>, dim3(grid_for(q * 16, 256, 16384)), dim3(256), 0, st,
                         ix, pairs, q, out, err);
      break;
    case 32:
      hipLaunchKernelGGL(k_wquery_group<32>, dim3(grid_for(q * 32, 256, 16384)), dim3(256), 0, st,
                         ix, pairs, q, out, err);
      break;
    default:
      hipLaunchKernelGGL(k_wquery_group<64>, dim3(grid_for(q * 64, 256, 16384)), dim3(256), 0, st,
                         ix, pairs, q, out, err);
      break;
  }
  return hipGetLastError();
}

}  // namespace pll
