// Pruned phase of the small graphs of a batch, one workgroup per graph.
//
// Section 4.2 runs a pruned BFS from every vertex in rank order; for a graph
// of at most kGMaxN vertices one workgroup does exactly that, one root at a
// time: the root's label distances go into an LDS array indexed by hub
// (the T array of Section 4.5.1), the BFS runs level by level with one
// barrier per level, and each reached vertex is tested by one wave: first
// against the bit-parallel labels (Section 5.3), then by scanning its label
// against T.  A vertex that is not pruned gets the entry (root, distance)
// and its neighbours ranked after the root join the next level (one ranked
// before the root is always pruned: its own BFS, or the bit-parallel label
// it belongs to, already answers its distance to the root exactly).
//
// The grid is persistent: workgroups take graphs from a cursor, largest
// first, until the list is done.  Given query pairs, a workgroup answers a
// graph's pairs as soon as the graph's labels are complete.  Labels grow in the build's label store
// (reservations of 16-entry multiples from the shared pool top, doubled
// when full), so the finalisation and every query path read them as they
// read the labels of the windowed path.

#include "pll_internal.h"

namespace pll {
namespace {

constexpr int kGThreads = 1024;
constexpr int kGWaves = kGThreads / kWave;
constexpr int32_t kStop = 1 << 30;  // above any queue length
static_assert(kGMaxN % 32 == 0 && kGMaxN <= 65536, "LDS tables index with 16 bits");

// QUERY(s, t) over a graph's finished labels (in the store, sorted by hub,
// no sentinel), by one wave: the bit-parallel slots one per lane (Section
// 5.3), then a merge join of L(s) and L(t) by chunks of 64 hubs, each lane
// finding its hub of the L(s) chunk in the L(t) chunk by a halving search
// across the lanes (Section 3.3); clamped to 255.
__device__ __forceinline__ uint8_t wave_query(const DBp &bp, const DStore &st, int32_t rs,
                                              int32_t rt) {
  const int lane = lane_id();
  int best = kInf8;
  if (lane < bp.t) {
    const int ds = bp.d[(int64_t)rs * bp.tpad + lane], dt = bp.d[(int64_t)rt * bp.tpad + lane];
    if (ds != kInf8 && dt != kInf8) {
      const uint64_t *ms = bp.m + 2 * ((int64_t)rs * bp.t + lane);
      const uint64_t *mt = bp.m + 2 * ((int64_t)rt * bp.t + lane);
      best = bp_pair_dist(ds, ms[0], ms[1], dt, mt[0], mt[1]);
    }
  }
  constexpr uint32_t kPast = 0xFFFFFFFFu;  // above every hub rank
  const int64_t a = st.off[rs], b = st.off[rt];
  const int32_t la = st.len[rs], lb = st.len[rt];
  int32_t ia = 0, ib = 0;
  while (ia < la && ib < lb) {
    const uint32_t ha = ia + lane < la ? st.hub[a + ia + lane] : kPast;
    const uint32_t hb = ib + lane < lb ? st.hub[b + ib + lane] : kPast;
    int lo = 0;  // first lane whose hb >= ha (or 63)
#pragma unroll
    for (int s = kWave / 2; s >= 1; s >>= 1)
      if (__shfl(hb, lo + s - 1) < ha) lo += s;
    if (__shfl(hb, lo) == ha && ha != kPast) {
      const int v = (int)st.dist[a + ia + lane] + (int)st.dist[b + ib + lo];
      best = v < best ? v : best;
    }
    const uint32_t lastA = __shfl(ha, kWave - 1), lastB = __shfl(hb, kWave - 1);
    if (lastA <= lastB) ia += kWave;
    if (lastB <= lastA) ib += kWave;
  }
  best = Group<kWave>::min_reduce(best);
  return (uint8_t)(best < (int)kInf8 ? best : (int)kInf8);
}

__global__ void __launch_bounds__(kGThreads)
    k_graph_pruned(DGraph g, DBp bp, const uint8_t *used, DStore st, const int64_t *gbase,
                   const int32_t *gn, int32_t ngraphs, GraphCtl *ctl, GraphPairs qp) {
  __shared__ uint32_t s_T4[kGMaxN / 4];   // T: distance from the root per local hub, 255 = none
  __shared__ uint32_t s_vis[kGMaxN / 32];  // vertices reached by the current BFS
  __shared__ uint16_t s_q[kGMaxN];         // BFS queue (local ranks), levels one after another
  __shared__ uint8_t s_rd[64];             // the root's bit-parallel distances
  __shared__ uint64_t s_rm[64][2];         // ... and sets (S^{-1}, S^{0})
  // appends to the next level, by level mod 3; kStop marks a level after
  // which the graph stops (range or pool exhausted)
  __shared__ int32_t s_cnt[3];
  __shared__ int32_t s_gi, s_abort;
  uint8_t *s_T = reinterpret_cast<uint8_t *>(s_T4);

  const int tid = threadIdx.x, wv = tid / kWave, lane = lane_id();
  unsigned long long c_vis = 0, c_tests = 0, c_scan = 0, c_lab = 0, c_edges = 0;

  for (;;) {
    __syncthreads();  // the previous graph's reads of s_gi / s_abort are done
    if (tid == 0) {
      s_gi = __hip_atomic_load(&ctl->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                 ? ngraphs
                 : atomicAdd(&ctl->cursor, 1);
      s_abort = 0;
    }
    __syncthreads();
    const int32_t gi = s_gi;
    if (gi >= ngraphs) break;
    const int64_t base = gbase[gi];
    const int32_t ng = gn[gi];
    const uint32_t ub = (uint32_t)base;
    for (int i = tid; i < (ng + 3) / 4; i += kGThreads) s_T4[i] = 0xFFFFFFFFu;
    for (int i = tid; i < (ng + 31) / 32; i += kGThreads) s_vis[i] = 0u;
    __syncthreads();

    for (int32_t l = 0; l < ng; l++) {
      const int32_t R = (int32_t)(base + l);
      if (used[R]) continue;  // bit-parallel roots and their neighbours run no BFS
      // stage L(R) in T and the root's bit-parallel row
      {
        const int64_t ro = st.off[R];
        const int32_t rl = st.len[R];
        for (int32_t i = tid; i < rl; i += kGThreads) {
          const uint32_t h = st.hub[ro + i] - ub;
          if (h < (uint32_t)ng) s_T[h] = st.dist[ro + i];
        }
      }
      if (tid < bp.t) {
        s_rd[tid] = bp.d[(int64_t)R * bp.tpad + tid];
        const uint64_t *m = bp.m + 2 * ((int64_t)R * bp.t + tid);
        s_rm[tid][0] = m[0];
        s_rm[tid][1] = m[1];
      }
      if (tid == 0) {
        s_q[0] = (uint16_t)l;
        s_vis[l >> 5] |= 1u << (l & 31);
        s_cnt[0] = 0;
        s_cnt[1] = 0;
        s_cnt[2] = 0;
        // another workgroup failed: stop (s_abort is written only here,
        // between barriers that every thread's read of it lies between)
        if (__hip_atomic_load(&ctl->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
          s_abort = 1;
      }
      __syncthreads();
      if (s_abort) break;

      bool stop = false;
      int32_t lo = 0, hi = 1;
      for (int d = 0; lo < hi; d++) {
        // appends of this level go to s_cnt[d % 3]; s_cnt[(d + 1) % 3] was
        // last read before the barrier that opened this level
        if (tid == 0) s_cnt[(d + 1) % 3] = 0;
        for (int32_t i = lo + wv; i < hi; i += kGWaves) {
          const int32_t u = (int32_t)(base + s_q[i]);
          c_vis++;
          bool pruned = false;
          if (bp.t > 0) {
            bool hit = false;
            if (lane < bp.t) {
              const int du = bp.d[(int64_t)u * bp.tpad + lane];
              const int dr = s_rd[lane];
              // a slot can only prune if its distances allow it
              if (du != kInf8 && dr != kInf8 && du + dr - 2 <= d) {
                const uint64_t *m = bp.m + 2 * ((int64_t)u * bp.t + lane);
                hit = bp_pair_dist(dr, s_rm[lane][0], s_rm[lane][1], du, m[0], m[1]) <= d;
              }
            }
            pruned = __ballot(hit) != 0;
          }
          if (pruned) continue;
          c_tests++;
          const int64_t uo = st.off[u];
          const int32_t ulen = st.len[u];
          int32_t e0 = 0;
          for (; e0 < ulen && !pruned; e0 += kWave) {
            const int32_t e = e0 + lane;
            bool hit = false;
            if (e < ulen) {
              const uint32_t h = st.hub[uo + e] - ub;
              if (h < (uint32_t)ng) {
                const int th = s_T[h];
                hit = th != kInf8 && th + (int)st.dist[uo + e] <= d;
              }
            }
            pruned = __ballot(hit) != 0;
          }
          c_scan += (unsigned long long)(e0 < ulen ? e0 : ulen);
          if (pruned) continue;
          if (d >= (int)kInf8) {  // (R, 255) cannot be stored
            if (lane == 0) {
              atomicOr(&ctl->flags, kFlagRange);
              atomicOr(&s_cnt[d % 3], kStop);
            }
            continue;
          }
          // append (R, d) to L(u), moving the label to a slot twice as large
          // when it is full
          int64_t o = uo;
          const int32_t cap = st.cap[u];
          if (ulen >= cap) {
            const int64_t nc = cap < 8 ? 16 : 2 * (int64_t)cap;
            unsigned long long no = 0;
            if (lane == 0) no = atomicAdd(st.top, (unsigned long long)nc);
            no = __shfl(no, 0);
            if ((int64_t)no + nc > st.pool_cap) {
              if (lane == 0) {
                atomicOr(&ctl->flags, kFlagOvfPool);
                atomicOr(&s_cnt[d % 3], kStop);
              }
              continue;
            }
            for (int32_t e = lane; e < ulen; e += kWave) {
              st.hub[no + e] = st.hub[uo + e];
              st.dist[no + e] = st.dist[uo + e];
            }
            o = (int64_t)no;
            if (lane == 0) {
              st.off[u] = o;
              st.cap[u] = (int32_t)nc;
            }
          }
          if (lane == 0) {
            st.hub[o + ulen] = (uint32_t)R;
            st.dist[o + ulen] = (uint8_t)d;
            st.len[u] = ulen + 1;
            reinterpret_cast<uint64_t *>(st.hdr + u)[1] =
                (uint64_t)(o >> 4) | ((uint64_t)(uint32_t)(ulen + 1) << 32);
          }
          c_lab++;
          // next level: unreached neighbours ranked after the root
          const int64_t a = g.row[u], b = g.row[u + 1];
          c_edges += (unsigned long long)(b - a);
          for (int64_t x0 = a; x0 < b; x0 += kWave) {
            const int64_t x = x0 + lane;
            bool add = false;
            uint32_t wl = 0;
            if (x < b) {
              const int32_t w = g.col[x];
              wl = (uint32_t)w - ub;
              if (w > R && wl < (uint32_t)ng) {
                const uint32_t bit = 1u << (wl & 31);
                add = (atomicOr(&s_vis[wl >> 5], bit) & bit) == 0u;
              }
            }
            const uint64_t m = __ballot(add);
            if (m) {
              const int lead = __ffsll((unsigned long long)m) - 1;
              int32_t p0 = 0;
              if (lane == lead) p0 = atomicAdd(&s_cnt[d % 3], __popcll(m)) & (kStop - 1);
              p0 = __shfl(p0, lead);
              if (add) s_q[hi + p0 + __popcll(m & lanes_below_mask())] = (uint16_t)wl;
            }
          }
        }
        __syncthreads();
        const int32_t c = s_cnt[d % 3];
        if (c & kStop) {
          stop = true;  // every thread read the same word after the same barrier
          break;
        }
        lo = hi;
        hi += c;
      }
      // clear T and the visited bits for the next root
      for (int i = tid; i < (ng + 3) / 4; i += kGThreads) s_T4[i] = 0xFFFFFFFFu;
      for (int i = tid; i < (ng + 31) / 32; i += kGThreads) s_vis[i] = 0u;
      __syncthreads();
      if (stop) break;
    }
    // the graph's labels are complete: answer its pairs, a wave per pair
    if (qp.pairs && !s_abort) {
      for (int64_t i = qp.range[2 * gi] + wv; i < qp.range[2 * gi + 1]; i += kGWaves) {
        const uint8_t v = wave_query(bp, st, qp.rank[qp.pairs[2 * i]], qp.rank[qp.pairs[2 * i + 1]]);
        if (lane == 0) qp.out[i] = v;
      }
    }
  }
  if (lane == 0) {
    atomicAdd(&ctl->visited, c_vis);
    atomicAdd(&ctl->tests, c_tests);
    atomicAdd(&ctl->scanned, c_scan);
    atomicAdd(&ctl->labeled, c_lab);
    atomicAdd(&ctl->edges, c_edges);
  }
}

}  // namespace

hipError_t launch_graph_pruned(DGraph g, DBp bp, const uint8_t *used, DStore s,
                               const int64_t *gbase, const int32_t *gn, int32_t ngraphs,
                               GraphCtl *ctl, GraphPairs qp, int32_t grid, hipStream_t st) {
  if (ngraphs <= 0) return hipSuccess;
  if (bp.t > 64) return hipErrorInvalidValue;
  if (grid < 1) grid = 1;
  if (grid > ngraphs) grid = ngraphs;
  hipLaunchKernelGGL(k_graph_pruned, dim3((unsigned)grid), dim3(kGThreads), 0, st, g, bp, used,
                     s, gbase, gn, ngraphs, ctl, qp);
  return hipGetLastError();
}

}  // namespace pll
