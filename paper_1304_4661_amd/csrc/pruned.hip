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

__global__ void k_win_reset_ctl(LevelCtl *ctl) {
  unsigned long long *p = reinterpret_cast<unsigned long long *>(ctl);
  const int words = (int)(sizeof(LevelCtl) / sizeof(unsigned long long));
  for (int i = threadIdx.x; i < words; i += blockDim.x) p[i] = 0;
}

// Block j: root k = s + j.  Scatter L(k) into T[j][.], mark k visited and
// put (j, k) on level 0.  Bit-parallel roots and neighbours run no pruned
// BFS (they would prune themselves at distance 0).
__global__ void __launch_bounds__(kBlock) k_win_init(DGraph g, DWindow w, DStore st, DFrontier f) {
  const int32_t j = blockIdx.x;
  const int32_t k = w.s + j;
  if (w.used[k]) return;
  uint8_t *Tj = w.T + (int64_t)j * g.n;
  const int64_t o = st.off[k];
  const int32_t len = st.len[k];
  for (int32_t e = threadIdx.x; e < len; e += blockDim.x) Tj[st.hub[o + e]] = st.dist[o + e];
  if (threadIdx.x == 0) {
    atomicOr(&w.vis[(int64_t)j * g.nwords + (k >> 5)], 1u << (k & 31));
    const unsigned long long p = atomicAdd(&f.ctl->cnt[0], 1ull);
    f.slot[p] = j;
    f.v[p] = k;
  }
}

// Full prune test of one vertex by one lane (used only for the rare vertex
// at distance 255, to decide whether the build must fail).
__device__ bool prune_test_serial(DBp bp, DStore st, const uint8_t *Tj, int32_t k, int32_t u,
                                  int d) {
  for (int32_t i = 0; i < bp.t; i++) {
    const int dk = bp.d[(int64_t)k * bp.t + i], du = bp.d[(int64_t)u * bp.t + i];
    if (dk == kInf8 || du == kInf8) continue;
    const uint64_t *mk = bp.m + 2 * ((int64_t)k * bp.t + i);
    const uint64_t *mu = bp.m + 2 * ((int64_t)u * bp.t + i);
    if (bp_pair_dist(dk, mk[0], mk[1], du, mu[0], mu[1]) <= d) return true;
  }
  const int64_t o = st.off[u];
  const int32_t len = st.len[u];
  for (int32_t e = 0; e < len; e++) {
    const int th = Tj[st.hub[o + e]];
    if (th != kInf8 && st.dist[o + e] + th <= d) return true;
  }
  return false;
}

// One BFS level of every root of the window.  A group of G lanes takes one
// (root slot j, vertex u) entry at distance d: bit-parallel test over the
// slots, then the normal-label test against T[j] (prune iff some hub gives
// <= d), else record the candidate label (k, d) and push u's unvisited
// neighbours to level d+1.  Long adjacency lists: the first `chunk` edges
// here, the rest as tasks for whole waves.
template <int G>
__global__ void __launch_bounds__(kBlock) k_win_level(DGraph g, DBp bp, DStore st, DWindow w,
                                                      DFrontier f, int d, int chunk) {
  LevelCtl *ctl = f.ctl;
  const unsigned long long beg = ctl->base[d], cnt = ctl->cnt[d];
  const unsigned long long nbase = beg + cnt;
  if (blockIdx.x == 0 && threadIdx.x == 0) ctl->base[d + 1] = nbase;
  // after an overflow the window is redone; never read past the buffer
  if (cnt == 0 || (ctl->flags & kOverflowFlags) || nbase > (unsigned long long)f.cap) return;
  const int64_t n = g.n;
  const int32_t t = bp.t;
  const int gr = Group<G>::rank();
  const int64_t gid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  const int64_t ngroups = ((int64_t)gridDim.x * blockDim.x) / G;
  // work counters, per lane (group leaders), summed once per wave at the end
  unsigned long long c_visit = 0, c_test = 0, c_scan = 0, c_lab = 0, c_edge = 0;
  for (int64_t p = gid; p < (int64_t)cnt; p += ngroups) {
    const int32_t j = f.slot[beg + p];
    const int32_t u = f.v[beg + p];
    const int32_t k = w.s + j;
    if (gr == 0) c_visit++;
    // bit-parallel labels first (Section 5.4)
    bool pr = false;
    for (int32_t i = gr; i < t; i += G) {
      const int dk = bp.d[(int64_t)k * t + i], du = bp.d[(int64_t)u * t + i];
      if (dk != kInf8 && du != kInf8 && dk + du - 2 <= d) {
        const uint64_t *mk = bp.m + 2 * ((int64_t)k * t + i);
        const uint64_t *mu = bp.m + 2 * ((int64_t)u * t + i);
        if (bp_pair_dist(dk, mk[0], mk[1], du, mu[0], mu[1]) <= d) pr = true;
      }
    }
    pr = Group<G>::any(pr);
    if (!pr) {
      const uint8_t *Tj = w.T + (int64_t)j * n;
      const int64_t o = st.off[u];
      const int32_t len = st.len[u];
      if (gr == 0) {
        c_test++;
        c_scan += (unsigned long long)len;
      }
      for (int32_t e = gr; e < len; e += G) {
        const int th = Tj[st.hub[o + e]];
        if (th != kInf8 && st.dist[o + e] + th <= d) pr = true;
      }
      pr = Group<G>::any(pr);
    }
    if (pr) continue;
    // label (k, d) for u, pending cleaning
    if (gr == 0) c_lab++;
    const int64_t c = wave_append(gr == 0, &ctl->ccnt);
    if (c >= 0) {
      if (c < w.ccap) {
        w.cu[c] = u;
        w.cj[c] = j;
        w.cd[c] = (uint8_t)d;
        w.wd[(int64_t)u * (w.words * 64) + j] = (uint8_t)d;
        atomicOr((unsigned long long *)&w.cmask[(int64_t)u * w.words + (j >> 6)],
                 1ull << (j & 63));
      } else {
        atomicOr(&ctl->flags, kFlagOvfCand);
      }
    }
    const int64_t e0 = g.row[u];
    const int64_t deg = g.row[u + 1] - e0;
    uint32_t *vs = w.vis + (int64_t)j * g.nwords;
    if (d + 1 >= (int)kInf8) {
      // neighbours would sit at distance 255: fine only if all are pruned
      const uint8_t *Tj = w.T + (int64_t)j * n;
      for (int64_t e = gr; e < deg; e += G) {
        const int32_t x = g.col[e0 + e];
        if ((vs[x >> 5] >> (x & 31)) & 1u) continue;
        if (!prune_test_serial(bp, st, Tj, k, x, d + 1)) atomicOr(&ctl->flags, kFlagRange);
      }
      continue;
    }
    const int64_t lim = deg < chunk ? deg : chunk;
    if (gr == 0) c_edge += (unsigned long long)lim;
    for (int64_t e = gr; e < lim; e += G) {
      const int32_t x = g.col[e0 + e];
      const uint32_t bit = 1u << (x & 31);
      bool claimed = false;
      if (!(vs[x >> 5] & bit)) claimed = !(atomicOr(&vs[x >> 5], bit) & bit);
      const int64_t pos = wave_append(claimed, &ctl->cnt[d + 1]);
      if (pos >= 0) {
        if ((int64_t)nbase + pos < f.cap) {
          f.slot[nbase + pos] = j;
          f.v[nbase + pos] = x;
        } else {
          atomicOr(&ctl->flags, kFlagOvfFrontier);
        }
      }
    }
    if (deg > chunk) {
      const int64_t extra = (deg + chunk - 1) / chunk - 1;
      unsigned long long tb = 0;
      if (gr == 0) tb = atomicAdd(&ctl->hcnt[d], (unsigned long long)extra);
      tb = __shfl(tb, Group<G>::base());
      for (int64_t q = gr; q < extra; q += G) {
        if ((int64_t)tb + q < f.hcap) {
          f.hslot[tb + q] = j;
          f.hv[tb + q] = u;
          f.hchunk[tb + q] = (int32_t)(q + 1);
        } else {
          atomicOr(&ctl->flags, kFlagOvfHeavy);
        }
      }
    }
  }
  c_visit = Group<kWave>::sum_reduce(c_visit);
  c_test = Group<kWave>::sum_reduce(c_test);
  c_scan = Group<kWave>::sum_reduce(c_scan);
  c_lab = Group<kWave>::sum_reduce(c_lab);
  c_edge = Group<kWave>::sum_reduce(c_edge);
  if (lane_id() == 0 && c_visit) {
    atomicAdd(&ctl->visited, c_visit);
    atomicAdd(&ctl->ntests, c_test);
    atomicAdd(&ctl->lscanned, c_scan);
    atomicAdd(&ctl->labeled, c_lab);
    atomicAdd(&ctl->edges, c_edge);
  }
}

__global__ void __launch_bounds__(kBlock) k_win_heavy(DGraph g, DWindow w, DFrontier f, int d,
                                                      int chunk) {
  LevelCtl *ctl = f.ctl;
  const unsigned long long ntask = ctl->hcnt[d];
  if (ntask == 0 || (ctl->flags & kOverflowFlags)) return;
  const int64_t ntasks = (int64_t)ntask < f.hcap ? (int64_t)ntask : f.hcap;
  const unsigned long long nbase = ctl->base[d] + ctl->cnt[d];
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t tk = wid; tk < ntasks; tk += nw) {
    const int32_t j = f.hslot[tk], u = f.hv[tk], c = f.hchunk[tk];
    const int64_t e0 = g.row[u], e1 = g.row[u + 1];
    const int64_t a = e0 + (int64_t)c * chunk;
    const int64_t b = a + chunk < e1 ? a + chunk : e1;
    uint32_t *vs = w.vis + (int64_t)j * g.nwords;
    if (lane_id() == 0) atomicAdd(&ctl->hedges, (unsigned long long)(b - a));
    for (int64_t e = a + lane_id(); e < b; e += kWave) {
      const int32_t x = g.col[e];
      const uint32_t bit = 1u << (x & 31);
      bool claimed = false;
      if (!(vs[x >> 5] & bit)) claimed = !(atomicOr(&vs[x >> 5], bit) & bit);
      const int64_t pos = wave_append(claimed, &ctl->cnt[d + 1]);
      if (pos >= 0) {
        if ((int64_t)nbase + pos < f.cap) {
          f.slot[nbase + pos] = j;
          f.v[nbase + pos] = x;
        } else {
          atomicOr(&ctl->flags, kFlagOvfFrontier);
        }
      }
    }
  }
}

// Clear visited words of every (slot, vertex) ever put on the frontier, and
// each root's row of T.
__global__ void __launch_bounds__(kBlock) k_win_reset_vis(DGraph g, DWindow w, DFrontier f,
                                                          int64_t nvisited) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nvisited;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t j = f.slot[p], x = f.v[p];
    w.vis[(int64_t)j * g.nwords + (x >> 5)] = 0u;
  }
}

__global__ void __launch_bounds__(kBlock) k_win_reset_T(DGraph g, DWindow w, DStore st) {
  const int32_t j = blockIdx.x;
  const int32_t k = w.s + j;
  if (w.used[k]) return;
  uint8_t *Tj = w.T + (int64_t)j * g.n;
  const int64_t o = st.off[k];
  const int32_t len = st.len[k];
  for (int32_t e = threadIdx.x; e < len; e += blockDim.x) Tj[st.hub[o + e]] = kInf8;
}

// Drop the window's candidates (a window is re-run smaller after an overflow).
__global__ void __launch_bounds__(kBlock) k_win_abort(DWindow w, int64_t ncand) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncand;
       c += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = w.cu[c];
    w.wd[(int64_t)u * (w.words * 64) + w.cj[c]] = kInf8;
    for (int i = 0; i < w.words; i++) w.cmask[(int64_t)u * w.words + i] = 0ull;
  }
}

// Cleaning: candidate (k = s+j, d) of u survives iff no window root j' < j
// labeled both u and v_k with d(j',u) + d(j',v_k) <= d.  Also marks one
// candidate per vertex (the lowest j) to commit the vertex's row.
__global__ void __launch_bounds__(kBlock) k_win_clean(DWindow w, int64_t ncand) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncand;
       c += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = w.cu[c], j = w.cj[c];
    const int d = w.cd[c];
    const int32_t k = w.s + j;
    const uint64_t *cu_row = w.cmask + (int64_t)u * w.words;
    const uint64_t *ck_row = w.cmask + (int64_t)k * w.words;
    const uint8_t *wu = w.wd + (int64_t)u * (w.words * 64);
    const uint8_t *wk = w.wd + (int64_t)k * (w.words * 64);
    const int jw = j >> 6, jb = j & 63;
    bool drop = false;
    for (int i = 0; i <= jw && !drop; i++) {
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
    if (!drop)
      atomicOr((unsigned long long *)&w.kmask[(int64_t)u * w.words + jw], 1ull << jb);
    int low = -1;
    for (int i = 0; i < w.words; i++) {
      if (cu_row[i]) {
        low = i * 64 + __ffsll((unsigned long long)cu_row[i]) - 1;
        break;
      }
    }
    w.cdes[c] = (low == j) ? 1 : 0;
  }
}

// Commit: one thread per touched vertex appends its surviving labels in
// root order (labels stay sorted by hub rank, Section 4.5.1), growing its
// slot in the pool when full, and clears the vertex's window rows.
__global__ void __launch_bounds__(kBlock) k_win_commit(DWindow w, DStore st, int64_t ncand) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncand;
       c += (int64_t)gridDim.x * blockDim.x) {
    if (!w.cdes[c]) continue;
    const int32_t u = w.cu[c];
    uint64_t *crow = w.cmask + (int64_t)u * w.words;
    uint64_t *krow = w.kmask + (int64_t)u * w.words;
    uint8_t *wu = w.wd + (int64_t)u * (w.words * 64);
    int32_t total = 0;
    for (int i = 0; i < w.words; i++) total += __popcll(krow[i]);
    if (total > 0) {
      const int32_t len = st.len[u];
      const int32_t need = len + total;
      if (need > st.cap[u]) {
        int64_t nc = 2 * (int64_t)need;
        if (nc < 16) nc = 16;
        nc = (nc + 15) & ~(int64_t)15;
        const int64_t no = (int64_t)atomicAdd(st.top, (unsigned long long)nc);
        const int64_t oo = st.off[u];
        for (int32_t e = 0; e < len; e++) {
          st.hub[no + e] = st.hub[oo + e];
          st.dist[no + e] = st.dist[oo + e];
        }
        st.off[u] = no;
        st.cap[u] = (int32_t)nc;
      }
      int64_t o = st.off[u] + len;
      for (int i = 0; i < w.words; i++) {
        uint64_t m = krow[i];
        while (m) {
          const int b = __ffsll((unsigned long long)m) - 1;
          m &= m - 1;
          const int jj = i * 64 + b;
          st.hub[o] = (uint32_t)(w.s + jj);
          st.dist[o] = wu[jj];
          o++;
        }
      }
      st.len[u] = need;
    }
    for (int i = 0; i < w.words; i++) {
      uint64_t m = crow[i];
      while (m) {
        const int b = __ffsll((unsigned long long)m) - 1;
        m &= m - 1;
        wu[i * 64 + b] = kInf8;
      }
      crow[i] = 0ull;
      krow[i] = 0ull;
    }
  }
}

__global__ void k_final_count(const int32_t *len, int64_t *cnt, int32_t n) {
  const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) cnt[r] = (int64_t)len[r] + 1;  // + sentinel
}

// One wave per vertex: copy its label into the final CSR and close it with
// the storage-only sentinel (Section 4.5.2).
__global__ void __launch_bounds__(kBlock) k_final_copy(DStore st, const int64_t *foff,
                                                       uint32_t *fhub, uint8_t *fdist, int32_t n) {
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

template <int G>
void launch_level_g(DGraph g, DBp bp, DStore st, DWindow w, DFrontier f, int d, int chunk,
                    hipStream_t s, int blocks, hipEvent_t ev0, hipEvent_t ev1) {
  if (ev0) (void)hipEventRecord(ev0, s);
  hipLaunchKernelGGL(k_win_level<G>, dim3(blocks), dim3(kBlock), 0, s, g, bp, st, w, f, d, chunk);
  if (ev1) (void)hipEventRecord(ev1, s);
  hipLaunchKernelGGL(k_win_heavy, dim3(blocks), dim3(kBlock), 0, s, g, w, f, d, chunk);
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
                           hipStream_t st) {
  if (nroots <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_win_init, dim3(nroots), dim3(kBlock), 0, st, g, w, s, f);
  return hipGetLastError();
}

hipError_t launch_win_level(DGraph g, DBp bp, DStore s, DWindow w, DFrontier f, int d, int group,
                            int chunk, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  const int blocks = 2048;
  switch (group) {
    case 4: launch_level_g<4>(g, bp, s, w, f, d, chunk, st, blocks, ev0, ev1); break;
    case 8: launch_level_g<8>(g, bp, s, w, f, d, chunk, st, blocks, ev0, ev1); break;
    case 16: launch_level_g<16>(g, bp, s, w, f, d, chunk, st, blocks, ev0, ev1); break;
    case 32: launch_level_g<32>(g, bp, s, w, f, d, chunk, st, blocks, ev0, ev1); break;
    default: launch_level_g<64>(g, bp, s, w, f, d, chunk, st, blocks, ev0, ev1); break;
  }
  return hipGetLastError();
}

hipError_t launch_win_reset(DGraph g, DWindow w, DStore s, DFrontier f, int32_t nroots,
                            int64_t nvisited, hipStream_t st) {
  if (nvisited > 0)
    hipLaunchKernelGGL(k_win_reset_vis, dim3(grid_for(nvisited, kBlock, 8192)), dim3(kBlock), 0,
                       st, g, w, f, nvisited);
  if (nroots > 0) hipLaunchKernelGGL(k_win_reset_T, dim3(nroots), dim3(kBlock), 0, st, g, w, s);
  return hipGetLastError();
}

hipError_t launch_win_abort(DGraph /*g*/, DWindow w, int64_t ncand, hipStream_t st) {
  if (ncand > 0)
    hipLaunchKernelGGL(k_win_abort, dim3(grid_for(ncand, kBlock, 8192)), dim3(kBlock), 0, st, w,
                       ncand);
  return hipGetLastError();
}

hipError_t launch_win_clean(DWindow w, int64_t ncand, hipStream_t st) {
  if (ncand > 0)
    hipLaunchKernelGGL(k_win_clean, dim3(grid_for(ncand, kBlock, 8192)), dim3(kBlock), 0, st, w,
                       ncand);
  return hipGetLastError();
}

hipError_t launch_win_commit(DWindow w, DStore s, int64_t ncand, hipStream_t st) {
  if (ncand > 0)
    hipLaunchKernelGGL(k_win_commit, dim3(grid_for(ncand, kBlock, 8192)), dim3(kBlock), 0, st, w,
                       s, ncand);
  return hipGetLastError();
}

hipError_t launch_final_count(const int32_t *len, int64_t *cnt, int32_t n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_final_count, dim3((n + 255) / 256), dim3(256), 0, st, len, cnt, n);
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
