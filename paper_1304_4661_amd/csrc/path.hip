// Shortest-path queries (Section 6, "Shortest-Path Queries"): every label
// entry (h, d) of v keeps the parent of v in the pruned BFS tree of h, so a
// path through the best common hub h is restored by ascending both trees.
// Of the vertices one step closer to h that the BFS from h labeled (any of
// them is a tree parent), the lowest-ranked one is kept, chosen after the
// build from the final labels (k_tree_parents), so parents do not depend on
// which concurrent search reached v first.
// Bit-parallel labels keep no tree; when a bit-parallel slot gives the
// distance, the path is walked through neighbours in ascending rank with
// the slot's distances and sets, always to the lowest-rank neighbour that
// fits: towards the root r (distance one less per step), towards a chosen
// neighbour w in S^{-1} (w stays in S^{-1} one level closer), or towards w
// in S^{0} (w in S^{0} one level closer, or in S^{-1} within the same level,
// then on as before).
//
// One wave per pair: the label merge and the tree ascent run on one lane,
// the neighbour scans of the bit-parallel walks on all 64.  For a digraph
// (no bit-parallel labels) the merge is of L_OUT(s) and L_IN(t).
#include <climits>

#include "pll_internal.h"

namespace pll {

namespace {

constexpr int kBlock = 256;

__global__ void k_invert_rank(const int32_t *rank, int32_t *ord, int32_t n) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x)
    ord[rank[v]] = (int32_t)v;
}

// entry of hub h in the label of rank c (sorted by hub rank), or -1
__device__ int64_t find_hub(const int64_t *off, const uint32_t *hub, int32_t c, uint32_t h) {
  int64_t lo = off[c], hi = off[c + 1] - 1;  // sentinel excluded
  const int64_t end = hi;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (hub[mid] < h)
      lo = mid + 1;
    else
      hi = mid;
  }
  return (lo < end && hub[lo] == h) ? lo : -1;
}

// Lowest-rank neighbour y of c with bit-parallel distance `want` in slot i
// and, when bit != 0, that bit in S^{-1}(y) (sel = 0) or S^{0}(y) (sel = 1);
// -1 if none.  The rank-space rows keep the input's neighbour order, so the
// whole row is scanned.  Called by the whole wave.
__device__ int32_t bp_scan(const DIndex &ix, int32_t c, int32_t i, int want, uint64_t bit,
                           int sel) {
  const int64_t a = ix.grow[c], b = ix.grow[c + 1];
  int best = INT_MAX;
  for (int64_t e0 = a; e0 < b; e0 += kWave) {
    const int64_t e = e0 + lane_id();
    int y = INT_MAX;
    if (e < b) {
      const int32_t x = ix.gcol[e];
      bool ok = (int)ix.bpd[(int64_t)x * ix.tpad + i] == want;
      if (ok && bit) ok = (ix.bpm[2 * ((int64_t)x * ix.t + i) + sel] & bit) != 0;
      if (ok) y = x;
    }
    y = Group<kWave>::min_reduce(y);
    best = y < best ? y : best;
  }
  return best == INT_MAX ? -1 : best;
}

// Walk from c on slot i (modes above: 0 to r, 1 to w in S^{-1}, 2 to w in
// S^{0}), writing ids at out[pos], out[pos + dir], ...  Returns the
// vertices written or -1.  Called by the whole wave.
__device__ int bp_walk(const DIndex &ix, int32_t c, int32_t i, uint64_t bit, int mode,
                       int32_t *out, int pos, int dir) {
  int nw = 0;
  for (int guard = 0; guard < 2 * (int)kInf8 + 4; guard++) {
    if (lane_id() == 0) out[pos] = ix.ord[c];
    pos += dir;
    nw++;
    const int dc = ix.bpd[(int64_t)c * ix.tpad + i];
    int32_t y;
    if (mode == 0) {
      if (dc == 0) return nw;
      y = bp_scan(ix, c, i, dc - 1, 0, 0);
    } else if (mode == 1) {
      if (dc == 1) return nw;  // c is w: S^{-1}(w) = {w} at level 1
      y = bp_scan(ix, c, i, dc - 1, bit, 0);
    } else {
      y = bp_scan(ix, c, i, dc - 1, bit, 1);
      if (y < 0) {
        y = bp_scan(ix, c, i, dc, bit, 0);
        if (y >= 0) mode = 1;
      }
    }
    if (y < 0) return -1;
    c = y;
  }
  return -1;
}

// Parents of the final labels.  The predecessors of a vertex u (row u of
// `pred`) are cut into chunks of kParChunk, one work item per chunk, so a
// high-degree vertex spreads over many waves.  k_tree_init gives the self
// entries their vertex and every other entry kSentinel; an item then takes
// the minimum, over its predecessors p, of p for each entry (h, d) of u with
// (h, d - 1) in L(p), and writes it (an atomic minimum when u has several
// items).  Labels of up to kParLds entries: L(u) is copied to LDS with a
// best-parent slot per entry and each predecessor's label streams through
// the wave, a lane per entry (h', d'): a binary search of h' in L(u) in
// LDS, and if u holds (h', d'+1), an LDS atomic minimum of p.  Longer
// labels: per entry of u, the lanes test the chunk's predecessors for
// (h, d - 1) by a binary search in global memory.
constexpr int kParLds = 1024;
constexpr int kParChunk = 64;
constexpr int kParWaves = kBlock / kWave;

__global__ void __launch_bounds__(kBlock) k_tree_init(const int64_t *foff, const uint8_t *fdist,
                                                      uint32_t *fpar, int32_t n) {
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t u = wid; u < n; u += nw) {
    const int64_t a = foff[u], b = foff[u + 1];  // sentinel at b - 1
    for (int64_t e = a + lane_id(); e < b; e += kWave)
      fpar[e] = (e < b - 1 && fdist[e] == 0) ? (uint32_t)u : kSentinel;
  }
}

__global__ void k_tree_count(DGraph pred, int64_t *cnt, int32_t n) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n;
       u += (int64_t)gridDim.x * blockDim.x) {
    const int64_t deg = pred.row[u + 1] - pred.row[u];
    cnt[u] = deg > 0 ? (deg + kParChunk - 1) / kParChunk : 0;
  }
}

// items[ioff[u] .. ioff[u+1]) = u
__global__ void __launch_bounds__(kBlock) k_tree_items(const int64_t *ioff, int32_t *items,
                                                       int32_t n) {
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t u = wid; u < n; u += nw)
    for (int64_t t = ioff[u] + lane_id(); t < ioff[u + 1]; t += kWave) items[t] = (int32_t)u;
}

__global__ void __launch_bounds__(kBlock) k_tree_parents(DGraph pred, const int64_t *foff,
                                                         const uint32_t *fhub,
                                                         const uint8_t *fdist, uint32_t *fpar,
                                                         const int64_t *ioff,
                                                         const int32_t *items, int64_t nitems) {
  __shared__ uint32_t s_h[kParWaves][kParLds];
  __shared__ int32_t s_best[kParWaves][kParLds];
  __shared__ uint8_t s_d[kParWaves][kParLds];
  const int wv = threadIdx.x / kWave;
  uint32_t *lh = s_h[wv];
  int32_t *lb = s_best[wv];
  uint8_t *ld = s_d[wv];
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t t = wid; t < nitems; t += nw) {
    const int32_t u = items[t];
    const bool single = ioff[u + 1] - ioff[u] == 1;  // no other item writes u's entries
    const int64_t a = foff[u], b = foff[u + 1] - 1;  // the sentinel sits at b
    const int32_t len = (int32_t)(b - a);
    const int64_t r0 = pred.row[u] + (t - ioff[u]) * kParChunk;
    const int64_t r1 = r0 + kParChunk < pred.row[u + 1] ? r0 + kParChunk : pred.row[u + 1];
    if (len <= kParLds) {
      for (int32_t i = lane_id(); i < len; i += kWave) {
        lh[i] = fhub[a + i];
        ld[i] = fdist[a + i];
        lb[i] = INT_MAX;
      }
      __threadfence_block();  // L(u) in LDS is visible to the whole wave
      for (int64_t x = r0; x < r1; x++) {
        const int32_t p = pred.col[x];
        const int64_t pa = foff[p], pb = foff[p + 1] - 1;
        for (int64_t e = pa + lane_id(); e < pb; e += kWave) {
          const uint32_t h = fhub[e];
          const int dp = fdist[e];
          int32_t lo = 0, hi = len;  // first entry of L(u) with hub >= h
          while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            if (lh[mid] < h)
              lo = mid + 1;
            else
              hi = mid;
          }
          if (lo < len && lh[lo] == h && (int)ld[lo] == dp + 1) atomicMin(&lb[lo], p);
        }
      }
      __threadfence_block();
      for (int32_t i = lane_id(); i < len; i += kWave) {
        if (lb[i] == INT_MAX) continue;
        if (single)
          fpar[a + i] = (uint32_t)lb[i];
        else
          atomicMin(&fpar[a + i], (uint32_t)lb[i]);
      }
      __threadfence_block();  // done with this wave's LDS before the next item
    } else {
      for (int64_t e = a; e < b; e++) {
        const uint32_t h = fhub[e];
        const int d = fdist[e];
        if (d == 0) continue;
        int y = INT_MAX;
        const int64_t x = r0 + lane_id();
        if (x < r1) {
          const int32_t p = pred.col[x];
          const int64_t f = find_hub(foff, fhub, p, h);
          if (f >= 0 && (int)fdist[f] == d - 1) y = p;
        }
        y = Group<kWave>::min_reduce(y);
        if (lane_id() == 0 && y != INT_MAX) {
          if (single)
            fpar[e] = (uint32_t)y;
          else
            atomicMin(&fpar[e], (uint32_t)y);
        }
      }
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_query_path(DIndex ix, const int32_t *pairs, int64_t q,
                                                       int32_t maxlen, int32_t *paths,
                                                       int32_t *lens, const int32_t *err) {
  if (err && *err) return;
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  const int lane = lane_id();
  for (int64_t pi = wid; pi < q; pi += nw) {
    const int32_t s = pairs[2 * pi], t = pairs[2 * pi + 1];
    const int32_t rs = ix.rank[s], rt = ix.rank[t];
    int32_t *out = paths + pi * (int64_t)maxlen;
    if (ix.rgid && ix.rgid[rs] != ix.rgid[rt]) {
      if (lane == 0) lens[pi] = 0;
      continue;
    }
    if (rs == rt) {
      if (lane == 0) {
        if (maxlen >= 1) out[0] = s;
        lens[pi] = maxlen >= 1 ? 1 : -1;
      }
      continue;
    }
    // normal part: best common hub, first on ties (one lane)
    int bn = 1 << 20;
    int64_t ia = -1, ib = -1;
    if (lane == 0) {
      int64_t i = ix.off[rs], j = ix.toff[rt];
      for (;;) {
        const uint32_t ha = ix.hub[i], hb = ix.thub[j];
        if (ha == hb) {
          if (ha == kSentinel) break;
          const int v = (int)ix.dist[i] + (int)ix.tdist[j];
          if (v < bn) {
            bn = v;
            ia = i;
            ib = j;
          }
          i++;
          j++;
        } else if (ha < hb) {
          i++;
        } else {
          j++;
        }
      }
    }
    bn = __shfl(bn, 0);
    ia = __shfl(ia, 0);
    ib = __shfl(ib, 0);
    // bit-parallel part: lane = slot; lowest slot on ties
    int key = INT_MAX, kind = 0;
    uint64_t wb = 0;
    if (lane < ix.t) {
      const int ds = ix.bpd[(int64_t)rs * ix.tpad + lane], dt = ix.bpd[(int64_t)rt * ix.tpad + lane];
      if (ds != kInf8 && dt != kInf8) {
        const uint64_t m1s = ix.bpm[2 * ((int64_t)rs * ix.t + lane)];
        const uint64_t m0s = ix.bpm[2 * ((int64_t)rs * ix.t + lane) + 1];
        const uint64_t m1t = ix.bpm[2 * ((int64_t)rt * ix.t + lane)];
        const uint64_t m0t = ix.bpm[2 * ((int64_t)rt * ix.t + lane) + 1];
        uint64_t m = 0;
        if (m1s & m1t) {
          kind = 2;
          m = m1s & m1t;
        } else if ((m1s & m0t) | (m0s & m1t)) {
          kind = 1;
          m = (m1s & m0t) ? (m1s & m0t) : (m0s & m1t);
        }
        wb = m & (~m + 1);
        key = (ds + dt - kind) * 64 + lane;
      }
    }
    const int best = Group<kWave>::min_reduce(key);
    const int bi = best == INT_MAX ? -1 : (best & 63);
    const int bb = best == INT_MAX ? (1 << 20) : (best >> 6);
    kind = __shfl(kind, bi < 0 ? 0 : bi);
    wb = __shfl(wb, bi < 0 ? 0 : bi);
    const int D = bn <= bb ? bn : bb;
    if (D >= (int)kInf8) {
      if (lane == 0) lens[pi] = 0;
      continue;
    }
    if (maxlen < D + 1) {
      if (lane == 0) lens[pi] = -(D + 1);
      continue;
    }
    bool ok = true;
    if (bn <= bb) {
      // ascend the BFS tree of h from s (positions 0..ds) and from t
      // (positions D down to ds+1); for a digraph the source side is L_OUT
      // (parents lead along the arcs to h), the target side L_IN (parents
      // lead back against the arcs to h)
      if (lane == 0) {
        const uint32_t h = ix.hub[ia];
        const int ds = ix.dist[ia], dt = ix.tdist[ib];
        int32_t c = rs;
        for (int k = 0; k <= ds && ok; k++) {
          out[k] = ix.ord[c];
          if (k < ds) {
            const int64_t e = find_hub(ix.off, ix.hub, c, h);
            if (e < 0) ok = false;
            else c = (int32_t)ix.par[e];
          }
        }
        c = rt;
        for (int k = 0; k < dt && ok; k++) {
          out[D - k] = ix.ord[c];
          const int64_t e = find_hub(ix.toff, ix.thub, c, h);
          if (e < 0) ok = false;
          else c = (int32_t)ix.tpar[e];
        }
        if (c != (int32_t)h) ok = false;
      }
      ok = __shfl(ok ? 1 : 0, 0) != 0;
    } else {
      const int ds = ix.bpd[(int64_t)rs * ix.tpad + bi], dt = ix.bpd[(int64_t)rt * ix.tpad + bi];
      const uint64_t m1s = ix.bpm[2 * ((int64_t)rs * ix.t + bi)];
      int ms, mt;
      if (kind == 0) {
        ms = 0;
        mt = 0;
      } else if (kind == 2) {
        ms = 1;
        mt = 1;
      } else if (m1s & wb) {
        ms = 1;
        mt = 2;
      } else {
        ms = 2;
        mt = 1;
      }
      const int ls = ms == 1 ? ds : ds + 1, lt = mt == 1 ? dt : dt + 1;
      const int a = bp_walk(ix, rs, bi, wb, ms, out, 0, 1);
      const int b = bp_walk(ix, rt, bi, wb, mt, out, D, -1);
      ok = a == ls && b == lt && ls + lt - 1 == D + 1;
    }
    if (lane == 0) lens[pi] = ok ? D + 1 : INT_MIN;
  }
}

unsigned grid_for(int64_t items, int per_block, int64_t cap) {
  int64_t b = (items + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

}  // namespace

hipError_t launch_invert_rank(const int32_t *rank, int32_t *ord, int32_t n, hipStream_t st) {
  if (n > 0)
    hipLaunchKernelGGL(k_invert_rank, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, rank, ord,
                       n);
  return hipGetLastError();
}

hipError_t launch_tree_count(DGraph pred, int64_t *cnt, int32_t n, hipStream_t st) {
  if (n > 0)
    hipLaunchKernelGGL(k_tree_count, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, pred, cnt, n);
  return hipGetLastError();
}

hipError_t launch_tree_parents(DGraph pred, const int64_t *foff, const uint32_t *fhub,
                               const uint8_t *fdist, uint32_t *fpar, int32_t n,
                               const int64_t *ioff, int32_t *items, int64_t nitems,
                               hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const unsigned gw = grid_for((int64_t)n * kWave, kBlock, 8192);
  hipLaunchKernelGGL(k_tree_init, dim3(gw), dim3(kBlock), 0, st, foff, fdist, fpar, n);
  if (nitems > 0) {
    hipLaunchKernelGGL(k_tree_items, dim3(gw), dim3(kBlock), 0, st, ioff, items, n);
    hipLaunchKernelGGL(k_tree_parents, dim3(grid_for(nitems * kWave, kBlock, 8192)),
                       dim3(kBlock), 0, st, pred, foff, fhub, fdist, fpar, ioff, items, nitems);
  }
  return hipGetLastError();
}

hipError_t launch_query_path(DIndex ix, const int32_t *pairs, int64_t q, int32_t maxlen,
                             int32_t *paths, int32_t *lens, const int32_t *err, hipStream_t st) {
  if (q <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_query_path, dim3(grid_for(q * kWave, kBlock, 4096)), dim3(kBlock), 0, st,
                     ix, pairs, q, maxlen, paths, lens, err);
  return hipGetLastError();
}

}  // namespace pll
