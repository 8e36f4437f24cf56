// Bit-parallel BFS (Algorithm 3, Section 5.2) for all slots at once.
//
// Each slot i has a root r and up to 64 neighbours S_r.  Per slot and vertex
// v the BFS computes d(r, v), S^{-1}(v) = members of S_r one step closer to
// v than r, and S^{0}(v) = members as far from v as r (Section 5.1).  The
// slots are independent once chosen, so all of them advance together: the
// frontier is a list of (slot, vertex) pairs, one level per launch pair.
//
// Level L, in the order the dynamic programme of Section 5.2 needs:
//   (a) over the level-L vertices: discover level L+1 (claim unvisited
//       neighbours) and, for same-level neighbours y, S^0(v) |= S^{-1}(y)
//       (the E0 edges);
//   (c) over the level-(L+1) vertices: for neighbours y at level L,
//       S^{-1}(u) |= S^{-1}(y) and S^{0}(u) |= S^{0}(y) (the E1 edges).
// Both are pulls: each vertex ORs what its neighbours hold, so a vertex's own
// sets are written by one group (or by atomics when its adjacency list is
// split into chunks), and (c) only runs after (a) has finished the level.
//
// Arrays are slot-major here (bd[s*n+v], bs1/bs0 likewise) so a slot's BFS
// touches one contiguous region; k_bp_finish transposes them to the
// vertex-major layout the pruned phase and the queries read.
#include "pll_internal.h"

namespace pll {

namespace {

constexpr int kBlock = 256;

template <int G>
__global__ void __launch_bounds__(kBlock) k_bp_a(DGraph g, int L, int chunk, uint8_t *bd,
                                                 const uint64_t *bs1, uint64_t *bs0,
                                                 uint32_t *vis, DFrontier f) {
  LevelCtl *ctl = f.ctl;
  const unsigned long long beg = ctl->base[L], cnt0 = ctl->cnt[L];
  const unsigned long long nbase = beg + cnt0;
  if (blockIdx.x == 0 && threadIdx.x == 0) ctl->base[L + 1] = nbase;
  // after an overflow the window is redone; never read past the buffer
  if (cnt0 == 0 || (ctl->flags & kOverflowFlags) || nbase > (unsigned long long)f.cap) return;
  const unsigned long long cnt = cnt0;
  const int64_t n = g.n;
  const int gr = Group<G>::rank();
  const int64_t gid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  const int64_t ngroups = ((int64_t)gridDim.x * blockDim.x) / G;
  for (int64_t p = gid; p < (int64_t)cnt; p += ngroups) {
    const int32_t s = f.slot[beg + p];
    const int32_t v = f.v[beg + p];
    const int64_t e0 = g.row[v];
    const int64_t deg = g.row[v + 1] - e0;
    const int64_t lim = deg < chunk ? deg : chunk;
    uint8_t *bds = bd + (int64_t)s * n;
    const uint64_t *b1 = bs1 + (int64_t)s * n;
    uint32_t *vs = vis + (int64_t)s * g.nwords;
    uint64_t acc = 0;
    for (int64_t e = gr; e < lim; e += G) {
      const int32_t u = g.col[e0 + e];
      const uint8_t du = bds[u];
      bool claimed = false;
      if (du == kInf8) {
        const uint32_t bit = 1u << (u & 31);
        if (!(vs[u >> 5] & bit)) claimed = !(atomicOr(&vs[u >> 5], bit) & bit);
      } else if (du == L) {
        acc |= b1[u];
      }
      if (claimed && L + 1 >= (int)kInf8) atomicOr(&ctl->flags, kFlagRange);
      const bool push = claimed && L + 1 < (int)kInf8;
      if (push) bds[u] = (uint8_t)(L + 1);
      const int64_t pos = wave_append(push, &ctl->cnt[L + 1]);
      if (pos >= 0) {
        if ((int64_t)nbase + pos < f.cap) {
          f.slot[nbase + pos] = s;
          f.v[nbase + pos] = u;
        } else {
          atomicOr(&ctl->flags, kFlagOvfFrontier);
        }
      }
    }
    acc = Group<G>::or_reduce(acc);
    if (gr == 0 && acc) bs0[(int64_t)s * n + v] |= acc;
    if (deg > chunk) {
      const int64_t extra = (deg + chunk - 1) / chunk - 1;
      unsigned long long tb = 0;
      if (gr == 0) tb = atomicAdd(&ctl->hcnt[L], (unsigned long long)extra);
      tb = __shfl(tb, Group<G>::base());
      for (int64_t k = gr; k < extra; k += G) {
        if ((int64_t)tb + k < f.hcap) {
          f.hslot[tb + k] = s;
          f.hv[tb + k] = v;
          f.hchunk[tb + k] = (int32_t)(k + 1);
        } else {
          atomicOr(&ctl->flags, kFlagOvfHeavy);
        }
      }
    }
  }
}

// One wave per chunk of a long adjacency list left over by k_bp_a.
__global__ void __launch_bounds__(kBlock) k_bp_a_heavy(DGraph g, int L, int chunk, uint8_t *bd,
                                                       const uint64_t *bs1, uint64_t *bs0,
                                                       uint32_t *vis, DFrontier f) {
  LevelCtl *ctl = f.ctl;
  const unsigned long long ntask = ctl->hcnt[L];
  if (ntask == 0 || (ctl->flags & kOverflowFlags)) return;
  const int64_t ntasks = (int64_t)ntask < f.hcap ? (int64_t)ntask : f.hcap;
  const unsigned long long nbase = ctl->base[L] + ctl->cnt[L];
  const int64_t n = g.n;
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t tk = wid; tk < ntasks; tk += nw) {
    const int32_t s = f.hslot[tk], v = f.hv[tk], c = f.hchunk[tk];
    const int64_t e0 = g.row[v], e1 = g.row[v + 1];
    const int64_t a = e0 + (int64_t)c * chunk;
    const int64_t b = a + chunk < e1 ? a + chunk : e1;
    uint8_t *bds = bd + (int64_t)s * n;
    const uint64_t *b1 = bs1 + (int64_t)s * n;
    uint32_t *vs = vis + (int64_t)s * g.nwords;
    uint64_t acc = 0;
    for (int64_t e = a + lane_id(); e < b; e += kWave) {
      const int32_t u = g.col[e];
      const uint8_t du = bds[u];
      bool claimed = false;
      if (du == kInf8) {
        const uint32_t bit = 1u << (u & 31);
        if (!(vs[u >> 5] & bit)) claimed = !(atomicOr(&vs[u >> 5], bit) & bit);
      } else if (du == L) {
        acc |= b1[u];
      }
      if (claimed && L + 1 >= (int)kInf8) atomicOr(&ctl->flags, kFlagRange);
      const bool push = claimed && L + 1 < (int)kInf8;
      if (push) bds[u] = (uint8_t)(L + 1);
      const int64_t pos = wave_append(push, &ctl->cnt[L + 1]);
      if (pos >= 0) {
        if ((int64_t)nbase + pos < f.cap) {
          f.slot[nbase + pos] = s;
          f.v[nbase + pos] = u;
        } else {
          atomicOr(&ctl->flags, kFlagOvfFrontier);
        }
      }
    }
    acc = Group<kWave>::or_reduce(acc);
    if (lane_id() == 0 && acc) atomicOr((unsigned long long *)&bs0[(int64_t)s * n + v],
                                        (unsigned long long)acc);
  }
}

template <int G>
__global__ void __launch_bounds__(kBlock) k_bp_c(DGraph g, int L, int chunk, const uint8_t *bd,
                                                 uint64_t *bs1, uint64_t *bs0, DFrontier f) {
  LevelCtl *ctl = f.ctl;
  const unsigned long long beg = ctl->base[L + 1], cnt = ctl->cnt[L + 1];
  if (cnt == 0 || (ctl->flags & kOverflowFlags) || beg + cnt > (unsigned long long)f.cap) return;
  const int64_t n = g.n;
  const int gr = Group<G>::rank();
  const int64_t gid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  const int64_t ngroups = ((int64_t)gridDim.x * blockDim.x) / G;
  for (int64_t p = gid; p < (int64_t)cnt; p += ngroups) {
    const int32_t s = f.slot[beg + p];
    const int32_t u = f.v[beg + p];
    const int64_t e0 = g.row[u];
    const int64_t deg = g.row[u + 1] - e0;
    const int64_t lim = deg < chunk ? deg : chunk;
    const uint8_t *bds = bd + (int64_t)s * n;
    const uint64_t *b1 = bs1 + (int64_t)s * n;
    const uint64_t *b0 = bs0 + (int64_t)s * n;
    uint64_t a1 = 0, a0 = 0;
    for (int64_t e = gr; e < lim; e += G) {
      const int32_t y = g.col[e0 + e];
      if (bds[y] == L) {
        a1 |= b1[y];
        a0 |= b0[y];
      }
    }
    a1 = Group<G>::or_reduce(a1);
    a0 = Group<G>::or_reduce(a0);
    if (gr == 0) {
      if (a1) bs1[(int64_t)s * n + u] |= a1;
      if (a0) bs0[(int64_t)s * n + u] |= a0;
    }
    if (deg > chunk) {
      const int64_t extra = (deg + chunk - 1) / chunk - 1;
      unsigned long long tb = 0;
      if (gr == 0) tb = atomicAdd(&ctl->hcnt2[L], (unsigned long long)extra);
      tb = __shfl(tb, Group<G>::base());
      for (int64_t k = gr; k < extra; k += G) {
        if ((int64_t)tb + k < f.hcap) {
          f.h2slot[tb + k] = s;
          f.h2v[tb + k] = u;
          f.h2chunk[tb + k] = (int32_t)(k + 1);
        } else {
          atomicOr(&ctl->flags, kFlagOvfHeavy);
        }
      }
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_bp_c_heavy(DGraph g, int L, int chunk,
                                                       const uint8_t *bd, uint64_t *bs1,
                                                       uint64_t *bs0, DFrontier f) {
  LevelCtl *ctl = f.ctl;
  const unsigned long long ntask = ctl->hcnt2[L];
  if (ntask == 0 || (ctl->flags & kOverflowFlags)) return;
  const int64_t ntasks = (int64_t)ntask < f.hcap ? (int64_t)ntask : f.hcap;
  const int64_t n = g.n;
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t tk = wid; tk < ntasks; tk += nw) {
    const int32_t s = f.h2slot[tk], u = f.h2v[tk], c = f.h2chunk[tk];
    const int64_t e0 = g.row[u], e1 = g.row[u + 1];
    const int64_t a = e0 + (int64_t)c * chunk;
    const int64_t b = a + chunk < e1 ? a + chunk : e1;
    const uint8_t *bds = bd + (int64_t)s * n;
    const uint64_t *b1 = bs1 + (int64_t)s * n;
    const uint64_t *b0 = bs0 + (int64_t)s * n;
    uint64_t a1 = 0, a0 = 0;
    for (int64_t e = a + lane_id(); e < b; e += kWave) {
      const int32_t y = g.col[e];
      if (bds[y] == L) {
        a1 |= b1[y];
        a0 |= b0[y];
      }
    }
    a1 = Group<kWave>::or_reduce(a1);
    a0 = Group<kWave>::or_reduce(a0);
    if (lane_id() == 0) {
      if (a1) atomicOr((unsigned long long *)&bs1[(int64_t)s * n + u], (unsigned long long)a1);
      if (a0) atomicOr((unsigned long long *)&bs0[(int64_t)s * n + u], (unsigned long long)a0);
    }
  }
}

// Roots at distance 0, chosen neighbours at distance 1 with S^{-1} = {self}
// (the initial state of Algorithm 3).  Block i handles slot i.
__global__ void k_bp_init(int32_t n, int32_t nwords, const int32_t *root, const int32_t *nsel,
                          const int32_t *sel, uint8_t *bd, uint64_t *bs1, uint32_t *vis) {
  const int32_t i = blockIdx.x;
  const int32_t r = root[i];
  if (r < 0) return;
  uint8_t *bds = bd + (int64_t)i * n;
  uint32_t *vs = vis + (int64_t)i * nwords;
  const int32_t j = threadIdx.x;
  if (j == 0) {
    bds[r] = 0;
    atomicOr(&vs[r >> 5], 1u << (r & 31));
  }
  if (j < nsel[i]) {
    const int32_t w = sel[i * 64 + j];
    bds[w] = 1;
    bs1[(int64_t)i * n + w] = 1ull << j;
    atomicOr(&vs[w >> 5], 1u << (w & 31));
  }
}

// Slot-major -> vertex-major, with S^0 reduced to its Section 5.1
// definition (disjoint from S^{-1}): the dynamic programme can also collect
// members that are one step closer on another path.
__global__ void k_bp_finish(int32_t n, int32_t t, const uint8_t *bd, const uint64_t *bs1,
                            const uint64_t *bs0, uint8_t *d, uint64_t *m) {
  const int64_t total = (int64_t)n * t;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total;
       x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t v = x / t, s = x - v * t;
    const int64_t src = s * n + v;
    const uint64_t a1 = bs1[src];
    d[x] = bd[src];
    m[2 * x] = a1;
    m[2 * x + 1] = bs0[src] & ~a1;
  }
}

template <int G>
void launch_bp_level_g(DGraph g, int L, int chunk, uint8_t *bd, uint64_t *bs1, uint64_t *bs0,
                       uint32_t *vis, DFrontier f, hipStream_t st, int blocks) {
  hipLaunchKernelGGL(k_bp_a<G>, dim3(blocks), dim3(kBlock), 0, st, g, L, chunk, bd, bs1, bs0,
                     vis, f);
  hipLaunchKernelGGL(k_bp_a_heavy, dim3(blocks), dim3(kBlock), 0, st, g, L, chunk, bd, bs1, bs0,
                     vis, f);
  hipLaunchKernelGGL(k_bp_c<G>, dim3(blocks), dim3(kBlock), 0, st, g, L, chunk, bd, bs1, bs0, f);
  hipLaunchKernelGGL(k_bp_c_heavy, dim3(blocks), dim3(kBlock), 0, st, g, L, chunk, bd, bs1, bs0,
                     f);
}

}  // namespace

hipError_t launch_bp_init(DGraph g, int32_t t, const int32_t *root, const int32_t *nsel,
                          const int32_t *sel, const int32_t * /*sel_pos*/, uint8_t *bd,
                          uint64_t *bs1, uint32_t *vis, DFrontier /*f*/, hipStream_t st) {
  if (t == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bp_init, dim3(t), dim3(64), 0, st, g.n, g.nwords, root, nsel, sel, bd,
                     bs1, vis);
  return hipGetLastError();
}

hipError_t launch_bp_level(DGraph g, int32_t /*t*/, int L, int group, int chunk, uint8_t *bd,
                           uint64_t *bs1, uint64_t *bs0, uint32_t *vis, DFrontier f,
                           hipStream_t st) {
  const int blocks = 2048;
  switch (group) {
    case 4: launch_bp_level_g<4>(g, L, chunk, bd, bs1, bs0, vis, f, st, blocks); break;
    case 8: launch_bp_level_g<8>(g, L, chunk, bd, bs1, bs0, vis, f, st, blocks); break;
    case 16: launch_bp_level_g<16>(g, L, chunk, bd, bs1, bs0, vis, f, st, blocks); break;
    case 32: launch_bp_level_g<32>(g, L, chunk, bd, bs1, bs0, vis, f, st, blocks); break;
    default: launch_bp_level_g<64>(g, L, chunk, bd, bs1, bs0, vis, f, st, blocks); break;
  }
  return hipGetLastError();
}

hipError_t launch_bp_finish(int32_t n, int32_t t, const uint8_t *bd, const uint64_t *bs1,
                            const uint64_t *bs0, uint8_t *d, uint64_t *m, hipStream_t st) {
  const int64_t total = (int64_t)n * t;
  if (total == 0) return hipSuccess;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_bp_finish, dim3((unsigned)blocks), dim3(256), 0, st, n, t, bd, bs1, bs0, d,
                     m);
  return hipGetLastError();
}

}  // namespace pll
