// Bit-parallel BFS (Algorithm 3, Section 5.2) for all slots at once.
//
// Each slot s has a root r and up to 64 neighbours S_r.  Per slot and vertex
// v the BFS computes d(r, v), S^{-1}(v) = members of S_r one step closer to
// v than r, and S^{0}(v) = members as far from v as r (Section 5.1).  Once
// the roots are chosen the slots are independent, so they advance together,
// one level at a time, in the vertex-major layout the index keeps:
//   d[v*tpad + s] (uint8, rows padded to 16 bytes with 255),
//   m[2*(v*t + s)] = S^{-1}, m[2*(v*t + s) + 1] = S^{0}.
// A wave handles one chunk of one vertex's adjacency list with lane s = slot
// s, so every neighbour costs one 64-byte row read for all slots together
// and no frontier, claim or atomic is needed for the distances.
//
// Level L, in the order the dynamic programme of Section 5.2 needs:
//   E0(L): for v at level L, S^0(v) |= S^{-1}(y) over neighbours y at
//          level L (same-level edges);
//   E1(L): for v not reached yet, if some neighbour y is at level L then v is
//          at level L+1 with S^{-1}(v) = OR S^{-1}(y) and S^0(v) = OR S^0(y)
//          over those y (next-level edges; S^0 of level L is final after E0);
//   commit(L): E1 only records "found" bits, so that every chunk of a long
//          list sees the same snapshot of d; commit writes d = L+1.
// Chunks of one vertex merge with atomic ORs; single-chunk vertices write
// plainly (one writer).  Finally S^0 is reduced to its Section 5.1
// definition (disjoint from S^{-1}); see k_bpv_finish.
#include "pll_internal.h"

namespace pll {

namespace {

constexpr int kBlock = 256;
constexpr int kUnroll = 8;  // neighbours whose rows a wave reads per round

__global__ void k_bpv_count_items(DGraph g, int chunk, int64_t *cnt) {
  const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < g.n) {
    const int64_t deg = g.row[v + 1] - g.row[v];
    cnt[v] = deg <= chunk ? 1 : (deg + chunk - 1) / chunk;
  }
}

__global__ void k_bpv_fill_items(DGraph g, const int64_t *ioff, int32_t *it_v, int32_t *it_c) {
  const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < g.n) {
    const int64_t a = ioff[v], b = ioff[v + 1];
    for (int64_t i = a; i < b; i++) {
      it_v[i] = v;
      it_c[i] = (int32_t)(i - a);
    }
  }
}

// Roots at distance 0, chosen neighbours at distance 1 with S^{-1} = {self}
// (the initial state of Algorithm 3).  Block x handles slot record x
// (graph x / t, slot x % t): the graphs of a batch are disjoint, so one slot
// is a BFS from every graph's root at once, each vertex reached only from
// its own graph's root.
__global__ void k_bpv_init(int32_t t, DBpW b, const int32_t *root, const int32_t *nsel,
                           const int32_t *sel) {
  const int32_t x = blockIdx.x;
  const int32_t s = x % t;
  const int32_t r = root[x];
  if (r < 0) return;
  const int32_t j = threadIdx.x;
  if (j == 0) b.d[(int64_t)r * b.tpad + s] = 0;
  if (j < nsel[x]) {
    const int32_t w = sel[(int64_t)x * 64 + j];
    b.d[(int64_t)w * b.tpad + s] = 1;
    b.m[2 * ((int64_t)w * b.t + s)] = 1ull << j;
  }
}

__global__ void __launch_bounds__(kBlock) k_bpv_e0(DGraph g, DBpW b, const int32_t *it_v,
                                                   const int32_t *it_c, int64_t nitems, int chunk,
                                                   int L) {
  const int s = lane_id();
  const bool lane_ok = s < b.t;
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t i = wid; i < nitems; i += nw) {
    const int32_t v = it_v[i], c = it_c[i];
    const int du = lane_ok ? b.d[(int64_t)v * b.tpad + s] : kInf8;
    const bool act = du == L;
    if (!__ballot(act)) continue;
    const int64_t rb = g.row[v], re = g.row[v + 1];
    const int64_t e0 = rb + (int64_t)c * chunk;
    const int64_t e1 = e0 + chunk < re ? e0 + chunk : re;
    uint64_t acc = 0;
    // kUnroll neighbours per round, so their row reads are in flight together
    for (int64_t e = e0; e < e1; e += kUnroll) {
      int32_t y[kUnroll];
      int dy[kUnroll];
#pragma unroll
      for (int q = 0; q < kUnroll; q++) y[q] = e + q < e1 ? g.col[e + q] : -1;
#pragma unroll
      for (int q = 0; q < kUnroll; q++)
        dy[q] = (lane_ok && y[q] >= 0) ? b.d[(int64_t)y[q] * b.tpad + s] : kInf8;
#pragma unroll
      for (int q = 0; q < kUnroll; q++)
        if (act && dy[q] == L) acc |= b.m[2 * ((int64_t)y[q] * b.t + s)];
    }
    if (act && acc) {
      uint64_t *dst = &b.m[2 * ((int64_t)v * b.t + s) + 1];
      if (re - rb <= chunk)
        *dst |= acc;
      else
        atomicOr((unsigned long long *)dst, (unsigned long long)acc);
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_bpv_e1(DGraph g, DBpW b, const int32_t *it_v,
                                                   const int32_t *it_c, int64_t nitems, int chunk,
                                                   int L) {
  const int s = lane_id();
  const bool lane_ok = s < b.t;
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t i = wid; i < nitems; i += nw) {
    const int32_t v = it_v[i], c = it_c[i];
    const int du = lane_ok ? b.d[(int64_t)v * b.tpad + s] : 0;
    const bool act = lane_ok && du == kInf8;
    if (!__ballot(act)) continue;
    const int64_t rb = g.row[v], re = g.row[v + 1];
    const int64_t e0 = rb + (int64_t)c * chunk;
    const int64_t e1 = e0 + chunk < re ? e0 + chunk : re;
    bool found = false;
    uint64_t a1 = 0, a0 = 0;
    for (int64_t e = e0; e < e1; e += kUnroll) {
      int32_t y[kUnroll];
      int dy[kUnroll];
#pragma unroll
      for (int q = 0; q < kUnroll; q++) y[q] = e + q < e1 ? g.col[e + q] : -1;
#pragma unroll
      for (int q = 0; q < kUnroll; q++)
        dy[q] = (lane_ok && y[q] >= 0) ? b.d[(int64_t)y[q] * b.tpad + s] : kInf8;
#pragma unroll
      for (int q = 0; q < kUnroll; q++) {
        if (act && dy[q] == L) {
          found = true;
          const ulonglong2 my = reinterpret_cast<const ulonglong2 *>(b.m)[(int64_t)y[q] * b.t + s];
          a1 |= my.x;
          a0 |= my.y;
        }
      }
    }
    const uint64_t fm = __ballot(found);
    if (!fm) continue;
    uint64_t *d1 = &b.m[2 * ((int64_t)v * b.t + s)];
    uint64_t *d0 = d1 + 1;
    if (re - rb <= chunk) {
      if (found) {
        *d1 = a1;  // unreached so far: both sets were empty
        *d0 = a0;
      }
      if (s == 0) b.found[v] = fm;
    } else {
      if (found) {
        if (a1) atomicOr((unsigned long long *)d1, (unsigned long long)a1);
        if (a0) atomicOr((unsigned long long *)d0, (unsigned long long)a0);
      }
      if (s == 0) atomicOr((unsigned long long *)&b.found[v], (unsigned long long)fm);
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_bpv_commit(int32_t n, DBpW b, int L,
                                                       unsigned long long *cnt, int32_t *flags) {
  unsigned long long mine = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    uint64_t f = b.found[v];
    if (!f) continue;
    b.found[v] = 0;
    mine += __popcll(f);
    if (L + 1 >= (int)kInf8) {
      atomicOr(flags, kFlagRange);
      continue;
    }
    while (f) {
      const int s = __ffsll((unsigned long long)f) - 1;
      f &= f - 1;
      b.d[v * b.tpad + s] = (uint8_t)(L + 1);
    }
  }
  mine = Group<kWave>::sum_reduce(mine);
  if (lane_id() == 0 && mine) atomicAdd(cnt, mine);
}

// S^0 as Section 5.1 defines it: the dynamic programme can also collect
// members that reach the vertex one step earlier on another path.
__global__ void k_bpv_finish(int64_t total, uint64_t *m) {
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total;
       x += (int64_t)gridDim.x * blockDim.x)
    m[2 * x + 1] &= ~m[2 * x];
}

// Per vertex, the slots whose S^{-1} is non-empty (bit i = slot i): a set
// check that needs S^{-1} of a vertex where it is empty cannot succeed.
__global__ void k_bpv_nonempty(int32_t n, int32_t t, const uint64_t *m, uint64_t *z) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    uint64_t b = 0;
    for (int32_t i = 0; i < t; i++)
      if (m[2 * (v * t + i)] != 0) b |= 1ull << i;
    z[v] = b;
  }
}

// 4-bit copy of the distance rows (DBp::q): one thread per packed 16 bytes
// of a vertex; byte k of packed uint4 qi takes slot 16 qi + k (low nibble)
// and slot tpad/2 + 16 qi + k (high nibble), each saturated at 15.
__global__ void k_bp_pack(const uint8_t *d, int32_t n, int32_t tpad, uint4 *q) {
  const int32_t per = tpad / 32;  // packed uint4 per vertex
  const int32_t half = tpad / 32;  // uint4 of the low half of a row
  const int64_t total = (int64_t)n * per;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t v = i / per;
    const int32_t qi = (int32_t)(i % per);
    const uint4 *row = reinterpret_cast<const uint4 *>(d + v * tpad);
    const uint4 lo = row[qi], hi = row[qi + half];
    const uint32_t lw[4] = {lo.x, lo.y, lo.z, lo.w}, hw[4] = {hi.x, hi.y, hi.z, hi.w};
    uint32_t o[4];
    for (int w = 0; w < 4; w++) {
      uint32_t r = 0;
      for (int b = 0; b < 4; b++) {
        uint32_t a = (lw[w] >> (8 * b)) & 0xFFu, c = (hw[w] >> (8 * b)) & 0xFFu;
        a = a < 15u ? a : 15u;
        c = c < 15u ? c : 15u;
        r |= (a | (c << 4)) << (8 * b);
      }
      o[w] = r;
    }
    q[i] = make_uint4(o[0], o[1], o[2], o[3]);
  }
}

unsigned grid_for(int64_t items, int per_block, int64_t cap) {
  int64_t bl = (items + per_block - 1) / per_block;
  if (bl < 1) bl = 1;
  if (bl > cap) bl = cap;
  return (unsigned)bl;
}

}  // namespace

hipError_t launch_bpv_items_count(DGraph g, int chunk, int64_t *cnt, int64_t *ioff, int64_t *tmp,
                                  hipStream_t st) {
  if (g.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bpv_count_items, dim3((g.n + 255) / 256), dim3(256), 0, st, g, chunk, cnt);
  return launch_exclusive_scan(cnt, ioff, g.n, tmp, st);
}

hipError_t launch_bpv_items_fill(DGraph g, const int64_t *ioff, int32_t *it_v, int32_t *it_c,
                                 hipStream_t st) {
  if (g.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bpv_fill_items, dim3((g.n + 255) / 256), dim3(256), 0, st, g, ioff, it_v,
                     it_c);
  return hipGetLastError();
}

hipError_t launch_bpv_init(int32_t nrec, int32_t t, DBpW b, const int32_t *root,
                           const int32_t *nsel, const int32_t *sel, hipStream_t st) {
  if (t == 0 || nrec == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bpv_init, dim3(nrec), dim3(64), 0, st, t, b, root, nsel, sel);
  return hipGetLastError();
}

hipError_t launch_bpv_level(DGraph g, DBpW b, const int32_t *it_v, const int32_t *it_c,
                            int64_t nitems, int chunk, int L, unsigned long long *cnt,
                            int32_t *flags, hipStream_t st) {
  const unsigned blocks = grid_for(nitems * kWave, kBlock, 8192);
  hipLaunchKernelGGL(k_bpv_e0, dim3(blocks), dim3(kBlock), 0, st, g, b, it_v, it_c, nitems, chunk,
                     L);
  hipLaunchKernelGGL(k_bpv_e1, dim3(blocks), dim3(kBlock), 0, st, g, b, it_v, it_c, nitems, chunk,
                     L);
  hipLaunchKernelGGL(k_bpv_commit, dim3(grid_for(g.n, kBlock, 4096)), dim3(kBlock), 0, st, g.n, b,
                     L, cnt, flags);
  return hipGetLastError();
}

hipError_t launch_bpv_nonempty(int32_t n, int32_t t, const uint64_t *m, uint64_t *z,
                               hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bpv_nonempty, dim3(grid_for(n, 256, 8192)), dim3(256), 0, st, n, t, m, z);
  return hipGetLastError();
}

hipError_t launch_bp_pack(const uint8_t *d, int32_t n, int32_t tpad, uint4 *q, hipStream_t st) {
  if (n == 0 || tpad == 0) return hipSuccess;
  if (tpad % 32) return hipErrorInvalidValue;
  const int64_t total = (int64_t)n * (tpad / 32);
  hipLaunchKernelGGL(k_bp_pack, dim3(grid_for(total, 256, 8192)), dim3(256), 0, st, d, n, tpad, q);
  return hipGetLastError();
}

hipError_t launch_bpv_finish(int64_t total, uint64_t *m, hipStream_t st) {
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bpv_finish, dim3(grid_for(total, 256, 8192)), dim3(256), 0, st, total, m);
  return hipGetLastError();
}

}  // namespace pll
