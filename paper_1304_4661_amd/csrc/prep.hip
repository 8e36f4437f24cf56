// Preparation kernels: ranks, the rank-space CSR, a device-wide exclusive
// scan, and the greedy choice of bit-parallel roots (Section 5.4).
#include "pll_internal.h"

namespace pll {

namespace {

constexpr int kScanThreads = 1024;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

// Inclusive scan across one wave.
__device__ __forceinline__ int64_t wave_incl_scan(int64_t v) {
  int l = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    int64_t w = __shfl_up(v, o);
    if (l >= o) v += w;
  }
  return v;
}

// Exclusive scan across the block; *total receives the block sum.
template <int NT>
__device__ __forceinline__ int64_t block_excl_scan(int64_t v, int64_t *total) {
  __shared__ int64_t s_w[NT / kWave];
  int64_t inc = wave_incl_scan(v);
  int w = threadIdx.x / kWave;
  if (lane_id() == kWave - 1) s_w[w] = inc;
  __syncthreads();
  if (w == 0) {
    int64_t x = lane_id() < NT / kWave ? s_w[lane_id()] : 0;
    int64_t xi = wave_incl_scan(x);
    if (lane_id() < NT / kWave) s_w[lane_id()] = xi - x;
  }
  __syncthreads();
  int64_t pre = s_w[w] + inc - v;
  // block total: exclusive prefix of the last wave + its inclusive sum
  __shared__ int64_t s_tot;
  if (threadIdx.x == NT - 1) s_tot = pre + v;
  __syncthreads();
  *total = s_tot;
  __syncthreads();
  return pre;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(const int64_t *in, int64_t n,
                                                              int64_t *bsum) {
  int64_t base = (int64_t)blockIdx.x * kScanTile;
  int64_t acc = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; k++) {
    int64_t i = base + (int64_t)k * kScanThreads + threadIdx.x;
    if (i < n) acc += in[i];
  }
  int64_t tot;
  block_excl_scan<kScanThreads>(acc, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_spine(int64_t *bsum, int64_t nb) {
  int64_t carry = 0;
  for (int64_t c = 0; c < nb; c += kScanThreads) {
    int64_t i = c + threadIdx.x;
    int64_t v = i < nb ? bsum[i] : 0;
    int64_t tot;
    int64_t pre = block_excl_scan<kScanThreads>(v, &tot);
    if (i < nb) bsum[i] = carry + pre;
    carry += tot;
  }
}

__global__ void __launch_bounds__(kScanThreads) k_scan_apply(const int64_t *in, int64_t *out,
                                                             int64_t n, const int64_t *bsum) {
  int64_t base = (int64_t)blockIdx.x * kScanTile;
  // each thread owns kScanItems consecutive elements
  int64_t v[kScanItems];
  int64_t acc = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; k++) {
    int64_t i = base + (int64_t)threadIdx.x * kScanItems + k;
    v[k] = i < n ? in[i] : 0;
    acc += v[k];
  }
  int64_t tot;
  int64_t pre = block_excl_scan<kScanThreads>(acc, &tot) + bsum[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; k++) {
    int64_t i = base + (int64_t)threadIdx.x * kScanItems + k;
    if (i < n) out[i] = pre;
    if (i == n - 1) out[n] = pre + v[k];
    pre += v[k];
  }
}

// Whole scan in one block for short inputs (a few tiles, walked in order
// with a running carry): one launch instead of three.
constexpr int64_t kScanSmallTiles = 4;

__global__ void __launch_bounds__(kScanThreads) k_scan_small(const int64_t *in, int64_t *out,
                                                             int64_t n) {
  int64_t carry = 0;
  for (int64_t base = 0; base < n; base += kScanTile) {
    int64_t v[kScanItems];
    int64_t acc = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
      const int64_t i = base + (int64_t)threadIdx.x * kScanItems + k;
      v[k] = i < n ? in[i] : 0;
      acc += v[k];
    }
    int64_t tot;
    int64_t pre = block_excl_scan<kScanThreads>(acc, &tot) + carry;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
      const int64_t i = base + (int64_t)threadIdx.x * kScanItems + k;
      if (i < n) out[i] = pre;
      if (i == n - 1) out[n] = pre + v[k];
      pre += v[k];
    }
    carry += tot;
  }
}

// Device-side argument checks for inputs given as device pointers: CSR
// offsets non-decreasing from 0, neighbours inside the vertex's own graph
// and not the vertex itself, and each graph's order a permutation of its
// local ids.  Any violation sets *err.  One wave per vertex.
__global__ void k_validate_graph(int32_t n, const int32_t *row, const int32_t *col,
                                 const int32_t *order, const int32_t *gid,
                                 const int64_t *vtx_off, uint32_t *seen, int32_t *err) {
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t v = wid; v < n; v += nw) {
    const int32_t a = row[v], b = row[v + 1];
    if ((v == 0 && a != 0) || b < a) {
      if (lane_id() == 0) atomicOr(err, 1);
      continue;
    }
    const int32_t g = gid[v];
    const int64_t lo = vtx_off[g], hi = vtx_off[g + 1];
    bool bad = false;
    for (int32_t j = a + lane_id(); j < b; j += kWave) {
      const int32_t w = col[j];
      bad |= w < lo || w >= hi || w == (int32_t)v;
    }
    if (bad) atomicOr(err, 1);
    if (lane_id() == 0) {
      const int32_t o = order[v];
      if (o < 0 || o >= hi - lo) {
        atomicOr(err, 1);
      } else {
        const int64_t x = lo + o;
        if (atomicOr(&seen[x >> 5], 1u << (x & 31)) & (1u << (x & 31))) atomicOr(err, 1);
      }
    }
  }
}

// Graph id of every vertex: block g fills its graph's range.
__global__ void k_fill_gid(const int64_t *vtx_off, int32_t *gid) {
  const int32_t g = blockIdx.x;
  for (int64_t v = vtx_off[g] + threadIdx.x; v < vtx_off[g + 1]; v += blockDim.x) gid[v] = g;
}

// Global rank of graph g's vertex of local rank l: gblk[g] + l for a graph
// given a block of consecutive ranks (gblk[g] >= 0), else lbase[l] + gpos[g]
// (graphs interleaved by local rank; see the batch notes in api.hip).
__device__ __forceinline__ int32_t batch_grank(const int64_t *lbase, const int32_t *gpos,
                                               const int64_t *gblk, int32_t g, int64_t l) {
  const int64_t b = gblk[g];
  return (int32_t)(b >= 0 ? b + l : lbase[l] + gpos[g]);
}

// Ranks of a batch of independent graphs (batch_grank), the inverse order,
// the local rank of every global rank and the graph of every global rank.
__global__ void k_batch_rank(int32_t N, const int32_t *gid, const int64_t *vtx_off,
                             const int32_t *order, const int64_t *lbase, const int32_t *gpos,
                             const int64_t *gblk, int32_t *rank, int32_t *gorder,
                             int32_t *lrank, int32_t *rgid) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < N;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t g = gid[p];
    const int64_t l = p - vtx_off[g];
    const int32_t v = (int32_t)(vtx_off[g] + order[p]);
    const int32_t r = batch_grank(lbase, gpos, gblk, g, l);
    rank[v] = r;
    gorder[r] = v;
    lrank[r] = (int32_t)l;
    rgid[r] = g;
  }
}

__global__ void k_iota_rank(const int32_t *order, int32_t *rank, int32_t n) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) rank[order[i]] = i;
}

__global__ void k_degrees(const int32_t *in_row, const int32_t *order, int64_t *deg, int32_t n) {
  int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) {
    int32_t v = order[r];
    deg[r] = (int64_t)in_row[v + 1] - in_row[v];
  }
}

// One wave per rank-space row: copy the row of vertex order[r], mapping
// neighbour ids to ranks.
__global__ void __launch_bounds__(256) k_relabel_cols(const int32_t *in_row,
                                                      const int32_t *in_col,
                                                      const int32_t *order,
                                                      const int32_t *rank, const int64_t *row,
                                                      int32_t *col, int32_t n) {
  int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t r = wave; r < n; r += nwaves) {
    int32_t v = order[r];
    int64_t a = in_row[v], b = in_row[v + 1], o = row[r];
    for (int64_t e = a + lane_id(); e < b; e += kWave) col[o + (e - a)] = rank[in_col[e]];
  }
}

// ---------------------------------------------------------------------------
// Greedy bit-parallel root choice (Section 5.4): for each slot, the root is
// the lowest-rank vertex not used yet, and S_r its (up to) 64 lowest-rank
// unused neighbours, in ascending rank (bit j = j-th of them).  One block;
// the slots are inherently sequential.

constexpr int kSelThreads = 1024;

__device__ int32_t block_min_i32(int32_t v) {
  __shared__ int32_t s[kSelThreads / kWave];
  for (int o = kWave / 2; o > 0; o >>= 1) {
    int32_t w = __shfl_xor(v, o);
    v = w < v ? w : v;
  }
  __syncthreads();
  if (lane_id() == 0) s[threadIdx.x / kWave] = v;
  __syncthreads();
  int32_t r = s[0];
  for (int i = 1; i < kSelThreads / kWave; i++) r = s[i] < r ? s[i] : r;
  __syncthreads();
  return r;
}

__device__ int32_t block_max_i32(int32_t v) { return -block_min_i32(-v); }

__global__ void __launch_bounds__(kSelThreads) k_bp_select(DGraph g, int32_t t,
                                                           const int64_t *vtx_off,
                                                           const int64_t *lbase,
                                                           const int32_t *gpos,
                                                           const int64_t *gblk,
                                                           const int32_t *lrank,
                                                           uint32_t *used_bits,
                                                           uint32_t *tmp_bits,
                                                           uint8_t *used_bytes, int32_t *root,
                                                           int32_t *nsel, int32_t *sel) {
  // block gi handles graph gi; its vertex of local rank l has global rank
  // batch_grank(.., gi, l); temporary bits are kept per local rank at
  // vtx_off[gi] + l (boundary words are shared with the next graph, hence
  // atomics for setting and clearing)
  const int tid = threadIdx.x;
  const int32_t gi = blockIdx.x;
  const int64_t g0 = vtx_off[gi];
  const int32_t ng = (int32_t)(vtx_off[gi + 1] - g0);
  auto grank = [&](int32_t l) { return batch_grank(lbase, gpos, gblk, gi, l); };
  int32_t cursor = 0;  // every local rank below cursor is used
  for (int32_t i = 0; i < t; i++) {
    const int64_t si = (int64_t)gi * t + i;
    // lowest unused local rank >= cursor
    int32_t lr = -1;
    while (cursor < ng) {
      const int32_t l = cursor + tid;
      int32_t cand = INT32_MAX;
      if (l < ng) {
        const int32_t r = grank(l);
        if (!((ld_acquire_agent(&used_bits[r >> 5]) >> (r & 31)) & 1u)) cand = l;
      }
      cand = block_min_i32(cand);
      if (cand != INT32_MAX) {
        lr = cand;
        break;
      }
      const int64_t next = (int64_t)cursor + kSelThreads;
      cursor = next < (int64_t)ng ? (int32_t)next : ng;
    }
    if (lr < 0) {
      if (tid == 0) {
        root[si] = -1;
        nsel[si] = 0;
      }
      continue;
    }
    cursor = lr + 1;
    const int32_t r = grank(lr);
    if (tid == 0) {
      atomicOr(&used_bits[r >> 5], 1u << (r & 31));
      used_bytes[r] = 1;
      root[si] = r;
    }
    __threadfence();
    __syncthreads();
    // unused neighbours of r, by local rank, into tmp_bits
    const int64_t e0 = g.row[r], e1 = g.row[r + 1];
    int32_t lo = INT32_MAX, hi = -1;
    for (int64_t e = e0 + tid; e < e1; e += kSelThreads) {
      const int32_t w = g.col[e];
      if (!((ld_acquire_agent(&used_bits[w >> 5]) >> (w & 31)) & 1u)) {
        const int32_t lw = lrank[w];
        const int64_t x = g0 + lw;
        atomicOr(&tmp_bits[x >> 5], 1u << (x & 31));
        lo = lw < lo ? lw : lo;
        hi = lw > hi ? lw : hi;
      }
    }
    lo = block_min_i32(lo);
    hi = block_max_i32(hi);
    __threadfence();
    __syncthreads();
    // the first 64 set bits in [g0+lo, g0+hi], ascending
    int32_t taken = 0;
    if (hi >= 0) {
      const int64_t xlo = g0 + lo, xhi = g0 + hi;
      for (int64_t wb = xlo >> 5; wb <= (xhi >> 5) && taken < 64; wb += kSelThreads) {
        const int64_t w = wb + tid;
        uint32_t bits = 0;
        if (w <= (xhi >> 5)) {
          bits = ld_acquire_agent(&tmp_bits[w]);
          // keep only this graph's bits inside [xlo, xhi]
          const int64_t b0 = w * 32;
          if (b0 < xlo) bits &= ~0u << (xlo - b0);
          if (b0 + 31 > xhi) bits &= ~0u >> (b0 + 31 - xhi);
        }
        int64_t tot;
        int32_t pos = taken + (int32_t)block_excl_scan<kSelThreads>(__popc(bits), &tot);
        while (bits && pos < 64) {
          const int b = __ffs(bits) - 1;
          bits &= bits - 1;
          sel[si * 64 + pos] = grank((int32_t)(w * 32 + b - g0));
          pos++;
        }
        taken += (int32_t)tot;
      }
    }
    const int32_t ns = taken < 64 ? taken : 64;
    __threadfence();
    __syncthreads();
    for (int32_t k = tid; k < ns; k += kSelThreads) {
      const int32_t v = sel[si * 64 + k];
      atomicOr(&used_bits[v >> 5], 1u << (v & 31));
      used_bytes[v] = 1;
    }
    for (int64_t e = e0 + tid; e < e1; e += kSelThreads) {
      const int64_t x = g0 + lrank[g.col[e]];
      atomicAnd(&tmp_bits[x >> 5], ~(1u << (x & 31)));
    }
    if (tid == 0) nsel[si] = ns;
    __threadfence();
    __syncthreads();
  }
}

// Transpose of the rank-space graph (in-edges of a directed graph): count
// the arcs into each vertex, then place each arc r -> c into c's row.  Row
// order follows the atomics (the searches do not depend on it).
__global__ void __launch_bounds__(256) k_in_count(const int64_t *row, const int32_t *col,
                                                  int32_t n, unsigned long long *cnt) {
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t r = wave; r < n; r += nwaves)
    for (int64_t e = row[r] + lane_id(); e < row[r + 1]; e += kWave)
      atomicAdd(&cnt[col[e]], 1ull);
}

__global__ void __launch_bounds__(256) k_in_fill(const int64_t *row, const int32_t *col, int32_t n,
                                                 const int64_t *irow, unsigned long long *cursor,
                                                 int32_t *icol, const uint32_t *wt,
                                                 uint32_t *iwt) {
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t r = wave; r < n; r += nwaves)
    for (int64_t e = row[r] + lane_id(); e < row[r + 1]; e += kWave) {
      const int32_t c = col[e];
      const int64_t p = irow[c] + (int64_t)atomicAdd(&cursor[c], 1ull);
      icol[p] = (int32_t)r;
      if (wt) iwt[p] = wt[e];  // an arc keeps its weight
    }
}

}  // namespace

int64_t scan_tmp_elems(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

hipError_t launch_exclusive_scan(const int64_t *in, int64_t *out, int64_t n, int64_t *tmp,
                                 hipStream_t st) {
  if (n <= 0) {
    return hipMemsetAsync(out, 0, sizeof(int64_t), st);
  }
  int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb <= kScanSmallTiles) {
    hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(kScanThreads), 0, st, in, out, n);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, st, in, n, tmp);
  hipLaunchKernelGGL(k_scan_spine, dim3(1), dim3(kScanThreads), 0, st, tmp, nb);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kScanThreads), 0, st, in, out, n,
                     tmp);
  return hipGetLastError();
}

hipError_t launch_validate_graph(int32_t n, const int32_t *row, const int32_t *col,
                                 const int32_t *order, const int32_t *gid,
                                 const int64_t *vtx_off, uint32_t *seen, int32_t *err,
                                 hipStream_t st) {
  if (n == 0) return hipSuccess;
  int64_t blocks = ((int64_t)n * kWave + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_validate_graph, dim3((unsigned)blocks), dim3(256), 0, st, n, row, col,
                     order, gid, vtx_off, seen, err);
  return hipGetLastError();
}

hipError_t launch_fill_gid(const int64_t *vtx_off, int32_t G, int32_t *gid, hipStream_t st) {
  if (G == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_gid, dim3(G), dim3(256), 0, st, vtx_off, gid);
  return hipGetLastError();
}

hipError_t launch_batch_rank(int32_t N, const int32_t *gid, const int64_t *vtx_off,
                             const int32_t *order, const int64_t *lbase, const int32_t *gpos,
                             const int64_t *gblk, int32_t *rank, int32_t *gorder,
                             int32_t *lrank, int32_t *rgid, hipStream_t st) {
  if (N == 0) return hipSuccess;
  int64_t blocks = ((int64_t)N + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_batch_rank, dim3((unsigned)blocks), dim3(256), 0, st, N, gid, vtx_off,
                     order, lbase, gpos, gblk, rank, gorder, lrank, rgid);
  return hipGetLastError();
}

hipError_t launch_iota_rank(const int32_t *order, int32_t *rank, int32_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_iota_rank, dim3((n + 255) / 256), dim3(256), 0, st, order, rank, n);
  return hipGetLastError();
}

hipError_t launch_degrees(const int32_t *in_row, const int32_t *order, int64_t *deg, int32_t n,
                          hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_degrees, dim3((n + 255) / 256), dim3(256), 0, st, in_row, order, deg, n);
  return hipGetLastError();
}

hipError_t launch_transpose(const int64_t *row, const int32_t *col, int32_t n, int64_t *irow,
                            int32_t *icol, int64_t *work, int64_t *tmp, hipStream_t st,
                            const uint32_t *wt, uint32_t *iwt) {
  hipError_t e = hipMemsetAsync(work, 0, ((size_t)n + 1) * sizeof(int64_t), st);
  if (e != hipSuccess) return e;
  if (n == 0) return hipMemsetAsync(irow, 0, sizeof(int64_t), st);
  int64_t blocks = ((int64_t)n * kWave + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  unsigned long long *cnt = reinterpret_cast<unsigned long long *>(work);
  hipLaunchKernelGGL(k_in_count, dim3((unsigned)blocks), dim3(256), 0, st, row, col, n, cnt);
  e = launch_exclusive_scan(work, irow, (int64_t)n, tmp, st);  // irow[n] = total
  if (e != hipSuccess) return e;
  e = hipMemsetAsync(work, 0, ((size_t)n + 1) * sizeof(int64_t), st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_in_fill, dim3((unsigned)blocks), dim3(256), 0, st, row, col, n, irow, cnt,
                     icol, wt, iwt);
  return hipGetLastError();
}

hipError_t launch_relabel_cols(const int32_t *in_row, const int32_t *in_col, const int32_t *order,
                               const int32_t *rank, const int64_t *row, int32_t *col, int32_t n,
                               hipStream_t st) {
  if (n == 0) return hipSuccess;
  int64_t blocks = ((int64_t)n * kWave + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_relabel_cols, dim3((unsigned)blocks), dim3(256), 0, st, in_row, in_col,
                     order, rank, row, col, n);
  return hipGetLastError();
}

hipError_t launch_bp_select(DGraph g, int32_t G, int32_t t, const int64_t *vtx_off,
                            const int64_t *lbase, const int32_t *gpos, const int64_t *gblk,
                            const int32_t *lrank, uint32_t *used_bits, uint32_t *tmp_bits,
                            uint8_t *used_bytes, int32_t *root, int32_t *nsel, int32_t *sel,
                            hipStream_t st) {
  if (t == 0 || G == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bp_select, dim3(G), dim3(kSelThreads), 0, st, g, t, vtx_off, lbase, gpos,
                     gblk, lrank, used_bits, tmp_bits, used_bytes, root, nsel, sel);
  return hipGetLastError();
}

}  // namespace pll
