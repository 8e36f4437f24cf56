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

// Device-side argument checks for inputs given as device pointers: CSR
// offsets non-decreasing from 0, neighbours in range and not the vertex
// itself, order a permutation.  Any violation sets *err.
__global__ void k_validate_graph(int32_t n, const int32_t *row, const int32_t *col,
                                 const int32_t *order, uint32_t *seen, int32_t *err) {
  // one wave per vertex: offsets and the order entry by lane 0, the row's
  // neighbours by all lanes
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t v = wid; v < n; v += nw) {
    const int32_t a = row[v], b = row[v + 1];
    if ((v == 0 && a != 0) || b < a) {
      if (lane_id() == 0) atomicOr(err, 1);
      continue;
    }
    bool bad = false;
    for (int32_t j = a + lane_id(); j < b; j += kWave) {
      const int32_t w = col[j];
      bad |= w < 0 || w >= n || w == (int32_t)v;
    }
    if (bad) atomicOr(err, 1);
    if (lane_id() == 0) {
      const int32_t o = order[v];
      if (o < 0 || o >= n) {
        atomicOr(err, 1);
      } else if (atomicOr(&seen[o >> 5], 1u << (o & 31)) & (1u << (o & 31))) {
        atomicOr(err, 1);
      }
    }
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
                                                           uint32_t *used_bits,
                                                           uint32_t *tmp_bits,
                                                           uint8_t *used_bytes, int32_t *root,
                                                           int32_t *nsel, int32_t *sel) {
  const int tid = threadIdx.x;
  const int32_t n = g.n, nwords = g.nwords;
  int32_t cursor = 0;  // every rank below cursor is used
  for (int32_t i = 0; i < t; i++) {
    // lowest unused rank >= cursor
    int32_t r = -1;
    while (cursor < n) {
      int32_t w0 = cursor >> 5;
      int32_t w = w0 + tid;
      int32_t cand = INT32_MAX;
      if (w < nwords) {
        uint32_t free_bits = ~ld_acquire_agent(&used_bits[w]);
        if (w == w0) free_bits &= ~((1u << (cursor & 31)) - 1u);
        if (w == nwords - 1 && (n & 31)) free_bits &= (1u << (n & 31)) - 1u;
        if (free_bits) cand = w * 32 + __ffs(free_bits) - 1;
      }
      cand = block_min_i32(cand);
      if (cand != INT32_MAX) {
        r = cand;
        break;
      }
      int64_t next = ((int64_t)w0 + kSelThreads) * 32;
      cursor = next < (int64_t)n ? (int32_t)next : n;
    }
    if (r < 0) {
      if (tid == 0) {
        root[i] = -1;
        nsel[i] = 0;
      }
      continue;
    }
    cursor = r + 1;
    if (tid == 0) {
      atomicOr(&used_bits[r >> 5], 1u << (r & 31));
      used_bytes[r] = 1;
      root[i] = r;
    }
    __threadfence();
    __syncthreads();
    // unused neighbours of r into tmp_bits
    const int64_t e0 = g.row[r], e1 = g.row[r + 1];
    int32_t lo = INT32_MAX, hi = -1;
    for (int64_t e = e0 + tid; e < e1; e += kSelThreads) {
      int32_t w = g.col[e];
      if (!((ld_acquire_agent(&used_bits[w >> 5]) >> (w & 31)) & 1u)) {
        atomicOr(&tmp_bits[w >> 5], 1u << (w & 31));
        lo = w < lo ? w : lo;
        hi = w > hi ? w : hi;
      }
    }
    lo = block_min_i32(lo);
    hi = block_max_i32(hi);
    __threadfence();
    __syncthreads();
    // the first 64 set bits of tmp_bits, ascending
    int32_t taken = 0;
    if (hi >= 0) {
      for (int32_t wb = lo >> 5; wb <= (hi >> 5) && taken < 64; wb += kSelThreads) {
        int32_t w = wb + tid;
        uint32_t bits = w <= (hi >> 5) ? ld_acquire_agent(&tmp_bits[w]) : 0u;
        int64_t tot;
        int32_t pos = taken + (int32_t)block_excl_scan<kSelThreads>(__popc(bits), &tot);
        while (bits && pos < 64) {
          int b = __ffs(bits) - 1;
          bits &= bits - 1;
          sel[i * 64 + pos] = w * 32 + b;
          pos++;
        }
        taken += (int32_t)tot;
      }
    }
    int32_t ns = taken < 64 ? taken : 64;
    __threadfence();
    __syncthreads();
    for (int32_t k = tid; k < ns; k += kSelThreads) {
      int32_t v = sel[i * 64 + k];
      atomicOr(&used_bits[v >> 5], 1u << (v & 31));
      used_bytes[v] = 1;
    }
    for (int64_t e = e0 + tid; e < e1; e += kSelThreads) {
      int32_t w = g.col[e];
      st_relaxed_agent(&tmp_bits[w >> 5], 0u);
    }
    if (tid == 0) nsel[i] = ns;
    __threadfence();
    __syncthreads();
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
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, st, in, n, tmp);
  hipLaunchKernelGGL(k_scan_spine, dim3(1), dim3(kScanThreads), 0, st, tmp, nb);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kScanThreads), 0, st, in, out, n,
                     tmp);
  return hipGetLastError();
}

hipError_t launch_validate_graph(int32_t n, const int32_t *row, const int32_t *col,
                                 const int32_t *order, uint32_t *seen, int32_t *err,
                                 hipStream_t st) {
  if (n == 0) return hipSuccess;
  int64_t blocks = ((int64_t)n * kWave + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_validate_graph, dim3((unsigned)blocks), dim3(256), 0, st, n, row, col,
                     order, seen, err);
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

hipError_t launch_bp_select(DGraph g, int32_t t, uint32_t *used_bits, uint32_t *tmp_bits,
                            uint8_t *used_bytes, int32_t *root, int32_t *nsel, int32_t *sel,
                            hipStream_t st) {
  if (t == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bp_select, dim3(1), dim3(kSelThreads), 0, st, g, t, used_bits, tmp_bits,
                     used_bytes, root, nsel, sel);
  return hipGetLastError();
}

}  // namespace pll
