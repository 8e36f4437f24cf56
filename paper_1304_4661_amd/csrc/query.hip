// Distance queries over the finished index.
//
// QUERY(s, t) = min of (a) the bit-parallel estimate of every slot both ends
// reach (Section 5.3) and (b) min over common hubs h of d(h,s) + d(h,t)
// (Section 3.3), clamped to 255.  Labels are sorted by hub rank and end in a
// sentinel (Section 4.5.2), so (b) is a merge join.
//
// Plain form: one thread per pair, the merge walked one entry at a time.
// Batched form: a group of G lanes per pair.  The bit-parallel slots are
// spread over the lanes, and only slots whose lower bound d_s + d_t - 2 can
// beat the best plain root estimate fetch their 16-byte set words.  The merge
// loads G hubs of each label at once and finds the common hubs of the two
// chunks by a per-lane binary search through the other chunk held in lanes
// (cross-lane reads), then advances the chunk(s) that end first.
#include "pll_internal.h"

namespace pll {

namespace {

__global__ void k_validate_pairs(const int32_t *pairs, int64_t q, int32_t n, int32_t *err) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 2 * q;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = pairs[i];
    if (v < 0 || v >= n) atomicOr(err, 1);
  }
}

__global__ void __launch_bounds__(256) k_query_plain(DIndex ix, const int32_t *pairs, int64_t q,
                                                     uint8_t *out, const int32_t *err) {
  if (err && *err) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < q;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t rs = ix.rank[pairs[2 * i]], rt = ix.rank[pairs[2 * i + 1]];
    if (ix.rgid && ix.rgid[rs] != ix.rgid[rt]) {  // different graphs of a batch
      out[i] = kInf8;
      continue;
    }
    int best = kInf8;
    const int32_t t = ix.t;
    for (int32_t k = 0; k < t; k++) {
      const int ds = ix.bpd[(int64_t)rs * ix.tpad + k], dt = ix.bpd[(int64_t)rt * ix.tpad + k];
      if (ds == kInf8 || dt == kInf8) continue;
      const uint64_t *ms = ix.bpm + 2 * ((int64_t)rs * t + k);
      const uint64_t *mt = ix.bpm + 2 * ((int64_t)rt * t + k);
      const int v = bp_pair_dist(ds, ms[0], ms[1], dt, mt[0], mt[1]);
      best = v < best ? v : best;
    }
    int64_t a = ix.off[rs], b = ix.toff[rt];
    for (;;) {
      const uint32_t ha = ix.hub[a], hb = ix.thub[b];
      if (ha == hb) {
        if (ha == kSentinel) break;
        const int v = (int)ix.dist[a] + (int)ix.tdist[b];
        best = v < best ? v : best;
        a++;
        b++;
      } else if (ha < hb) {
        a++;
      } else {
        b++;
      }
    }
    out[i] = (uint8_t)(best < (int)kInf8 ? best : (int)kInf8);
  }
}

// One pair by a group of G lanes (all lanes of the group call it together).
template <int G>
__device__ __forceinline__ void query_pair(const DIndex &ix, const int32_t *pairs, int64_t i,
                                           uint8_t *out) {
  const int gr = Group<G>::rank();
  const int gb = Group<G>::base();
  const int32_t t = ix.t;
  const int32_t rs = ix.rank[pairs[2 * i]], rt = ix.rank[pairs[2 * i + 1]];
  if (ix.rgid && ix.rgid[rs] != ix.rgid[rt]) {  // different graphs of a batch
    if (gr == 0) out[i] = kInf8;
    return;
  }
  // (a) bit-parallel: lane k takes slot k (and k+G, ...).  The root alone
  // gives d_s + d_t; the sets can only take 1 or 2 off it, so a slot's
  // (S^{-1}, S^{0}) pairs are read only if d_s + d_t - 2 beats the best
  // root estimate of the group.
  int ub = kInf8;
  for (int32_t k = gr; k < t; k += G) {
    const int ds = ix.bpd[(int64_t)rs * ix.tpad + k], dt = ix.bpd[(int64_t)rt * ix.tpad + k];
    if (ds != kInf8 && dt != kInf8 && ds + dt < ub) ub = ds + dt;
  }
  ub = Group<G>::min_reduce(ub);
  int best = ub;
  for (int32_t k = gr; k < t; k += G) {
    const int ds = ix.bpd[(int64_t)rs * ix.tpad + k], dt = ix.bpd[(int64_t)rt * ix.tpad + k];
    if (ds != kInf8 && dt != kInf8 && ds + dt - 2 < best) {
      const ulonglong2 ms = reinterpret_cast<const ulonglong2 *>(ix.bpm)[(int64_t)rs * t + k];
      const ulonglong2 mt = reinterpret_cast<const ulonglong2 *>(ix.bpm)[(int64_t)rt * t + k];
      const int v = bp_pair_dist(ds, ms.x, ms.y, dt, mt.x, mt.y);
      best = v < best ? v : best;
    }
  }
  // (b) merge join by chunks of G entries
  int64_t a = ix.off[rs], b = ix.toff[rt];
  const int64_t ea = ix.off[rs + 1], eb = ix.toff[rt + 1];
  for (;;) {
    const uint32_t ha = ix.hub[a + gr < ea ? a + gr : ea - 1];
    const uint32_t hb = ix.thub[b + gr < eb ? b + gr : eb - 1];
    // position of ha among this group's hb values (sorted): halving search
    // for the first index with hb >= ha (or G-1)
    int lo = 0;
#pragma unroll
    for (int s = G / 2; s >= 1; s >>= 1) {
      const uint32_t hm = __shfl(hb, gb + lo + s - 1);
      if (hm < ha) lo += s;
    }
    const uint32_t hf = __shfl(hb, gb + lo);
    if (hf == ha && ha != kSentinel) {
      const int v = (int)ix.dist[a + gr] + (int)ix.tdist[b + lo];
      best = v < best ? v : best;
    }
    const uint32_t lastA = __shfl(ha, gb + G - 1), lastB = __shfl(hb, gb + G - 1);
    if (lastA == kSentinel && lastB == kSentinel) break;
    if (lastA <= lastB) a += G;
    if (lastB <= lastA) b += G;
  }
  best = Group<G>::min_reduce(best);
  if (gr == 0) out[i] = (uint8_t)(best < (int)kInf8 ? best : (int)kInf8);
}

// Batched form: pair i goes to group i mod (groups of the grid).
template <int G>
__global__ void __launch_bounds__(256) k_query_group(DIndex ix, const int32_t *pairs, int64_t q,
                                                     uint8_t *out, const int32_t *err) {
  if (err && *err) return;
  const int64_t gid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  const int64_t ngroups = ((int64_t)gridDim.x * blockDim.x) / G;
  for (int64_t i = gid; i < q; i += ngroups) query_pair<G>(ix, pairs, i, out);
}

// Persistent form: a grid sized to the device; each group takes the next
// chunk of pairs from a shared cursor until none is left, so groups that
// meet short labels take more pairs (pairs differ by up to 100x in label
// length).  *cursor must be 0 at launch (k_zero_u64).
template <int G>
__global__ void __launch_bounds__(256) k_query_persist(DIndex ix, const int32_t *pairs, int64_t q,
                                                       uint8_t *out, const int32_t *err,
                                                       unsigned long long *cursor, int64_t chunk) {
  if (err && *err) return;
  const int gr = Group<G>::rank();
  const int gb = Group<G>::base();
  for (;;) {
    unsigned long long c0 = 0;
    if (gr == 0) c0 = atomicAdd(cursor, (unsigned long long)chunk);
    c0 = __shfl(c0, gb);
    if ((int64_t)c0 >= q) break;
    const int64_t c1 = (int64_t)c0 + chunk < q ? (int64_t)c0 + chunk : q;
    for (int64_t i = (int64_t)c0; i < c1; i++) query_pair<G>(ix, pairs, i, out);
  }
}

__global__ void k_zero_u64(unsigned long long *p) {
  if (threadIdx.x == 0) *p = 0ull;
}

__global__ void k_zero_i32(int32_t *p) {
  if (threadIdx.x == 0) *p = 0;
}

__global__ void k_or_flag(const int32_t *src, int32_t *dst) {
  if (threadIdx.x == 0 && *src) atomicOr(dst, *src);
}

unsigned grid_for(int64_t items, int per_block, int64_t cap) {
  int64_t b = (items + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

}  // namespace

hipError_t launch_validate_pairs(const int32_t *pairs, int64_t q, int32_t n, int32_t *err,
                                 hipStream_t st) {
  if (q <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_validate_pairs, dim3(grid_for(2 * q, 256, 4096)), dim3(256), 0, st, pairs,
                     q, n, err);
  return hipGetLastError();
}

hipError_t launch_or_flag(const int32_t *src, int32_t *dst, hipStream_t st) {
  hipLaunchKernelGGL(k_or_flag, dim3(1), dim3(64), 0, st, src, dst);
  return hipGetLastError();
}

hipError_t launch_query(DIndex ix, const int32_t *pairs, int64_t q, uint8_t *out,
                        const int32_t *err, bool plain, int qgroup, hipStream_t st,
                        unsigned long long *cursor) {
  if (!plain && cursor) return launch_query_persist(ix, pairs, q, out, err, qgroup, cursor, st);
  if (q <= 0) return hipSuccess;
  if (plain) {
    hipLaunchKernelGGL(k_query_plain, dim3(grid_for(q, 256, 65536)), dim3(256), 0, st, ix, pairs,
                       q, out, err);
    return hipGetLastError();
  }
  switch (qgroup) {
    case 16:
      hipLaunchKernelGGL(k_query_group<16>, dim3(grid_for(q * 16, 256, 16384)), dim3(256), 0, st,
                         ix, pairs, q, out, err);
      break;
    case 32:
      hipLaunchKernelGGL(k_query_group<32>, dim3(grid_for(q * 32, 256, 16384)), dim3(256), 0, st,
                         ix, pairs, q, out, err);
      break;
    default:
      hipLaunchKernelGGL(k_query_group<64>, dim3(grid_for(q * 64, 256, 16384)), dim3(256), 0, st,
                         ix, pairs, q, out, err);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_zero_flag(int32_t *flag, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, st, flag);
  return hipGetLastError();
}

hipError_t launch_query_persist(DIndex ix, const int32_t *pairs, int64_t q, uint8_t *out,
                                const int32_t *err, int qgroup, unsigned long long *cursor,
                                hipStream_t st) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, cursor);
  if (q <= 0) return hipGetLastError();
  // 256 CUs x 8 blocks; chunks so that every group takes about 8 of them
  const int blocks = 2048;
  const int64_t groups = (int64_t)blocks * 256 / qgroup;
  int64_t chunk = q / (groups * 8);
  if (chunk < 1) chunk = 1;
  if (chunk > 256) chunk = 256;
  switch (qgroup) {
    case 16:
      hipLaunchKernelGGL(k_query_persist<16>, dim3(blocks), dim3(256), 0, st, ix, pairs, q, out,
                         err, cursor, chunk);
      break;
    case 32:
      hipLaunchKernelGGL(k_query_persist<32>, dim3(blocks), dim3(256), 0, st, ix, pairs, q, out,
                         err, cursor, chunk);
      break;
    default:
      hipLaunchKernelGGL(k_query_persist<64>, dim3(blocks), dim3(256), 0, st, ix, pairs, q, out,
                         err, cursor, chunk);
      break;
  }
  return hipGetLastError();
}

}  // namespace pll
