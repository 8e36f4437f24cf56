// Gathers one graph of an index into contiguous, canonical arrays for
// pll_export: rows in the graph's local rank order, hubs as local ranks,
// sentinels dropped, bit-parallel rows without padding.
#include "pll_internal.h"

namespace pll {

namespace {

// one wave per output row
__global__ void k_gather_labels(const int64_t *rows, int64_t m, const int64_t *src_off,
                                const uint32_t *hub, const uint8_t *dist, const int32_t *lrank,
                                const int64_t *out_off, uint32_t *out_hub, uint8_t *out_dist) {
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t i = wid; i < m; i += nw) {
    const int64_t r = rows[i];
    const int64_t a = src_off[r], len = src_off[r + 1] - 1 - a;
    const int64_t o = out_off[i];
    for (int64_t x = lane_id(); x < len; x += kWave) {
      out_hub[o + x] = (uint32_t)lrank[hub[a + x]];
      out_dist[o + x] = dist[a + x];
    }
  }
}

__global__ void k_gather_bp(const int64_t *rows, int64_t m, int32_t t, int32_t tpad,
                            const uint8_t *bpd, const uint64_t *bpm, uint8_t *out_d,
                            uint64_t *out_m1, uint64_t *out_m0) {
  const int64_t total = m * t;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total;
       x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = x / t, s = x - i * t;
    const int64_t r = rows[i];
    out_d[x] = bpd[r * tpad + s];
    out_m1[x] = bpm[2 * (r * t + s)];
    out_m0[x] = bpm[2 * (r * t + s) + 1];
  }
}

__global__ void k_gather_rank(int64_t g0, int64_t ng, const int32_t *rank, const int32_t *lrank,
                              int32_t *out) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < ng;
       v += (int64_t)gridDim.x * blockDim.x)
    out[v] = lrank[rank[g0 + v]];
}

unsigned grid_for(int64_t items, int per_block, int64_t cap) {
  int64_t b = (items + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

}  // namespace

hipError_t launch_gather_labels(const int64_t *rows, int64_t m, const int64_t *src_off,
                                const uint32_t *hub, const uint8_t *dist, const int32_t *lrank,
                                const int64_t *out_off, uint32_t *out_hub, uint8_t *out_dist,
                                hipStream_t st) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_labels, dim3(grid_for(m * kWave, 256, 8192)), dim3(256), 0, st, rows,
                     m, src_off, hub, dist, lrank, out_off, out_hub, out_dist);
  return hipGetLastError();
}

hipError_t launch_gather_bp(const int64_t *rows, int64_t m, int32_t t, int32_t tpad,
                            const uint8_t *bpd, const uint64_t *bpm, uint8_t *out_d,
                            uint64_t *out_m1, uint64_t *out_m0, hipStream_t st) {
  if (m <= 0 || t <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_bp, dim3(grid_for(m * t, 256, 8192)), dim3(256), 0, st, rows, m, t,
                     tpad, bpd, bpm, out_d, out_m1, out_m0);
  return hipGetLastError();
}

hipError_t launch_gather_rank(int64_t g0, int64_t ng, const int32_t *rank, const int32_t *lrank,
                              int32_t *out, hipStream_t st) {
  if (ng <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_rank, dim3(grid_for(ng, 256, 8192)), dim3(256), 0, st, g0, ng, rank,
                     lrank, out);
  return hipGetLastError();
}

}  // namespace pll
