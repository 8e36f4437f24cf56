// Distance queries that allocate nothing: pll_query with its per-call device
// memory (the error flag of a device-pointer call, the staging of a
// host-pointer call's pairs and answers) placed in one static device array
// instead of hipMalloc'ed buffers.
#include <mutex>

#include "pll_internal.h"

namespace pll {
DIndex index_view(const pll_index *idx);
int32_t index_n(const pll_index *idx);
bool index_weighted(const pll_index *idx);
int32_t *index_err(const pll_index *idx);
int64_t query_group_size();
bool query_persistent();
}  // namespace pll

namespace {

// Layout of the array: the error flag (offset 0) and the persistent query
// form's work cursor (offset 128) in the first 256 bytes, then staging for
// kNoAllocMaxPairs pairs (int32[2q]) and their answers (uint8[q]).
constexpr int64_t kNoAllocMaxPairs = 1ll << 21;
constexpr int64_t kFlagBytes = 256;
constexpr int64_t kPairsOff = kFlagBytes;
constexpr int64_t kOutOff = kPairsOff + 8 * kNoAllocMaxPairs;
constexpr int64_t kScratchBytes = kOutOff + kNoAllocMaxPairs;

// One copy per GPU, held until the process ends.  In host code `scratch`
// only names the symbol: its device address comes from hipGetSymbolAddress.
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
uint8_t *g_ptr[kMaxDevices] = {};

// Device address of this device's array, looked up once per device (with
// that device current).  nullptr on failure.
uint8_t *scratch_ptr() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_ptr[dev] = (uint8_t *)p;
  }
  return g_ptr[dev];
}

__global__ void k_clear_flag(int32_t *flag) {
  if (threadIdx.x == 0) *flag = 0;
}

}  // namespace

extern "C" int64_t pll_query_noalloc_max_pairs(void) { return kNoAllocMaxPairs; }

extern "C" int pll_query_noalloc(const pll_index *idx, const int32_t *pairs, int64_t q,
                                 uint8_t *out, uint32_t flags, void *stream) {
  using namespace pll;
  if (!idx || q < 0) return PLL_E_INVAL;
  if (index_weighted(idx)) return PLL_E_UNSUPPORTED;
  if (q == 0) return PLL_OK;
  if (!pairs || !out) return PLL_E_INVAL;
  const bool device = (flags & PLL_DEVICE_PTRS) != 0;
  if (!device && q > kNoAllocMaxPairs) return PLL_E_INVAL;
  const int32_t n = index_n(idx);
  if (!device)
    for (int64_t i = 0; i < 2 * q; i++)
      if (pairs[i] < 0 || pairs[i] >= n) return PLL_E_INVAL;
  uint8_t *base = scratch_ptr();
  if (!base) return PLL_E_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  const bool plain = (flags & PLL_PLAIN) != 0;
  const int qgroup = (int)query_group_size();
  unsigned long long *cursor =
      query_persistent() ? reinterpret_cast<unsigned long long *>(base + 128) : nullptr;
  const DIndex view = index_view(idx);
  auto ok = [](hipError_t e) { return e == hipSuccess; };
  if (!device) {
    int32_t *dp = reinterpret_cast<int32_t *>(base + kPairsOff);
    uint8_t *dout = base + kOutOff;
    if (!ok(hipMemcpyAsync(dp, pairs, (size_t)(2 * q) * sizeof(int32_t), hipMemcpyHostToDevice,
                           st)) ||
        !ok(launch_query(view, dp, q, dout, nullptr, plain, qgroup, st, cursor)) ||
        !ok(hipMemcpyAsync(out, dout, (size_t)q, hipMemcpyDeviceToHost, st)) ||
        !ok(hipStreamSynchronize(st)))
      return PLL_E_DEVICE;
    return PLL_OK;
  }
  int32_t *flag = reinterpret_cast<int32_t *>(base);
  hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(64), 0, st, flag);
  if (!ok(hipGetLastError()) || !ok(launch_validate_pairs(pairs, q, n, flag, st)) ||
      !ok(launch_query(view, pairs, q, out, flag, plain, qgroup, st, cursor)))
    return PLL_E_DEVICE;
  if (flags & PLL_SYNC) {
    int32_t herr = 0;
    if (!ok(hipMemcpyAsync(&herr, flag, sizeof(int32_t), hipMemcpyDeviceToHost, st)) ||
        !ok(hipStreamSynchronize(st)))
      return PLL_E_DEVICE;
    return herr ? PLL_E_INVAL : PLL_OK;
  }
  // as pll_query: fold this call's outcome into the index's sticky error
  return ok(launch_or_flag(flag, index_err(idx), st)) ? PLL_OK : PLL_E_DEVICE;
}
