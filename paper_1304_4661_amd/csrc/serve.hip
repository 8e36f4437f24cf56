// Serving over a device-resident index: continuous batching of distance
// queries (Sections 3.3 and 5.3 answered by the library's query kernel; on a
// weighted index, Section 6's, with 32-bit answers).
//
// A worker thread owns `nslots` slots, each a HIP stream with pinned host
// staging and device buffers for up to `slot_pairs` pairs.  Requests queue
// FIFO.  Whenever a slot is free the worker packs the oldest requests that
// fit into it (a batch), copies their pairs in, launches the query kernel
// and the copy back, and records an event; meanwhile other slots' batches
// run, so requests that arrive while earlier ones are on the GPU are
// admitted as soon as a slot (and its memory) frees up, and their work
// overlaps on the device.  Completed batches are scattered back to each
// request's output and stamped.  A request larger than a slot is queued as
// slot-sized parts and stamped when its last part completes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "pll_internal.h"

namespace pll {
// defined in api.hip
DIndex index_view(const pll_index *idx);
int32_t index_n(const pll_index *idx);
bool index_weighted(const pll_index *idx);
int64_t query_group_size();
int64_t serve_coalesce();
}  // namespace pll

using namespace pll;

namespace {

using Clock = std::chrono::steady_clock;
int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now().time_since_epoch())
      .count();
}

// A request, or one slot-sized part of a request larger than a slot (then
// `parent` is the request; it is answered when its last part is).  Records
// are recycled: a request's record is freed once pll_server_done has
// reported it answered, a part's once its answers are copied out; a ticket
// carries the record's index and its generation, so a stale ticket is
// rejected.
struct Req {
  int64_t idx = 0;   // position in the server's records
  uint32_t gen = 0;  // bumped each time the record is freed
  const int32_t *pairs = nullptr;
  void *out = nullptr;  // es bytes per answer (the server's answer size)
  int64_t q = 0;
  int64_t t_arrive = 0;             // ns, steady clock
  std::atomic<int64_t> t_done{0};   // 0 until answered
  Req *parent = nullptr;
  std::atomic<int64_t> parts_left{0};  // parts not yet answered (split requests)
};

struct Slot {
  hipStream_t s = nullptr;
  hipEvent_t ev = nullptr;
  int32_t *hp = nullptr;   // pinned pairs
  uint8_t *ho = nullptr;   // pinned answers (es bytes each)
  int32_t *dp = nullptr;   // device pairs
  uint8_t *dout = nullptr; // device answers (es bytes each)
  std::vector<Req *> reqs;
  int64_t n = 0;
  bool busy = false;
  int64_t t_dispatch = 0;  // ns, when the batch was queued on the stream
  int64_t launch = 0;      // its number among the server's launches
};

}  // namespace

struct pll_server {
  const pll_index *idx = nullptr;
  DIndex view{};
  int32_t n = 0;
  bool weighted = false;  // 32-bit answers of a weighted index
  int es = 1;             // bytes per answer
  int qgroup = 64;
  bool coalesce = true;  // false: one request per launch (the plain form)
  int64_t slot_pairs = 0;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Req> recs;          // request and part records (addresses stay put)
  std::vector<int64_t> free_recs;  // indices of free records
  std::deque<Req *> pending;     // FIFO of submitted, not yet dispatched
  std::atomic<bool> stopping{false};
  std::atomic<int> err{0};
  std::thread worker;
  Req *take() {  // a free record (the caller holds mu)
    if (free_recs.empty()) {
      recs.emplace_back();
      recs.back().idx = (int64_t)recs.size() - 1;
      return &recs.back();
    }
    Req *r = &recs[(size_t)free_recs.back()];
    free_recs.pop_back();
    return r;
  }
  void give_back(Req *r) {  // the caller holds mu
    r->gen++;
    r->pairs = nullptr;
    r->out = nullptr;
    r->parent = nullptr;
    r->t_done.store(0, std::memory_order_relaxed);
    free_recs.push_back(r->idx);
  }
  // statistics; the longest launch is timed from its dispatch to the host
  // seeing its event
  int64_t launches = 0, batched_pairs = 0, max_pending = 0, max_launch_ns = 0,
          max_launch_at = -1, max_gap_ns = 0;

  void run();
  void release();
};

namespace {

bool dispatch(pll_server *sv, Slot &sl) {
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->pending.empty()) return false;
    sl.reqs.clear();
    sl.n = 0;
    while (!sv->pending.empty()) {
      Req *r = sv->pending.front();
      if (!sl.reqs.empty() && (!sv->coalesce || sl.n + r->q > sv->slot_pairs)) break;
      sl.reqs.push_back(r);
      sl.n += r->q;
      sv->pending.pop_front();
    }
  }
  int64_t off = 0;
  for (Req *r : sl.reqs) {
    std::copy(r->pairs, r->pairs + 2 * r->q, sl.hp + 2 * off);
    off += r->q;
  }
  hipError_t e = hipMemcpyAsync(sl.dp, sl.hp, (size_t)sl.n * 2 * sizeof(int32_t),
                                hipMemcpyHostToDevice, sl.s);
  if (e == hipSuccess)
    e = sv->weighted ? launch_wquery(sv->view, sl.dp, sl.n, reinterpret_cast<uint32_t *>(sl.dout),
                                     nullptr, false, sv->qgroup, sl.s)
                     : launch_query(sv->view, sl.dp, sl.n, sl.dout, nullptr, false, sv->qgroup,
                                    sl.s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(sl.ho, sl.dout, (size_t)sl.n * sv->es, hipMemcpyDeviceToHost, sl.s);
  if (e == hipSuccess) e = hipEventRecord(sl.ev, sl.s);
  if (e != hipSuccess) sv->err = PLL_E_DEVICE;
  sl.busy = true;
  sl.t_dispatch = now_ns();
  sl.launch = sv->launches;
  sv->launches++;
  sv->batched_pairs += sl.n;
  return true;
}

bool complete(pll_server *sv, Slot &sl) {
  if (!sl.busy) return false;
  hipError_t e = hipEventQuery(sl.ev);
  if (e == hipErrorNotReady) return false;
  if (e != hipSuccess) sv->err = PLL_E_DEVICE;
  const int64_t t = now_ns();
  if (t - sl.t_dispatch > sv->max_launch_ns) {
    sv->max_launch_ns = t - sl.t_dispatch;
    sv->max_launch_at = sl.launch;
  }
  int64_t off = 0;
  bool parts = false;
  for (Req *r : sl.reqs) {
    std::copy(sl.ho + off * sv->es, sl.ho + (off + r->q) * sv->es, static_cast<uint8_t *>(r->out));
    off += r->q;
    if (!r->parent) {
      r->t_done.store(t, std::memory_order_release);
    } else {
      parts = true;
      if (r->parent->parts_left.fetch_sub(1) == 1)  // its last part
        r->parent->t_done.store(t, std::memory_order_release);
    }
  }
  if (parts) {
    std::lock_guard<std::mutex> lk(sv->mu);
    for (Req *r : sl.reqs)
      if (r->parent) sv->give_back(r);
  }
  sl.reqs.clear();
  sl.busy = false;
  return true;
}

}  // namespace

void pll_server::run() {
  int64_t t_prev = now_ns();
  for (;;) {
    // the longest time between two passes of the worker while it had work
    // (a pause here delays every request in flight)
    const int64_t t_now = now_ns();
    if (t_now - t_prev > max_gap_ns) max_gap_ns = t_now - t_prev;
    t_prev = t_now;
    bool progress = false;
    for (Slot &sl : slots) progress |= complete(this, sl);
    for (Slot &sl : slots)
      if (!sl.busy) progress |= dispatch(this, sl);
    bool any_busy = false;
    for (Slot &sl : slots) any_busy |= sl.busy;
    if (!any_busy) {
      std::unique_lock<std::mutex> lk(mu);
      if (pending.empty()) {
        if (stopping.load()) return;
        cv.wait_for(lk, std::chrono::microseconds(200));
        t_prev = now_ns();  // an idle wait is not a pause
      }
    } else if (!progress) {
      std::this_thread::yield();
    }
  }
}

void pll_server::release() {
  for (Slot &sl : slots) {
    if (sl.s) (void)hipStreamSynchronize(sl.s);
    if (sl.ev) (void)hipEventDestroy(sl.ev);
    if (sl.s) (void)hipStreamDestroy(sl.s);
    if (sl.hp) (void)hipHostFree(sl.hp);
    if (sl.ho) (void)hipHostFree(sl.ho);
    if (sl.dp) (void)hipFree(sl.dp);
    if (sl.dout) (void)hipFree(sl.dout);
  }
  slots.clear();
}

extern "C" {

int pll_server_start(const pll_index *idx, int32_t nslots, int64_t slot_pairs, pll_server **out) {
  if (!out) return PLL_E_INVAL;
  *out = nullptr;
  if (!idx || nslots < 1 || nslots > 32 || slot_pairs < 1 || slot_pairs > (1ll << 30))
    return PLL_E_INVAL;
  pll_server *sv = new (std::nothrow) pll_server();
  if (!sv) return PLL_E_NOMEM;
  sv->idx = idx;
  sv->weighted = index_weighted(idx);
  sv->es = sv->weighted ? 4 : 1;
  sv->view = index_view(idx);
  sv->n = index_n(idx);
  sv->qgroup = (int)query_group_size();
  sv->coalesce = serve_coalesce() != 0;
  sv->slot_pairs = slot_pairs;
  sv->slots.resize((size_t)nslots);
  for (Slot &sl : sv->slots) {
    bool ok = hipStreamCreateWithFlags(&sl.s, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) == hipSuccess &&
              hipHostMalloc((void **)&sl.hp, (size_t)slot_pairs * 2 * sizeof(int32_t),
                            hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc((void **)&sl.ho, (size_t)slot_pairs * sv->es, hipHostMallocDefault) ==
                  hipSuccess &&
              hipMalloc((void **)&sl.dp, (size_t)slot_pairs * 2 * sizeof(int32_t)) ==
                  hipSuccess &&
              hipMalloc((void **)&sl.dout, (size_t)slot_pairs * sv->es) == hipSuccess;
    // One request's worth of work per slot now, over the whole staging
    // buffers, so that neither the runtime's set-up of the stream's queues
    // nor the first touch of the pinned pages (by the host and by the copy
    // engines) lands on a request: a first dispatch on a new stream was
    // measured to stall the worker for up to 9 ms, and the first launch that
    // used a larger part of the staging than any before it for 6.5 ms.
    // The staged pairs are (0, 0), a valid query of any non-empty index.
    if (ok) {
      std::memset(sl.hp, 0, (size_t)slot_pairs * 2 * sizeof(int32_t));
      std::memset(sl.ho, 0, (size_t)slot_pairs * sv->es);
    }
    ok = ok && hipMemcpyAsync(sl.dp, sl.hp, (size_t)slot_pairs * 2 * sizeof(int32_t),
                              hipMemcpyHostToDevice, sl.s) == hipSuccess;
    if (ok && sv->n > 0)
      ok = (sv->weighted ? launch_wquery(sv->view, sl.dp, 1, reinterpret_cast<uint32_t *>(sl.dout),
                                         nullptr, false, sv->qgroup, sl.s)
                         : launch_query(sv->view, sl.dp, 1, sl.dout, nullptr, false, sv->qgroup,
                                        sl.s)) == hipSuccess;
    ok = ok && hipMemcpyAsync(sl.ho, sl.dout, (size_t)slot_pairs * sv->es, hipMemcpyDeviceToHost,
                              sl.s) == hipSuccess &&
         hipEventRecord(sl.ev, sl.s) == hipSuccess && hipStreamSynchronize(sl.s) == hipSuccess;
    if (!ok) {
      (void)hipGetLastError();
      sv->release();
      delete sv;
      return PLL_E_NOMEM;
    }
  }
  try {
    sv->worker = std::thread([sv] { sv->run(); });
  } catch (...) {
    sv->release();
    delete sv;
    return PLL_E_NOMEM;
  }
  *out = sv;
  return PLL_OK;
}

// Internal: submit with an explicit arrival time (ns, steady clock).  A
// request larger than a slot is queued as consecutive slot-sized parts.
static int submit_at(pll_server *sv, const int32_t *pairs, int64_t q, void *out,
                     int64_t t_arrive, int64_t *ticket) {
  if (!sv || q < 1 || !pairs || !out) return PLL_E_INVAL;
  for (int64_t i = 0; i < 2 * q; i++)
    if (pairs[i] < 0 || pairs[i] >= sv->n) return PLL_E_INVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  Req &r = *sv->take();
  r.pairs = pairs;
  r.out = out;
  r.q = q;
  r.t_arrive = t_arrive;
  if (q <= sv->slot_pairs) {
    sv->pending.push_back(&r);
  } else {
    r.parts_left = (q + sv->slot_pairs - 1) / sv->slot_pairs;
    for (int64_t o = 0; o < q; o += sv->slot_pairs) {
      Req &p = *sv->take();
      p.pairs = pairs + 2 * o;
      p.out = static_cast<uint8_t *>(out) + o * sv->es;
      p.q = std::min<int64_t>(sv->slot_pairs, q - o);
      p.t_arrive = t_arrive;
      p.parent = &r;
      sv->pending.push_back(&p);
    }
  }
  sv->max_pending = std::max<int64_t>(sv->max_pending, (int64_t)sv->pending.size());
  if (ticket) *ticket = (int64_t)r.gen << 32 | r.idx;
  sv->cv.notify_one();
  return PLL_OK;
}

int pll_server_submit(pll_server *sv, const int32_t *pairs, int64_t q, uint8_t *out,
                      int64_t *ticket) {
  if (sv && sv->weighted) return PLL_E_UNSUPPORTED;  // 32-bit answers: the call below
  return submit_at(sv, pairs, q, out, now_ns(), ticket);
}

int pll_server_submit_weighted(pll_server *sv, const int32_t *pairs, int64_t q, uint32_t *out,
                               int64_t *ticket) {
  if (sv && !sv->weighted) return PLL_E_UNSUPPORTED;  // 8-bit answers: the call above
  return submit_at(sv, pairs, q, out, now_ns(), ticket);
}

int pll_server_done(pll_server *sv, int64_t ticket, int32_t wait, double *latency_us) {
  if (!sv) return PLL_E_INVAL;
  const int64_t i = ticket & 0xFFFFFFFFll;
  const uint32_t gen = (uint32_t)((uint64_t)ticket >> 32);
  Req *r;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (ticket < 0 || i >= (int64_t)sv->recs.size()) return PLL_E_INVAL;
    r = &sv->recs[(size_t)i];
    if (r->gen != gen || r->parent || !r->out) return PLL_E_INVAL;  // stale or not a request
  }
  int64_t t = r->t_done.load(std::memory_order_acquire);
  while (wait && !t) {
    if (sv->err.load()) return sv->err.load();
    std::this_thread::yield();
    t = r->t_done.load(std::memory_order_acquire);
  }
  if (sv->err.load()) return sv->err.load();
  if (!t) return 0;
  if (latency_us) *latency_us = (double)(t - r->t_arrive) * 1e-3;
  std::lock_guard<std::mutex> lk(sv->mu);
  if (r->gen == gen) sv->give_back(r);  // answered and reported: the record is free
  return 1;
}

int pll_server_stop(pll_server *sv, int64_t *stats, int32_t nstats) {
  if (!sv) return PLL_E_INVAL;
  sv->stopping = true;
  sv->cv.notify_all();
  if (sv->worker.joinable()) sv->worker.join();
  const int rc = sv->err.load();
  const int64_t st[7] = {sv->launches,      sv->batched_pairs, sv->max_pending,
                         sv->max_launch_ns, sv->max_launch_at, sv->max_gap_ns,
                         (int64_t)sv->recs.size()};
  for (int32_t i = 0; stats && i < nstats && i < 7; i++) stats[i] = st[i];
  sv->release();
  delete sv;
  return rc;
}

// Open-loop load test: nreq requests with sizes round(exp(U*ln(max_batch)))
// (log-uniform in [1, max_batch]) and uniform random pairs, arriving as a
// Poisson process of `rate` requests/s (rate <= 0: all at once, which
// measures the saturated throughput).  Randomness: SplitMix64 from `seed`.
// Latency = answer time - scheduled arrival (queueing counts).
// stats: [p50 us, p99 us, mean us, pairs/s, requests/s, seconds, launches,
//         mean pairs per launch, max queued requests, longest launch us,
//         its launch number, the longest pause of the worker us]
int pll_serve_bench(const pll_index *idx, double rate, int64_t nreq, int64_t max_batch,
                    uint64_t seed, int32_t nslots, int64_t slot_pairs, double *stats,
                    int32_t nstats) {
  if (!idx || nreq < 1 || max_batch < 1 || max_batch > slot_pairs) return PLL_E_INVAL;
  const int32_t n = index_n(idx);
  if (n < 1) return PLL_E_INVAL;
  uint64_t x = seed;
  auto next = [&x]() {
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  auto unif = [&]() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); };
  std::vector<int64_t> size((size_t)nreq), off((size_t)nreq + 1, 0);
  std::vector<double> at((size_t)nreq, 0.0);
  double t = 0.0;
  for (int64_t k = 0; k < nreq; k++) {
    int64_t s = (int64_t)std::llround(std::exp(unif() * std::log((double)max_batch)));
    size[k] = std::max<int64_t>(1, std::min<int64_t>(s, max_batch));
    off[k + 1] = off[k] + size[k];
    if (rate > 0) t += -std::log(unif()) / rate;
    at[k] = t;
  }
  std::vector<int32_t> pairs((size_t)off[nreq] * 2);
  for (auto &p : pairs) p = (int32_t)(next() % (uint64_t)n);
  // answers: 1 byte each (4 on a weighted index)
  std::vector<uint8_t> outb((size_t)off[nreq] * (index_weighted(idx) ? 4 : 1));
  pll_server *sv = nullptr;
  int rc = pll_server_start(idx, nslots, slot_pairs, &sv);
  if (rc != PLL_OK) return rc;
  const int64_t t0 = now_ns() + 1000000;  // start 1 ms from now
  std::vector<int64_t> tickets((size_t)nreq, -1);
  for (int64_t k = 0; k < nreq; k++) {
    const int64_t due = t0 + (int64_t)(at[k] * 1e9);
    while (now_ns() < due) {
    }
    rc = submit_at(sv, pairs.data() + 2 * off[k], size[k], outb.data() + off[k] * sv->es, due,
                   &tickets[(size_t)k]);
    if (rc != PLL_OK) break;
  }
  std::vector<double> lat((size_t)nreq);
  int64_t t_last = t0;
  for (int64_t k = 0; rc == PLL_OK && k < nreq; k++) {
    double us = 0;
    const int r = pll_server_done(sv, tickets[(size_t)k], 1, &us);
    if (r < 0) {
      rc = r;
      break;
    }
    lat[k] = us;
    // answered at its scheduled arrival + its latency
    t_last = std::max<int64_t>(t_last, t0 + (int64_t)(at[k] * 1e9) + (int64_t)(us * 1e3));
  }
  int64_t sst[6] = {0, 0, 0, 0, -1, -1};
  const int rc2 = pll_server_stop(sv, sst, 6);
  if (rc != PLL_OK) return rc;
  if (rc2 != PLL_OK) return rc2;
  std::vector<double> sorted(lat);
  std::sort(sorted.begin(), sorted.end());
  auto pct = [&](double p) {
    const double pos = p / 100.0 * (double)(nreq - 1);
    const int64_t a = (int64_t)pos;
    const int64_t b = std::min<int64_t>(a + 1, nreq - 1);
    return sorted[a] + (sorted[b] - sorted[a]) * (pos - (double)a);
  };
  double mean = 0;
  for (double v : lat) mean += v;
  mean /= (double)nreq;
  const double secs = (double)(t_last - t0) * 1e-9;
  const double st[12] = {pct(50),
                         pct(99),
                         mean,
                         (double)off[nreq] / secs,
                         (double)nreq / secs,
                         secs,
                         (double)sst[0],
                         sst[0] ? (double)sst[1] / (double)sst[0] : 0.0,
                         (double)sst[2],
                         (double)sst[3] * 1e-3,
                         (double)sst[4],
                         (double)sst[5] * 1e-3};
  for (int32_t i = 0; stats && i < nstats && i < 12; i++) stats[i] = st[i];
  return PLL_OK;
}

}  // extern "C"
