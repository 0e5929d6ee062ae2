// server.hip — continuous-batching serving loop over a context (the C ABI
// inc_server_* of include/inc.h).
//
// Event batches (requests) come from a proton-transport stepper as they
// arrive.  A request is admitted when its buffers fit in the HBM budget and
// joins the queue.  Whenever one of the server's slots (HIP streams) is free,
// every queued request with the same random-stream key is launched together
// as ONE persistent-kernel launch: each request is a segment of that launch
// with its own event ids and output buffers, so a request's results do not
// depend on what it was batched with.  Launches on different slots overlap
// on the device, so the tail of one launch runs beside the bulk of the next.
// Nucleus, cross-section and binding tables stay resident in the context.
// Results come back through a pinned host mirror of the device pool.
#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ctx.h"

using incdev::MidState;
using incdev::Segment;

namespace {

constexpr size_t kAlign = 256;
constexpr size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

// Requests per launch: a secondary record names its request (segment of the
// launch) in 16 bits of its kind word (species | stage << 8 | segment << 16).
constexpr size_t kMaxLaunchSegments = 65535;
// Pool bytes a launch needs beyond its requests' own (work-queue heads, and
// alignment of the segment table and the hand-over buffer); admission keeps
// this much free for every slot, so the queue head can always start once the
// launches in flight have been fetched.
constexpr size_t kLaunchFixed = 16 * 16 + 2 * kAlign;

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over [0, size) of the device pool.
class Pool {
 public:
  void reset(size_t size) {
    free_.clear();
    free_[0] = size;
  }
  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t largest() const {
    size_t m = 0;
    for (const auto& kv : free_) m = std::max(m, kv.second);
    return m;
  }

 private:
  std::map<size_t, size_t> free_;
};

// Secondary records reserved for a request that names no capacity: above the
// mean multiplicity of every real target up to 250 MeV (about 4.6 per event
// for 16O, 5.8 for 40Ca, 15 for A = 250), at most A + 1 per event.
size_t default_cap(const inc_ctx* ctx, size_t n) {
  const size_t a = (size_t)ctx->amax;  // largest target A + 1
  const size_t per_event = std::min(a, 6 + (a - 1) / 10);
  return n * per_event + 4096;
}

// Device bytes a request needs inside a launch (inputs, its share of the
// staged hand-over buffer, residuals, secondaries, counters, segment entry).
size_t request_bytes(size_t n, size_t cap) {
  return align_up(4 * n) + align_up(n) + align_up(incdev::mid_bytes(n)) + align_up(sizeof(inc_residual) * n) +
         5 * align_up(4 * cap) + 2 * align_up(cap) + align_up(4 * sizeof(unsigned long long)) +
         align_up(sizeof(Segment));
}

enum RState { kQueued = 0, kLaunched = 1, kReady = 2 };
enum LPhase { kRunning = 0, kDone = 1 };

// Offsets of one request's buffers inside its launch region.
struct ROffsets {
  size_t res, cnt, T, ux, uy, uz, ev, sp, st;
};

struct Request {
  size_t n, cap;
  uint64_t seed, first_id;
  std::vector<float> T0;
  std::vector<uint8_t> tidx;
  bool has_tidx;
  size_t bytes;       // admission charge
  int state;
  int launch;
  size_t start;       // first event of the request in its launch
  ROffsets o;
  unsigned long long n_sec;
  int rc;
  double t_submit, t_done;
  double t_arrival;   // latency origin: submit, or the arrival time a replay gives
};

struct Launch {
  int slot;
  size_t off, bytes;
  size_t n;
  std::vector<uint64_t> tickets;
  size_t seg_off, queue_off;
  int phase;
  hipEvent_t ev_kernel;  // after the cascade, evaporation and export kernels (NULL if not created)
  int pending_fetch;
};

}  // namespace

struct inc_server {
  inc_ctx* ctx;
  char* d_pool;
  char* h_pool;       // pinned host mirror of d_pool (mapped)
  char* h_pool_dev;   // device address of h_pool
  size_t budget;
  size_t charged;     // bytes promised to admitted, not yet fetched requests
  Pool pool;
  std::vector<hipStream_t> streams;
  std::vector<int> slot_busy;
  std::unordered_map<uint64_t, Request> reqs;
  std::deque<uint64_t> queue;
  std::map<int, Launch> launches;
  int next_launch;
  uint64_t next_ticket;
  inc_server_stats st;
  int hold;                      // 1: admit and queue, start no launch
  std::vector<double> latencies; // arrival -> results on host, completed requests
  double t_first_arrival, t_last_done;
};

namespace {

// Copy every request's results of a launch into the mapped host mirror of the
// pool (same layout, `delta` bytes away): counters, residuals and the
// secondaries the request produced (at most its capacity), so that one event
// after the kernels says the results are on the host.  Grid: (segments, parts).
__global__ void k_export(const Segment* segs, long long delta) {
  const Segment& S = segs[blockIdx.x];
  const unsigned long long produced = S.counters[0];
  const size_t k = (size_t)(produced < S.cap ? produced : S.cap);
  const size_t tid = (size_t)blockIdx.y * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.y * blockDim.x;
  if (tid < 4) ((unsigned long long*)((char*)S.counters + delta))[tid] = S.counters[tid];
  static_assert(sizeof(inc_residual) % sizeof(uint4) == 0, "residuals move as 16-byte words");
  const uint4* rs = (const uint4*)S.res;
  uint4* rd = (uint4*)((char*)S.res + delta);
  const size_t words = sizeof(inc_residual) / sizeof(uint4) * (size_t)S.n;
  for (size_t i = tid; i < words; i += stride) rd[i] = rs[i];
  float* T = (float*)((char*)S.T + delta);
  float* ux = (float*)((char*)S.ux + delta);
  float* uy = (float*)((char*)S.uy + delta);
  float* uz = (float*)((char*)S.uz + delta);
  uint32_t* ev = (uint32_t*)((char*)S.ev + delta);
  uint8_t* sp = (uint8_t*)((char*)S.species + delta);
  uint8_t* st = (uint8_t*)((char*)S.stage + delta);
  for (size_t i = tid; i < k; i += stride) {
    T[i] = S.T[i];
    ux[i] = S.ux[i];
    uy[i] = S.uy[i];
    uz[i] = S.uz[i];
    ev[i] = S.ev[i];
    sp[i] = S.species[i];
    st[i] = S.stage[i];
  }
}

void complete_launch(inc_server* s, Launch& L, int rc) {
  const double t = now_s();
  for (uint64_t tk : L.tickets) {
    Request& r = s->reqs[tk];
    if (rc != INC_OK && r.rc == INC_OK) r.rc = rc;
    r.state = kReady;
    r.t_done = t;
    s->st.completed += 1;
    s->st.events += r.n;
    s->st.secondaries += r.n_sec;
    s->latencies.push_back(t - r.t_arrival);
    if (s->latencies.size() == 1 || r.t_arrival < s->t_first_arrival) s->t_first_arrival = r.t_arrival;
    s->t_last_done = t;
  }
  L.phase = kDone;
  s->slot_busy[L.slot] = 0;
}

// Advance a launch without blocking.
void advance_launch(inc_server* s, Launch& L) {
  if (L.phase == kRunning && L.ev_kernel) {
    const hipError_t q = hipEventQuery(L.ev_kernel);
    if (q == hipErrorNotReady) return;
    if (q != hipSuccess) {
      complete_launch(s, L, inc_map_hip_error(q));
      return;
    }
    // the export kernel has put counters, residuals and secondaries in the mirror
    for (uint64_t tk : L.tickets) {
      Request& r = s->reqs[tk];
      const unsigned long long* cnt = (const unsigned long long*)(s->h_pool + L.off + r.o.cnt);
      r.n_sec = cnt[0];
      if (r.n_sec > r.cap) r.rc = INC_ERR_CAPACITY;
    }
    complete_launch(s, L, INC_OK);
  }
}

// Launch the queued requests that share the head's key on a free slot.
int start_launch(inc_server* s) {
  if (s->queue.empty() || s->hold) return INC_OK;
  int slot = -1;
  for (size_t i = 0; i < s->streams.size(); ++i)
    if (!s->slot_busy[i]) {
      slot = (int)i;
      break;
    }
  if (slot < 0) return INC_OK;
  // the longest prefix of the queue with the head's key that fits the
  // largest free block of the pool
  const uint64_t key = s->reqs[s->queue.front()].seed;
  const size_t room = s->pool.largest();
  const size_t fixed = align_up(2 * sizeof(unsigned long long)) + 2 * kAlign;
  static_assert(align_up(2 * sizeof(unsigned long long)) + 2 * kAlign <= kLaunchFixed, "admission reserve");
  std::vector<uint64_t> take;
  size_t n = 0, bytes = fixed;
  for (uint64_t tk : s->queue) {
    const Request& r = s->reqs[tk];
    if (r.seed != key || n + r.n >= (1ull << 31) || bytes + r.bytes > room || take.size() >= kMaxLaunchSegments)
      break;
    take.push_back(tk);
    n += r.n;
    bytes += r.bytes;
  }
  if (take.empty()) return INC_OK;  // wait for memory
  Launch L;
  if (!s->pool.alloc(bytes, &L.off)) return INC_OK;  // wait for memory
  for (size_t k = 0; k < take.size(); ++k) s->queue.pop_front();
  L.slot = slot;
  L.bytes = bytes;
  L.n = n;
  L.tickets = take;
  L.phase = kRunning;
  L.pending_fetch = (int)take.size();
  L.ev_kernel = nullptr;
  const int id = s->next_launch++;
  s->st.launches += 1;
  // layout: [T0][tidx][segments][queues][hand-over][per request: counters res T ux uy uz ev sp st]
  size_t o = 0;
  const size_t T0_off = o;   o += align_up(4 * n);
  const size_t tidx_off = o; o += align_up(n);
  L.seg_off = o;             o += align_up(sizeof(Segment) * take.size());
  L.queue_off = o;           o += align_up(2 * sizeof(unsigned long long));
  const size_t mid_off = o;  o += align_up(incdev::mid_bytes(n));
  char* h = s->h_pool + L.off;
  char* d = s->d_pool + L.off;
  bool any_tidx = false;
  size_t start = 0;
  std::vector<Segment> segs(take.size());
  for (size_t k = 0; k < take.size(); ++k) {
    Request& r = s->reqs[take[k]];
    r.state = kLaunched;
    r.launch = id;
    r.start = start;
    r.o.cnt = o; o += align_up(4 * sizeof(unsigned long long));
    r.o.res = o; o += align_up(sizeof(inc_residual) * r.n);
    r.o.T = o;   o += align_up(4 * r.cap);
    r.o.ux = o;  o += align_up(4 * r.cap);
    r.o.uy = o;  o += align_up(4 * r.cap);
    r.o.uz = o;  o += align_up(4 * r.cap);
    r.o.ev = o;  o += align_up(4 * r.cap);
    r.o.sp = o;  o += align_up(r.cap);
    r.o.st = o;  o += align_up(r.cap);
    memcpy(h + T0_off + 4 * start, r.T0.data(), 4 * r.n);
    if (r.has_tidx) {
      memcpy(h + tidx_off + start, r.tidx.data(), r.n);
      any_tidx = true;
    } else {
      memset(h + tidx_off + start, 0, r.n);
    }
    Segment& g = segs[k];
    g.start = (uint32_t)start;
    g.n = (uint32_t)r.n;
    g.first_id = r.first_id;
    g.res = (inc_residual*)(d + r.o.res);
    g.ev = (uint32_t*)(d + r.o.ev);
    g.species = (uint8_t*)(d + r.o.sp);
    g.stage = (uint8_t*)(d + r.o.st);
    g.T = (float*)(d + r.o.T);
    g.ux = (float*)(d + r.o.ux);
    g.uy = (float*)(d + r.o.uy);
    g.uz = (float*)(d + r.o.uz);
    g.cap = r.cap;
    g.counters = (unsigned long long*)(d + r.o.cnt);
    g.hist = nullptr;
    start += r.n;
  }
  memcpy(h + L.seg_off, segs.data(), sizeof(Segment) * segs.size());
  hipStream_t st = s->streams[slot];
  const size_t in_bytes = L.queue_off;  // T0, tidx and segment table are contiguous at the front
  hipError_t e = hipEventCreateWithFlags(&L.ev_kernel, hipEventDisableTiming);
  if (e != hipSuccess) L.ev_kernel = nullptr;
  if (e == hipSuccess) e = hipMemcpyAsync(d, h, in_bytes, hipMemcpyHostToDevice, st);
  int rc = inc_map_hip_error(e);
  if (rc == INC_OK) {
    // one lane per event at most: small launches take fewer blocks
    const int blocks = (int)((n + s->ctx->block - 1) / s->ctx->block);
    rc = inc_launch_segments(s->ctx, n, any_tidx ? (const uint8_t*)(d + tidx_off) : nullptr, (const float*)(d + T0_off),
                             (const Segment*)(d + L.seg_off), (int)segs.size(), key,
                             (unsigned long long*)(d + L.queue_off), st, INC_MODE_STAGED, blocks, nullptr,
                             (MidState*)(d + mid_off));
  }
  if (rc == INC_OK) {
    // results straight into the mapped mirror, exactly what each request produced
    hipLaunchKernelGGL(k_export, dim3((unsigned)segs.size(), 16), dim3(256), 0, st, (const Segment*)(d + L.seg_off),
                       (long long)(s->h_pool_dev - s->d_pool));
    rc = inc_map_hip_error(hipGetLastError());
  }
  if (rc == INC_OK) rc = inc_map_hip_error(hipEventRecord(L.ev_kernel, st));
  s->slot_busy[slot] = 1;
  s->launches.emplace(id, L);
  if (rc != INC_OK) {
    (void)hipStreamSynchronize(st);
    complete_launch(s, s->launches[id], rc);
  }
  return INC_OK;
}

// Make progress: finish launches, start new ones on free slots.
void pump(inc_server* s) {
  for (auto& kv : s->launches) advance_launch(s, kv.second);
  while (!s->queue.empty()) {
    const size_t before = s->queue.size();
    start_launch(s);
    if (s->queue.size() == before) break;
  }
}

// Pool bytes admission keeps free beyond the requests' own: one launch's fixed
// share per slot.
size_t reserve(const inc_server* s) { return kLaunchFixed * s->streams.size(); }

// True when queued work can make no progress by itself: nothing is running
// and the queue head does not fit the pool (its memory is held by results not
// yet fetched).
bool stalled(inc_server* s) {
  if (s->queue.empty() || s->hold) return false;
  for (const auto& kv : s->launches)
    if (kv.second.phase == kRunning) return false;
  return true;
}

void release_request(inc_server* s, uint64_t ticket) {
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return;
  Request& r = it->second;
  s->charged -= r.bytes;
  if (r.state != kQueued) {
    auto lt = s->launches.find(r.launch);
    if (lt != s->launches.end() && --lt->second.pending_fetch == 0) {
      Launch& L = lt->second;
      if (L.ev_kernel) (void)hipEventDestroy(L.ev_kernel);
      s->pool.release(L.off, L.bytes);
      s->launches.erase(lt);
    }
  } else {
    s->queue.erase(std::remove(s->queue.begin(), s->queue.end(), ticket), s->queue.end());
  }
  s->reqs.erase(it);
}

}  // namespace

extern "C" {

int inc_server_create(inc_ctx* ctx, size_t hbm_budget, int max_slots, inc_server** out) {
  if (!out) return INC_ERR_ARG;
  *out = nullptr;
  if (!ctx || hbm_budget < (1u << 20) || max_slots < 1 || max_slots > 16) return INC_ERR_ARG;
  inc_server* s = new (std::nothrow) inc_server;
  if (!s) return INC_ERR_OOM;
  s->ctx = ctx;
  s->budget = hbm_budget;
  s->charged = 0;
  s->d_pool = nullptr;
  s->h_pool = nullptr;
  s->h_pool_dev = nullptr;
  s->next_ticket = 1;
  s->next_launch = 1;
  memset(&s->st, 0, sizeof(s->st));
  s->hold = 0;
  s->t_first_arrival = s->t_last_done = 0.0;
  hipError_t e = hipMalloc(&s->d_pool, hbm_budget);
  if (e == hipSuccess) e = hipHostMalloc(&s->h_pool, hbm_budget, hipHostMallocMapped);
  if (e == hipSuccess) e = hipHostGetDevicePointer((void**)&s->h_pool_dev, s->h_pool, 0);
  for (int i = 0; i < max_slots && e == hipSuccess; ++i) {
    hipStream_t st;
    e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) {
      s->streams.push_back(st);
      s->slot_busy.push_back(0);
    }
  }
  if (e != hipSuccess) {
    inc_server_destroy(s);
    return inc_map_hip_error(e);
  }
  s->pool.reset(hbm_budget);
  *out = s;
  return INC_OK;
}

int inc_server_destroy(inc_server* s) {
  if (!s) return INC_ERR_ARG;
  for (hipStream_t st : s->streams) (void)hipStreamSynchronize(st);
  for (auto& kv : s->launches) {
    if (kv.second.ev_kernel) (void)hipEventDestroy(kv.second.ev_kernel);
  }
  for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
  if (s->d_pool) (void)hipFree(s->d_pool);
  if (s->h_pool) (void)hipHostFree(s->h_pool);
  delete s;
  return INC_OK;
}

int inc_server_submit(inc_server* s, const inc_request* q, uint64_t* ticket) {
  if (!s || !q || !ticket || !q->T0 || q->n < 1 || q->n >= (1ull << 31)) return INC_ERR_ARG;
  const size_t cap = q->sec_capacity ? q->sec_capacity : default_cap(s->ctx, q->n);
  const size_t bytes = request_bytes(q->n, cap);
  // a launch of this request alone must fit the pool
  if (bytes + reserve(s) > s->budget) return INC_ERR_ARG;
  pump(s);
  if (s->charged + bytes + reserve(s) > s->budget) {
    s->st.rejected_busy += 1;
    return INC_ERR_BUSY;
  }
  Request r;
  r.n = q->n;
  r.cap = cap;
  r.seed = q->seed;
  r.first_id = q->first_event_id;
  r.T0.assign(q->T0, q->T0 + q->n);
  r.has_tidx = q->target_idx != nullptr;
  if (r.has_tidx) r.tidx.assign(q->target_idx, q->target_idx + q->n);
  r.bytes = bytes;
  r.state = kQueued;
  r.launch = 0;
  r.start = 0;
  memset(&r.o, 0, sizeof(r.o));
  r.n_sec = 0;
  r.rc = INC_OK;
  r.t_submit = now_s();
  r.t_arrival = r.t_submit;
  r.t_done = 0.0;
  const uint64_t t = s->next_ticket++;
  s->reqs.emplace(t, std::move(r));
  s->queue.push_back(t);
  s->charged += bytes;
  s->st.submitted += 1;
  *ticket = t;
  pump(s);
  return INC_OK;
}

int inc_server_poll(inc_server* s, uint64_t ticket) {
  if (!s) return INC_ERR_ARG;
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return INC_ERR_ARG;
  pump(s);
  return it->second.state == kReady ? 1 : 0;
}

int inc_server_wait(inc_server* s, uint64_t ticket) {
  if (!s) return INC_ERR_ARG;
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return INC_ERR_ARG;
  while (true) {
    pump(s);
    if (it->second.state == kReady) return 1;
    // a queued request behind results nobody fetched, or held back: it
    // cannot launch until the caller acts
    if (it->second.state == kQueued && (s->hold || stalled(s))) return INC_ERR_BUSY;
    std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
}

int inc_server_hold(inc_server* s, int hold) {
  if (!s || hold < 0 || hold > 1) return INC_ERR_ARG;
  s->hold = hold;
  pump(s);
  return INC_OK;
}

int inc_server_fetch(inc_server* s, uint64_t ticket, const inc_host_output* out) {
  if (!s) return INC_ERR_ARG;
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return INC_ERR_ARG;
  Request& r = it->second;
  if (r.state != kReady) return INC_ERR_BUSY;
  const int rc = r.rc;
  if (out) {
    const char* h = s->h_pool + s->launches[r.launch].off;
    const size_t k = (size_t)std::min<unsigned long long>(r.n_sec, std::min(r.cap, out->sec_capacity));
    if (out->res) memcpy(out->res, h + r.o.res, sizeof(inc_residual) * r.n);
    if (k) {
      if (out->sec_T) memcpy(out->sec_T, h + r.o.T, 4 * k);
      if (out->sec_ux) memcpy(out->sec_ux, h + r.o.ux, 4 * k);
      if (out->sec_uy) memcpy(out->sec_uy, h + r.o.uy, 4 * k);
      if (out->sec_uz) memcpy(out->sec_uz, h + r.o.uz, 4 * k);
      if (out->sec_event) memcpy(out->sec_event, h + r.o.ev, 4 * k);
      if (out->sec_species) memcpy(out->sec_species, h + r.o.sp, k);
      if (out->sec_stage) memcpy(out->sec_stage, h + r.o.st, k);
    }
    if (out->n_sec) *out->n_sec = r.n_sec;
    if (out->latency_s) *out->latency_s = r.t_done - r.t_submit;
  }
  release_request(s, ticket);
  pump(s);
  return rc;
}

// q-quantile of a sample by linear interpolation between order statistics
// (position q (n - 1) in the sorted sample).
double quantile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  const double pos = q * (double)(v.size() - 1);
  const size_t lo = (size_t)pos;
  std::nth_element(v.begin(), v.begin() + lo, v.end());
  const double a = v[lo];
  if (lo + 1 >= v.size()) return a;
  const double b = *std::min_element(v.begin() + lo + 1, v.end());
  return a + (pos - (double)lo) * (b - a);
}

int inc_server_stats_get(inc_server* s, inc_server_stats* out) {
  if (!s || !out) return INC_ERR_ARG;
  *out = s->st;
  out->in_flight = s->reqs.size();
  out->pool_free_largest = s->pool.largest();
  out->latency_p50_s = quantile(s->latencies, 0.50);
  out->latency_p99_s = quantile(s->latencies, 0.99);
  const double span = s->t_last_done - s->t_first_arrival;
  out->events_per_s = s->latencies.empty() || !(span > 0.0) ? 0.0 : (double)s->st.events / span;
  return INC_OK;
}

int inc_server_stats_reset(inc_server* s) {
  if (!s) return INC_ERR_ARG;
  memset(&s->st, 0, sizeof(s->st));
  s->latencies.clear();
  s->t_first_arrival = s->t_last_done = 0.0;
  return INC_OK;
}

int inc_server_replay(inc_server* s, int n_req, const double* arrival_s, const inc_request* reqs, double* latency_s,
                      double* span_s) {
  if (!s || n_req < 1 || !arrival_s || !reqs || !latency_s) return INC_ERR_ARG;
  for (int i = 0; i < n_req; ++i) {
    if (i && arrival_s[i] < arrival_s[i - 1]) return INC_ERR_ARG;
    const size_t cap = reqs[i].sec_capacity ? reqs[i].sec_capacity : default_cap(s->ctx, reqs[i].n);
    if (request_bytes(reqs[i].n, cap) + reserve(s) > s->budget) return INC_ERR_ARG;
  }
  std::vector<uint64_t> ticket(n_req, 0);
  std::vector<int> state(n_req, 0);  // 0 waiting, 1 admitted, 2 done
  std::vector<int> admitted;
  int next_arrival = 0, head = 0, done = 0, rc_all = INC_OK;
  std::vector<int> fifo;
  const double t0 = now_s();
  double t_last = t0;
  while (done < n_req) {
    const double t = now_s() - t0;
    while (next_arrival < n_req && arrival_s[next_arrival] <= t) fifo.push_back(next_arrival++);
    bool progressed = false;
    // admit in arrival order (first come, first served)
    while (head < (int)fifo.size()) {
      const int k = fifo[head];
      const int rc = inc_server_submit(s, &reqs[k], &ticket[k]);
      if (rc == INC_ERR_BUSY) break;
      if (rc != INC_OK) return rc;
      s->reqs[ticket[k]].t_arrival = t0 + arrival_s[k];
      state[k] = 1;
      admitted.push_back(k);
      ++head;
      progressed = true;
    }
    pump(s);
    for (size_t a = 0; a < admitted.size();) {
      const int k = admitted[a];
      Request& r = s->reqs[ticket[k]];
      if (r.state == kReady) {
        latency_s[k] = r.t_done - r.t_arrival;
        t_last = std::max(t_last, r.t_done);
        const int rc = inc_server_fetch(s, ticket[k], nullptr);
        if (rc != INC_OK && rc_all == INC_OK) rc_all = rc;
        state[k] = 2;
        ++done;
        progressed = true;
        admitted[a] = admitted.back();
        admitted.pop_back();
      } else {
        ++a;
      }
    }
    if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
  if (span_s) *span_s = t_last - t0 - arrival_s[0];
  return rc_all;
}

}  // extern "C"
