// server.hip — continuous-batching serving loop over a context (the C ABI
// inc_server_* of include/inc.h).
//
// Event batches (requests) come from a proton-transport stepper as they
// arrive.  A request is admitted when a slot (a HIP stream) is free and its
// buffers fit in the HBM budget; it then runs as its own persistent-kernel
// launch sized to its event count, so requests admitted while others run
// overlap on the device.  The nucleus, cross-section and binding tables stay
// resident in the context; each request keeps its own event ids, so its
// results are the same alone and in the mix.  Results come back through a
// pinned host mirror of the device pool.
#include <string.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ctx.h"

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

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

// Offsets of one request's buffers inside its pool region.
struct Layout {
  size_t T0, tidx, res, cnt, sec_T, sec_ux, sec_uy, sec_uz, sec_event, sec_species, sec_stage, total;
  static Layout of(size_t n, size_t cap) {
    Layout L;
    size_t o = 0;
    L.T0 = o;          o += align_up(4 * n);
    L.tidx = o;        o += align_up(n);
    L.res = o;         o += align_up(sizeof(inc_residual) * n);
    L.cnt = o;         o += align_up(4 * sizeof(unsigned long long));
    L.sec_T = o;       o += align_up(4 * cap);
    L.sec_ux = o;      o += align_up(4 * cap);
    L.sec_uy = o;      o += align_up(4 * cap);
    L.sec_uz = o;      o += align_up(4 * cap);
    L.sec_event = o;   o += align_up(4 * cap);
    L.sec_species = o; o += align_up(cap);
    L.sec_stage = o;   o += align_up(cap);
    L.total = o;
    return L;
  }
};

enum Phase { kRunning = 0, kCopying = 1, kReady = 2 };

struct Request {
  size_t n, cap, off;
  Layout L;
  int slot;
  int phase;
  hipEvent_t ev_kernel, ev_copy;
  unsigned long long n_sec;
  int rc;
  double t_submit, t_done;
};

}  // namespace

struct inc_server {
  inc_ctx* ctx;
  char* d_pool;
  char* h_pool;
  size_t budget;
  Pool pool;
  std::vector<hipStream_t> streams;
  std::vector<int> slot_busy;
  std::unordered_map<uint64_t, Request> reqs;
  uint64_t next_ticket;
  inc_server_stats st;
};

namespace {

void finish_copy_phase(inc_server* s, Request& r) {
  // results are in the pinned mirror; the slot (stream) is free again
  r.phase = kReady;
  r.t_done = now_s();
  s->slot_busy[r.slot] = 0;
  s->st.completed += 1;
  s->st.events += r.n;
  s->st.secondaries += r.n_sec;
}

// Advance one request's phase without blocking; returns 1 when ready.
int advance(inc_server* s, Request& r) {
  if (r.phase == kRunning) {
    const hipError_t q = hipEventQuery(r.ev_kernel);
    if (q == hipErrorNotReady) return 0;
    if (q != hipSuccess) {
      r.rc = inc_map_hip_error(q);
      finish_copy_phase(s, r);
      return 1;
    }
    const unsigned long long* cnt = (const unsigned long long*)(s->h_pool + r.off + r.L.cnt);
    r.n_sec = cnt[0];
    if (r.n_sec > r.cap) r.rc = INC_ERR_CAPACITY;
    const size_t k = (size_t)std::min<unsigned long long>(r.n_sec, r.cap);
    hipStream_t st = s->streams[r.slot];
    hipError_t e = hipSuccess;
    const size_t offs[7] = {r.L.sec_T, r.L.sec_ux, r.L.sec_uy, r.L.sec_uz, r.L.sec_event, r.L.sec_species,
                            r.L.sec_stage};
    const size_t width[7] = {4, 4, 4, 4, 4, 1, 1};
    for (int f = 0; f < 7 && e == hipSuccess && k; ++f)
      e = hipMemcpyAsync(s->h_pool + r.off + offs[f], s->d_pool + r.off + offs[f], width[f] * k,
                         hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipEventRecord(r.ev_copy, st);
    if (e != hipSuccess) {
      r.rc = inc_map_hip_error(e);
      finish_copy_phase(s, r);
      return 1;
    }
    r.phase = kCopying;
  }
  if (r.phase == kCopying) {
    const hipError_t q = hipEventQuery(r.ev_copy);
    if (q == hipErrorNotReady) return 0;
    if (q != hipSuccess && r.rc == INC_OK) r.rc = inc_map_hip_error(q);
    finish_copy_phase(s, r);
  }
  return 1;
}

void drop(inc_server* s, uint64_t ticket) {
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return;
  Request& r = it->second;
  (void)hipEventDestroy(r.ev_kernel);
  (void)hipEventDestroy(r.ev_copy);
  if (r.phase != kReady) s->slot_busy[r.slot] = 0;
  s->pool.release(r.off, r.L.total);
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
  s->d_pool = nullptr;
  s->h_pool = nullptr;
  s->next_ticket = 1;
  memset(&s->st, 0, sizeof(s->st));
  hipError_t e = hipMalloc(&s->d_pool, hbm_budget);
  if (e == hipSuccess) e = hipHostMalloc(&s->h_pool, hbm_budget, hipHostMallocDefault);
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
  std::vector<uint64_t> tickets;
  for (auto& kv : s->reqs) tickets.push_back(kv.first);
  for (uint64_t t : tickets) drop(s, t);
  for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
  if (s->d_pool) (void)hipFree(s->d_pool);
  if (s->h_pool) (void)hipHostFree(s->h_pool);
  delete s;
  return INC_OK;
}

int inc_server_submit(inc_server* s, const inc_request* q, uint64_t* ticket) {
  if (!s || !q || !ticket || !q->T0 || q->n < 1 || q->n >= (1ull << 32)) return INC_ERR_ARG;
  const size_t cap = q->sec_capacity ? q->sec_capacity : q->n * 12 + 4096;
  const Layout L = Layout::of(q->n, cap);
  if (L.total > s->budget) return INC_ERR_ARG;  // never admissible
  int slot = -1;
  for (size_t i = 0; i < s->streams.size(); ++i)
    if (!s->slot_busy[i]) {
      slot = (int)i;
      break;
    }
  size_t off = 0;
  if (slot < 0 || !s->pool.alloc(L.total, &off)) {
    s->st.rejected_busy += 1;
    return INC_ERR_BUSY;
  }
  Request r;
  r.n = q->n;
  r.cap = cap;
  r.off = off;
  r.L = L;
  r.slot = slot;
  r.phase = kRunning;
  r.n_sec = 0;
  r.rc = INC_OK;
  r.t_submit = now_s();
  r.t_done = 0.0;
  hipStream_t st = s->streams[slot];
  char* h = s->h_pool + off;
  char* d = s->d_pool + off;
  memcpy(h + L.T0, q->T0, 4 * q->n);
  if (q->target_idx) memcpy(h + L.tidx, q->target_idx, q->n);
  hipError_t e = hipEventCreateWithFlags(&r.ev_kernel, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&r.ev_copy, hipEventDisableTiming);
  if (e == hipSuccess) e = hipMemcpyAsync(d + L.T0, h + L.T0, 4 * q->n, hipMemcpyHostToDevice, st);
  if (e == hipSuccess && q->target_idx) e = hipMemcpyAsync(d + L.tidx, h + L.tidx, q->n, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) {
    s->pool.release(off, L.total);
    return inc_map_hip_error(e);
  }
  inc_batch b = {q->n, q->target_idx ? (const uint8_t*)(d + L.tidx) : nullptr, (const float*)(d + L.T0), q->seed,
                 q->first_event_id};
  inc_output o;
  o.res = (inc_residual*)(d + L.res);
  o.sec_T = (float*)(d + L.sec_T);
  o.sec_ux = (float*)(d + L.sec_ux);
  o.sec_uy = (float*)(d + L.sec_uy);
  o.sec_uz = (float*)(d + L.sec_uz);
  o.sec_event = (uint32_t*)(d + L.sec_event);
  o.sec_species = (uint8_t*)(d + L.sec_species);
  o.sec_stage = (uint8_t*)(d + L.sec_stage);
  o.sec_capacity = cap;
  o.counters = (unsigned long long*)(d + L.cnt);
  // one lane per event at most: small requests take fewer blocks
  const int blocks = (int)((q->n + s->ctx->block - 1) / s->ctx->block);
  int rc = inc_launch_batch(s->ctx, &b, &o, st, INC_MODE_PERSISTENT, blocks);
  if (rc == INC_OK) {
    e = hipMemcpyAsync(h + L.cnt, d + L.cnt, 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(h + L.res, d + L.res, sizeof(inc_residual) * q->n, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipEventRecord(r.ev_kernel, st);
    rc = inc_map_hip_error(e);
  }
  if (rc != INC_OK) {
    (void)hipStreamSynchronize(st);
    (void)hipEventDestroy(r.ev_kernel);
    (void)hipEventDestroy(r.ev_copy);
    s->pool.release(off, L.total);
    return rc;
  }
  s->slot_busy[slot] = 1;
  *ticket = s->next_ticket++;
  s->reqs.emplace(*ticket, r);
  s->st.submitted += 1;
  return INC_OK;
}

int inc_server_poll(inc_server* s, uint64_t ticket) {
  if (!s) return INC_ERR_ARG;
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return INC_ERR_ARG;
  return advance(s, it->second);
}

int inc_server_wait(inc_server* s, uint64_t ticket) {
  if (!s) return INC_ERR_ARG;
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return INC_ERR_ARG;
  Request& r = it->second;
  while (advance(s, r) == 0) {
    (void)hipEventSynchronize(r.phase == kRunning ? r.ev_kernel : r.ev_copy);
  }
  return 1;
}

int inc_server_fetch(inc_server* s, uint64_t ticket, const inc_host_output* out) {
  if (!s) return INC_ERR_ARG;
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return INC_ERR_ARG;
  Request& r = it->second;
  if (r.phase != kReady) return INC_ERR_BUSY;
  const int rc = r.rc;
  if (out) {
    const char* h = s->h_pool + r.off;
    const size_t k = (size_t)std::min<unsigned long long>(r.n_sec, std::min(r.cap, out->sec_capacity));
    if (out->res) memcpy(out->res, h + r.L.res, sizeof(inc_residual) * r.n);
    if (k) {
      if (out->sec_T) memcpy(out->sec_T, h + r.L.sec_T, 4 * k);
      if (out->sec_ux) memcpy(out->sec_ux, h + r.L.sec_ux, 4 * k);
      if (out->sec_uy) memcpy(out->sec_uy, h + r.L.sec_uy, 4 * k);
      if (out->sec_uz) memcpy(out->sec_uz, h + r.L.sec_uz, 4 * k);
      if (out->sec_event) memcpy(out->sec_event, h + r.L.sec_event, 4 * k);
      if (out->sec_species) memcpy(out->sec_species, h + r.L.sec_species, k);
      if (out->sec_stage) memcpy(out->sec_stage, h + r.L.sec_stage, k);
    }
    if (out->n_sec) *out->n_sec = r.n_sec;
    if (out->latency_s) *out->latency_s = r.t_done - r.t_submit;
  }
  drop(s, ticket);
  return rc;
}

int inc_server_stats_get(inc_server* s, inc_server_stats* out) {
  if (!s || !out) return INC_ERR_ARG;
  *out = s->st;
  out->in_flight = s->reqs.size();
  out->pool_free_largest = s->pool.largest();
  return INC_OK;
}

int inc_server_replay(inc_server* s, int n_req, const double* arrival_s, const inc_request* reqs, double* latency_s,
                      double* span_s) {
  if (!s || n_req < 1 || !arrival_s || !reqs || !latency_s) return INC_ERR_ARG;
  for (int i = 0; i < n_req; ++i) {
    if (i && arrival_s[i] < arrival_s[i - 1]) return INC_ERR_ARG;
    const size_t cap = reqs[i].sec_capacity ? reqs[i].sec_capacity : reqs[i].n * 12 + 4096;
    if (Layout::of(reqs[i].n, cap).total > s->budget) return INC_ERR_ARG;
  }
  std::vector<uint64_t> ticket(n_req, 0);
  std::vector<int> state(n_req, 0);  // 0 waiting, 1 in flight, 2 done
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
      state[k] = 1;
      ++head;
      progressed = true;
    }
    for (int k = 0; k < n_req; ++k) {
      if (state[k] != 1) continue;
      auto it = s->reqs.find(ticket[k]);
      if (advance(s, it->second)) {
        latency_s[k] = it->second.t_done - t0 - arrival_s[k];
        t_last = it->second.t_done;
        const int rc = inc_server_fetch(s, ticket[k], nullptr);
        if (rc != INC_OK && rc_all == INC_OK) rc_all = rc;
        state[k] = 2;
        ++done;
        progressed = true;
      }
    }
    if (!progressed) {
      // nothing to do: the next arrival or a completion
      std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
  }
  if (span_s) *span_s = t_last - t0 - arrival_s[0];
  return rc_all;
}

}  // extern "C"
