// ring.hip — streaming output through a bounded ring (the C ABI inc_ring_* of
// include/inc.h).  The secondaries of a batch flow through a ring of a fixed
// number of records in coherent host memory while the kernel runs; the
// calling thread drains the ring into the caller's arrays and hands the space
// back, so the secondary output needs no device buffer sized by the batch.
// The producer waits (bounded) when the ring is full; no record is lost or
// duplicated.  Sequence numbers run on across calls, so stale tags of an
// earlier call can never be taken for new records.
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "copy_pool.h"
#include "ctx.h"

using incdev::CopyPool;
using incdev::RingDev;
using incdev::Segment;

namespace {

constexpr size_t kCopyChunk = 16384;  // records per chunk of a parallel copy

}  // namespace

struct inc_ring {
  inc_ctx* ctx;
  size_t slots;
  uint32_t* h_rec;                // 7 arrays of `slots` words (tag, ev, kind, T, ux, uy, uz), coherent host memory
  unsigned long long* h_ctrl;     // [0] tail (consumed), [1] error flag word
  uint32_t* d_rec;
  unsigned long long* d_ctrl;
  unsigned long long* d_dev;      // device: [0] head, [1..2] work queues, [4..5] counters
  Segment* d_seg;
  unsigned long long next_seq;    // head after the last call
  CopyPool* pool;                 // host copy workers (NULL: the caller copies alone)
};

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

extern "C" {

int inc_ring_create(inc_ctx* ctx, size_t slots, inc_ring** out) {
  if (!out) return INC_ERR_ARG;
  *out = nullptr;
  if (!ctx || slots < 1024 || (slots & (slots - 1)) != 0 || slots > (1ull << 30)) return INC_ERR_ARG;
  inc_ring* r = new (std::nothrow) inc_ring;
  if (!r) return INC_ERR_OOM;
  memset(r, 0, sizeof(*r));
  r->ctx = ctx;
  r->slots = slots;
  hipError_t e = hipHostMalloc(&r->h_rec, slots * 28, hipHostMallocCoherent | hipHostMallocMapped);
  if (e == hipSuccess) e = hipHostMalloc(&r->h_ctrl, 64, hipHostMallocCoherent | hipHostMallocMapped);
  if (e == hipSuccess) {
    memset(r->h_rec, 0, slots * 28);
    memset(r->h_ctrl, 0, 64);
    e = hipHostGetDevicePointer((void**)&r->d_rec, r->h_rec, 0);
  }
  if (e == hipSuccess) e = hipHostGetDevicePointer((void**)&r->d_ctrl, r->h_ctrl, 0);
  if (e == hipSuccess) e = hipMalloc(&r->d_dev, 8 * sizeof(unsigned long long));
  if (e == hipSuccess) e = hipMalloc(&r->d_seg, sizeof(Segment));
  if (e == hipSuccess) {
    const unsigned long long zero[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    e = hipMemcpy(r->d_dev, zero, sizeof(zero), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    inc_ring_destroy(r);
    return inc_map_hip_error(e);
  }
  const unsigned hw = std::thread::hardware_concurrency();
  const int workers = hw > 1 ? (int)std::min(hw - 1, 7u) : 0;
  if (workers > 0) r->pool = new (std::nothrow) CopyPool(workers);
  *out = r;
  return INC_OK;
}

int inc_ring_destroy(inc_ring* r) {
  if (!r) return INC_ERR_ARG;
  if (r->h_rec) (void)hipHostFree(r->h_rec);
  if (r->h_ctrl) (void)hipHostFree(r->h_ctrl);
  if (r->d_dev) (void)hipFree(r->d_dev);
  if (r->d_seg) (void)hipFree(r->d_seg);
  delete r->pool;
  delete r;
  return INC_OK;
}

}  // extern "C"

namespace {

// One batch through the ring: launch, drain while the kernel runs, and hand
// each run of ready records either to `consumer` or into the host arrays of
// `out` (one of the two), then the slots back to the producer.
int ring_run(inc_ring* r, const inc_batch* b, inc_residual* d_res, inc_residual* h_res, const inc_host_output* out,
             inc_ring_consumer consumer, void* user, unsigned long long* n_sec_out, void* stream, int mode,
             inc_ring_stats* stats) {
  if (!r || !b || !d_res || !b->T0 || b->n < 1 || b->n >= (1ull << 32)) return INC_ERR_ARG;
  if (mode != INC_MODE_PLAIN && mode != INC_MODE_PERSISTENT && mode != INC_MODE_STAGED) return INC_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  volatile unsigned long long* tail_p = r->h_ctrl;
  volatile unsigned int* err_p = (volatile unsigned int*)(r->h_ctrl + 1);
  if (*err_p) return INC_ERR_DEVICE;  // an earlier call gave up: the ring state is unknown
  const unsigned long long start = r->next_seq;
  Segment seg;
  memset(&seg, 0, sizeof(seg));
  seg.start = 0;
  seg.n = (uint32_t)b->n;
  seg.first_id = b->first_event_id;
  seg.res = d_res;
  seg.counters = r->d_dev + 4;
  RingDev R;
  R.tag = r->d_rec;
  R.ev = r->d_rec + r->slots;
  R.kind = r->d_rec + 2 * r->slots;
  R.T = r->d_rec + 3 * r->slots;
  R.ux = r->d_rec + 4 * r->slots;
  R.uy = r->d_rec + 5 * r->slots;
  R.uz = r->d_rec + 6 * r->slots;
  R.mask = r->slots - 1;
  R.head = r->d_dev;
  R.tail = r->d_ctrl;
  R.error = (unsigned int*)(r->d_ctrl + 1);
  R.spin_limit = 2000000ull;  // ~3 s without progress of the consumer
  hipEvent_t done;
  hipError_t e = hipEventCreateWithFlags(&done, hipEventDisableTiming);
  if (e != hipSuccess) return inc_map_hip_error(e);
  int rc = inc_map_hip_error(inc_upload_segment(seg, r->d_seg, st));
  if (rc == INC_OK)
    rc = inc_launch_segments(r->ctx, b->n, b->target_idx, b->T0, r->d_seg, 1, b->seed, r->d_dev + 1, st, mode, 0,
                             &R);
  if (rc == INC_OK) rc = inc_map_hip_error(hipEventRecord(done, st));
  // residuals to the host as well: into pinned memory the copy is queued
  // behind the kernel now and overlaps the drain; pageable memory is copied
  // once the drain is over (a blocking copy now would stall the drain the
  // kernel waits on)
  bool res_queued = false;
  if (rc == INC_OK && h_res) {
    hipPointerAttribute_t pa;
    if (hipPointerGetAttributes(&pa, h_res) == hipSuccess && pa.type == hipMemoryTypeHost) {
      rc = inc_map_hip_error(
          hipMemcpyAsync(h_res, d_res, sizeof(inc_residual) * b->n, hipMemcpyDeviceToHost, st));
      res_queued = rc == INC_OK;
    } else {
      (void)hipGetLastError();  // pageable memory is not an error here
    }
  }
  if (rc != INC_OK) {
    (void)hipStreamSynchronize(st);
    (void)hipEventDestroy(done);
    return rc;
  }
  // ---- drain while the kernel runs
  unsigned long long tail = start, final_head = ~0ull, max_fill = 0, copied = 0, waits = 0;
  const size_t cap_out = out ? out->sec_capacity : 0;
  const unsigned long long mask = r->slots - 1;
  bool kernel_done = false;
  const double t0 = now_s();
  double t_last = t0;
  while (true) {
    bool progressed = false;
    const uint32_t* h_tag = r->h_rec;
    const size_t S = r->slots;
    while (true) {
      // the run of ready records starting at tail, within the ring's linear
      // range: tags are compared 16 at a time (plain loads; the acquire fence
      // below orders the record reads after them)
      const size_t j = (size_t)(tail & mask);
      const size_t lim = std::min<size_t>(S - j, 1u << 18);
      size_t run = 0;
      while (run < lim) {
        const size_t q = std::min<size_t>(16, lim - run);
        uint32_t t16[16];
        memcpy(t16, h_tag + j + run, 4 * q);
        std::atomic_signal_fence(std::memory_order_seq_cst);
        size_t ok = 0;
        while (ok < q && t16[ok] == (uint32_t)(tail + run + ok + 1ull)) ++ok;
        run += ok;
        if (ok < q) break;
      }
      if (run == 0) break;
      __atomic_thread_fence(__ATOMIC_ACQUIRE);
      const unsigned long long k = tail - start;
      if (consumer) {
        const uint32_t* rec = r->h_rec;
        inc_ring_chunk c;
        c.first = k;
        c.n = run;
        c.event = rec + S + j;
        c.kind = rec + 2 * S + j;
        c.T = (const float*)(rec + 3 * S + j);
        c.ux = (const float*)(rec + 4 * S + j);
        c.uy = (const float*)(rec + 5 * S + j);
        c.uz = (const float*)(rec + 6 * S + j);
        consumer(&c, user);
        copied += run;
      } else if (out && k < cap_out) {
        const size_t m = (size_t)std::min<unsigned long long>(run, cap_out - k);
        const uint32_t* rec = r->h_rec;
        auto copy = [&, j, k](size_t a, size_t b) {
          const size_t n = b - a;
          if (out->sec_event) memcpy(out->sec_event + k + a, rec + S + j + a, 4 * n);
          if (out->sec_T) memcpy(out->sec_T + k + a, rec + 3 * S + j + a, 4 * n);
          if (out->sec_ux) memcpy(out->sec_ux + k + a, rec + 4 * S + j + a, 4 * n);
          if (out->sec_uy) memcpy(out->sec_uy + k + a, rec + 5 * S + j + a, 4 * n);
          if (out->sec_uz) memcpy(out->sec_uz + k + a, rec + 6 * S + j + a, 4 * n);
          if (out->sec_species || out->sec_stage) {
            const uint32_t* kind = rec + 2 * S + j;
            for (size_t q = a; q < b; ++q) {
              const uint32_t kd = kind[q];
              if (out->sec_species) out->sec_species[k + q] = (uint8_t)(kd & 0xFFu);
              if (out->sec_stage) out->sec_stage[k + q] = (uint8_t)((kd >> 8) & 0xFFu);
            }
          }
        };
        if (r->pool && m >= 2 * kCopyChunk) {
          const int nc = (int)((m + kCopyChunk - 1) / kCopyChunk);
          const std::function<void(int)> fn = [&](int c) {
            copy((size_t)c * kCopyChunk, std::min(m, (size_t)(c + 1) * kCopyChunk));
          };
          r->pool->run(nc, fn);
        } else {
          copy(0, m);
        }
        copied += m;
      }
      tail += run;
      progressed = true;
      __atomic_store_n((unsigned long long*)tail_p, tail, __ATOMIC_RELEASE);
    }
    if (progressed) __atomic_store_n((unsigned long long*)tail_p, tail, __ATOMIC_RELEASE);
    if (!kernel_done) {
      const hipError_t q = hipEventQuery(done);
      if (q == hipSuccess) {
        kernel_done = true;
        t_last = now_s();
        e = hipMemcpy(&final_head, r->d_dev, sizeof(final_head), hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
          rc = inc_map_hip_error(e);
          break;
        }
      } else if (q != hipErrorNotReady) {
        rc = inc_map_hip_error(q);
        (void)hipStreamSynchronize(st);
        break;
      }
    }
    if (kernel_done && (tail >= final_head || *err_p)) break;
    if (progressed) {
      t_last = now_s();
    } else {
      ++waits;
      // every record is tagged before the kernel ends: a missing tag after
      // the end (2 s without progress) is an error, not a reason to wait on
      if (kernel_done && now_s() - t_last > 2.0) {
        rc = INC_ERR_DEVICE;
        break;
      }
      std::this_thread::sleep_for(std::chrono::microseconds(5));
    }
  }
  (void)hipEventDestroy(done);
  if (h_res && rc == INC_OK) {
    const hipError_t ce =
        res_queued ? hipStreamSynchronize(st)
                   : hipMemcpy(h_res, d_res, sizeof(inc_residual) * b->n, hipMemcpyDeviceToHost);
    if (ce != hipSuccess) rc = inc_map_hip_error(ce);
  } else if (res_queued) {
    (void)hipStreamSynchronize(st);
  }
  if (kernel_done) r->next_seq = final_head;
  if (rc == INC_OK && *err_p) rc = INC_ERR_DEVICE;
  const unsigned long long produced = kernel_done ? final_head - start : tail - start;
  if (n_sec_out) *n_sec_out = produced;
  if (stats) {
    stats->records = produced;
    stats->slots = r->slots;
    stats->wraps = produced / r->slots;
    stats->consumer_idle_polls = waits;
    stats->seconds = now_s() - t0;
    stats->producer_gave_up = *err_p;
  }
  (void)max_fill;
  if (rc == INC_OK && !consumer && out && produced > cap_out) rc = INC_ERR_CAPACITY;
  (void)copied;
  return rc;
}

}  // namespace

extern "C" {

int inc_ring_simulate(inc_ring* r, const inc_batch* b, inc_residual* d_res, const inc_host_output* out, void* stream,
                      int mode, inc_ring_stats* stats) {
  return ring_run(r, b, d_res, out ? out->res : nullptr, out, nullptr, nullptr, out ? out->n_sec : nullptr, stream,
                  mode, stats);
}

int inc_ring_simulate_to(inc_ring* r, const inc_batch* b, inc_residual* d_res, inc_residual* h_res,
                         inc_ring_consumer consumer, void* user, unsigned long long* n_sec, void* stream, int mode,
                         inc_ring_stats* stats) {
  if (!consumer || !n_sec) return INC_ERR_ARG;
  return ring_run(r, b, d_res, h_res, nullptr, consumer, user, n_sec, stream, mode, stats);
}

}  // extern "C"
