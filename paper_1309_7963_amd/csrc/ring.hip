// ring.hip — streaming output through a bounded ring (the C ABI inc_ring_* of
// include/inc.h).  The secondaries of a batch flow through a ring of a fixed
// number of records while the kernel runs; the calling thread drains the ring
// into the caller's arrays and hands the space back, so the secondary output
// needs no device buffer sized by the batch.  The producer waits (bounded)
// when the ring is full; no record is lost or duplicated.  Sequence numbers
// run on across calls, so stale tags of an earlier call can never be taken
// for new records.  Two placements: the ring in coherent host memory (every
// record crosses PCIe as the waves store it, tagged one by one), or in device
// memory, cut into chunks that the host copies out with asynchronous copies
// on a stream of its own once the device has marked them complete.
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
  // device placement (d_ring != NULL): h_rec is the pinned mirror the chunks
  // are copied into, at the same slots (its tag array is unused)
  uint32_t* d_ring;               // chunk-major: per chunk 6 arrays of `chunk` words (ev, kind, T, ux, uy, uz)
  unsigned long long* d_done;     // records written per chunk
  unsigned long long* h_ready;    // coherent host: chunk number + 1 once complete
  unsigned long long* d_ready;
  unsigned long long* h_done0;    // pinned: the counters' values at the start of a call
  size_t chunk;                   // slots per chunk (a power of two)
  hipStream_t copy_stream;
  std::vector<hipEvent_t> copied; // completion of each queued chunk copy (round robin)
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
  inc_ring* r = new (std::nothrow) inc_ring();  // value-initialised: every pointer NULL
  if (!r) return INC_ERR_OOM;
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

int inc_ring_create_device(inc_ctx* ctx, size_t slots, size_t chunk, inc_ring** out) {
  if (!out) return INC_ERR_ARG;
  *out = nullptr;
  if (!ctx || slots < 1024 || (slots & (slots - 1)) != 0 || slots > (1ull << 30) || chunk < 1024 ||
      (chunk & (chunk - 1)) != 0 || chunk > slots / 2)
    return INC_ERR_ARG;
  inc_ring* r = nullptr;
  int rc = inc_ring_create(ctx, slots, &r);
  if (rc != INC_OK) return rc;
  const size_t nchunk = slots / chunk;
  r->chunk = chunk;
  hipError_t e = hipMalloc(&r->d_ring, slots * 24);
  if (e == hipSuccess) e = hipMalloc(&r->d_done, nchunk * sizeof(unsigned long long));
  if (e == hipSuccess) e = hipHostMalloc(&r->h_ready, nchunk * sizeof(unsigned long long),
                                         hipHostMallocCoherent | hipHostMallocMapped);
  if (e == hipSuccess) {
    memset(r->h_ready, 0, nchunk * sizeof(unsigned long long));
    e = hipHostGetDevicePointer((void**)&r->d_ready, r->h_ready, 0);
  }
  if (e == hipSuccess) e = hipHostMalloc(&r->h_done0, nchunk * sizeof(unsigned long long), hipHostMallocDefault);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&r->copy_stream, hipStreamNonBlocking);
  for (size_t i = 0; e == hipSuccess && i < nchunk + 2; ++i) {
    hipEvent_t ev;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) r->copied.push_back(ev);
  }
  if (e != hipSuccess) {
    inc_ring_destroy(r);
    return inc_map_hip_error(e);
  }
  *out = r;
  return INC_OK;
}

int inc_ring_destroy(inc_ring* r) {
  if (!r) return INC_ERR_ARG;
  if (r->h_rec) (void)hipHostFree(r->h_rec);
  if (r->h_ctrl) (void)hipHostFree(r->h_ctrl);
  if (r->d_dev) (void)hipFree(r->d_dev);
  if (r->d_seg) (void)hipFree(r->d_seg);
  if (r->copy_stream) (void)hipStreamSynchronize(r->copy_stream);
  for (hipEvent_t ev : r->copied) (void)hipEventDestroy(ev);
  if (r->copy_stream) (void)hipStreamDestroy(r->copy_stream);
  if (r->d_ring) (void)hipFree(r->d_ring);
  if (r->d_done) (void)hipFree(r->d_done);
  if (r->h_ready) (void)hipHostFree(r->h_ready);
  if (r->h_done0) (void)hipHostFree(r->h_done0);
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
  RingDev R{};
  const size_t S = r->slots;
  const bool dev = r->d_ring != nullptr;
  if (dev) {
    R.ev = r->d_ring;  // chunk-major: chunk q's six fields from d_ring + 6 q chunk
    R.done = r->d_done;
    R.ready = r->d_ready;
    R.chunk_mask = S / r->chunk - 1;
    R.chunk_shift = (unsigned)__builtin_ctzll(r->chunk);
  } else {
    R.tag = r->d_rec;
    R.ev = r->d_rec + S;
    R.kind = r->d_rec + 2 * S;
    R.T = r->d_rec + 3 * S;
    R.ux = r->d_rec + 4 * S;
    R.uy = r->d_rec + 5 * S;
    R.uz = r->d_rec + 6 * S;
  }
  R.mask = S - 1;
  R.head = r->d_dev;
  R.tail = r->d_ctrl;
  R.error = (unsigned int*)(r->d_ctrl + 1);
  R.spin_limit = 2000000ull;  // ~3 s without progress of the consumer
  hipEvent_t done;
  hipError_t e = hipEventCreateWithFlags(&done, hipEventDisableTiming);
  if (e != hipSuccess) return inc_map_hip_error(e);
  int rc = inc_map_hip_error(inc_upload_segment(seg, r->d_seg, st));
  if (rc == INC_OK && dev) {
    // the call's first chunk counts the slots before `start` (the previous
    // call's records) as written, so that it completes with this call's part
    const size_t nchunk = S / r->chunk;
    memset(r->h_done0, 0, nchunk * sizeof(unsigned long long));
    r->h_done0[(start / r->chunk) & (nchunk - 1)] = start & (r->chunk - 1);
    rc = inc_map_hip_error(
        hipMemcpyAsync(r->d_done, r->h_done0, nchunk * sizeof(unsigned long long), hipMemcpyHostToDevice, st));
  }
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
  unsigned long long tail = start, final_head = ~0ull, waits = 0;
  const size_t cap_out = out ? out->sec_capacity : 0;
  const unsigned long long mask = r->slots - 1;
  bool kernel_done = false;
  const double t0 = now_s();
  double t_last = t0;
  // hand `run` records, field f's first at fld[f] (ev, kind, T, ux, uy, uz;
  // in the host ring or the mirror), the batch's records k .. k + run - 1,
  // to the consumer or into the host arrays
  auto deliver = [&](const uint32_t* const* fld, unsigned long long k, size_t run) {
    if (consumer) {
      inc_ring_chunk c;
      c.first = k;
      c.n = run;
      c.event = fld[0];
      c.kind = fld[1];
      c.T = (const float*)fld[2];
      c.ux = (const float*)fld[3];
      c.uy = (const float*)fld[4];
      c.uz = (const float*)fld[5];
      consumer(&c, user);
    } else if (out && k < cap_out) {
      const size_t m = (size_t)std::min<unsigned long long>(run, cap_out - k);
      auto copy = [&, k](size_t a, size_t b) {
        const size_t n = b - a;
        if (out->sec_event) memcpy(out->sec_event + k + a, fld[0] + a, 4 * n);
        if (out->sec_T) memcpy(out->sec_T + k + a, fld[2] + a, 4 * n);
        if (out->sec_ux) memcpy(out->sec_ux + k + a, fld[3] + a, 4 * n);
        if (out->sec_uy) memcpy(out->sec_uy + k + a, fld[4] + a, 4 * n);
        if (out->sec_uz) memcpy(out->sec_uz + k + a, fld[5] + a, 4 * n);
        if (out->sec_species || out->sec_stage) {
          const uint32_t* kind = fld[1];
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
    }
  };
  // device placement: chunk copies queued on the copy stream, in order
  struct Pending {
    unsigned long long lo, hi;
    hipEvent_t ev;
  };
  std::vector<Pending> pending;  // a FIFO: [pend_head, size)
  size_t pend_head = 0, next_ev = 0;
  unsigned long long issued = start;  // records whose copy has been queued
  // the whole chunk that holds [lo, hi) goes to the mirror in one copy
  auto queue_copy = [&](unsigned long long lo, unsigned long long hi) -> hipError_t {
    const size_t off = (size_t)((lo & mask) / r->chunk) * 6 * r->chunk;
    hipError_t ce = hipMemcpyAsync(r->h_rec + off, r->d_ring + off, 24 * r->chunk, hipMemcpyDeviceToHost,
                                   r->copy_stream);
    hipEvent_t ev = r->copied[next_ev++ % r->copied.size()];
    if (ce == hipSuccess) ce = hipEventRecord(ev, r->copy_stream);
    if (ce == hipSuccess) pending.push_back({lo, hi, ev});
    return ce;
  };
  while (true) {
    bool progressed = false;
    if (!dev) {
      const uint32_t* h_tag = r->h_rec;
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
        const uint32_t* fld[6];
        for (int f = 0; f < 6; ++f) fld[f] = r->h_rec + (size_t)(f + 1) * S + j;
        deliver(fld, tail - start, run);
        tail += run;
        progressed = true;
        __atomic_store_n((unsigned long long*)tail_p, tail, __ATOMIC_RELEASE);
      }
    } else {
      // queue a copy for every chunk the device has marked complete (the
      // mirror holds the slots [tail, tail + S), as the ring does)
      const unsigned long long C = r->chunk;
      const unsigned long long nchunk = S / C;
      while (true) {
        const unsigned long long c = issued / C;
        const unsigned long long hi = (c + 1) * C;
        if (__atomic_load_n(r->h_ready + (c & (nchunk - 1)), __ATOMIC_ACQUIRE) != c + 1) break;
        e = queue_copy(issued, hi);
        if (e != hipSuccess) break;
        issued = hi;
        progressed = true;
      }
      // after the kernel: the last, incomplete chunk
      if (e == hipSuccess && kernel_done && issued < final_head && final_head - issued < C &&
          issued / C == (final_head - 1) / C) {
        e = queue_copy(issued, final_head);
        if (e == hipSuccess) issued = final_head;
      }
      if (e != hipSuccess) {
        rc = inc_map_hip_error(e);
        (void)hipStreamSynchronize(st);
        break;
      }
      // hand over the copied chunks in order
      while (pend_head < pending.size()) {
        const Pending& pc = pending[pend_head];
        const hipError_t q = hipEventQuery(pc.ev);
        if (q == hipErrorNotReady) break;
        if (q != hipSuccess) {
          e = q;
          break;
        }
        const size_t j = (size_t)(pc.lo & mask);
        const uint32_t* cb = r->h_rec + (j / r->chunk) * 6 * r->chunk + (j & (r->chunk - 1));
        const uint32_t* fld[6];
        for (int f = 0; f < 6; ++f) fld[f] = cb + (size_t)f * r->chunk;
        deliver(fld, pc.lo - start, (size_t)(pc.hi - pc.lo));
        tail = pc.hi;
        ++pend_head;
        progressed = true;
        __atomic_store_n((unsigned long long*)tail_p, tail, __ATOMIC_RELEASE);
      }
      if (e != hipSuccess) {
        rc = inc_map_hip_error(e);
        (void)hipStreamSynchronize(st);
        break;
      }
    }
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
        continue;  // the device placement queues the last chunk on the next pass
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
  if (dev) (void)hipStreamSynchronize(r->copy_stream);  // no copy outlives the call
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
  if (rc == INC_OK && !consumer && out && produced > cap_out) rc = INC_ERR_CAPACITY;
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
