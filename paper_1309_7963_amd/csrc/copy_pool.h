// copy_pool.h — host worker pool that runs the chunks of one parallel copy
// together with the calling thread (used by the ring drain, ring.hip).  Plain
// C++ (no HIP), so it can also be built alone for a host-side race test.
#pragma once

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

namespace incdev {

// run(n, fn) calls fn(c) once for every chunk c in [0, n), on the workers and
// the calling thread, and returns when all chunks are done.  A chunk is
// claimed by a compare-and-swap on one 64-bit word holding the run's
// generation (high half) and the next chunk (low half), so a worker that wakes
// late for an earlier run can neither take a chunk of a later run under the
// earlier run's bounds nor use the earlier run's (by then destroyed) function:
// its claim fails once the generation has moved.
class CopyPool {
 public:
  explicit CopyPool(int workers) {
    for (int i = 0; i < workers; ++i) th_.emplace_back([this] { loop(); });
  }
  ~CopyPool() {
    {
      std::lock_guard<std::mutex> g(m_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto& t : th_) t.join();
  }
  CopyPool(const CopyPool&) = delete;
  CopyPool& operator=(const CopyPool&) = delete;

  void run(int n, const std::function<void(int)>& fn) {
    if (n <= 0) return;
    Job job;
    {
      std::lock_guard<std::mutex> g(m_);
      ++gen_;
      job = {gen_, n, &fn};
      job_ = job;
      left_ = n;
      next_.store((uint64_t)gen_ << 32);
    }
    cv_.notify_all();
    work(job);
    std::unique_lock<std::mutex> l(m_);
    done_cv_.wait(l, [this] { return left_ == 0; });
  }

 private:
  struct Job {
    uint32_t gen;
    int n;
    const std::function<void(int)>* fn;
  };

  // Claim and run chunks of `job` until none is left or a newer run began.
  void work(const Job& job) {
    int done = 0;
    uint64_t v = next_.load();
    for (;;) {
      if ((uint32_t)(v >> 32) != job.gen || (int)(uint32_t)v >= job.n) break;
      if (!next_.compare_exchange_weak(v, v + 1)) continue;  // v reloaded
      (*job.fn)((int)(uint32_t)v);
      ++done;
      v = next_.load();
    }
    if (done) {
      // a claimed chunk keeps its run from returning, so `left_` is still this run's
      std::lock_guard<std::mutex> g(m_);
      left_ -= done;
      if (left_ == 0) done_cv_.notify_all();
    }
  }
  void loop() {
    uint32_t seen = 0;
    std::unique_lock<std::mutex> l(m_);
    for (;;) {
      cv_.wait(l, [&] { return stop_ || gen_ != seen; });
      if (stop_) return;
      seen = gen_;
      const Job job = job_;
      l.unlock();
      work(job);
      l.lock();
    }
  }

  std::vector<std::thread> th_;
  std::mutex m_;
  std::condition_variable cv_, done_cv_;
  Job job_ = {0, 0, nullptr};
  int left_ = 0;
  std::atomic<uint64_t> next_{0};
  uint32_t gen_ = 0;
  bool stop_ = false;
};

}  // namespace incdev
