// Host-side parallel loop over independent cells (index bookkeeping of the
// factorisation: proxy disks, near sets, block requests), on a pool of
// worker threads started once per process: starting threads per loop cost
// more than the loops' work (and each new thread rebuilt its thread-local
// scratch).
#pragma once

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <cstdlib>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

namespace fds {

inline int host_threads() {
  static int n = [] {
    int t = (int)std::thread::hardware_concurrency();
    if (const char* e = std::getenv("FDS_HOST_THREADS")) t = std::atoi(e);
    return std::max(1, std::min(t, 16));
  }();
  return n;
}

// Workers wait for a job generation, run the job (which takes indices from
// a shared counter until none are left) and report back.  One job at a
// time; a loop started while another runs (another host thread, or a loop
// inside a loop) runs on its caller alone.  The pool is never destroyed:
// its threads end with the process.
class HostPool {
 public:
  static HostPool& get() {
    static HostPool* p = new HostPool(host_threads() - 1);
    return *p;
  }
  int workers() const { return (int)th_.size(); }
  // job() on the caller and every worker; false if the pool is busy
  bool run(const std::function<void()>& job) {
    std::unique_lock<std::mutex> busy(run_mu_, std::try_to_lock);
    if (!busy.owns_lock()) return false;
    {
      std::lock_guard<std::mutex> lk(mu_);
      job_ = &job;
      pending_ = (int)th_.size();
      ++gen_;
    }
    cv_.notify_all();
    job();
    std::unique_lock<std::mutex> lk(mu_);
    done_.wait(lk, [&] { return pending_ == 0; });
    job_ = nullptr;
    return true;
  }

 private:
  explicit HostPool(int n) {
    for (int t = 0; t < n; ++t) th_.emplace_back([this] { loop(); });
  }
  void loop() {
    uint64_t seen = 0;
    for (;;) {
      const std::function<void()>* job;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return gen_ != seen; });
        seen = gen_;
        job = job_;
      }
      (*job)();
      std::lock_guard<std::mutex> lk(mu_);
      if (--pending_ == 0) done_.notify_one();
    }
  }
  std::mutex run_mu_, mu_;
  std::condition_variable cv_, done_;
  const std::function<void()>* job_ = nullptr;
  uint64_t gen_ = 0;
  int pending_ = 0;
  std::vector<std::thread> th_;
};

// f(i) for i in [0, n); f must not throw.
template <typename F>
void parallel_for(int n, F&& f, int grain = 8) {
  if (n <= 0) return;
  if ((n + grain - 1) / grain <= 1 || host_threads() <= 1) {
    for (int i = 0; i < n; ++i) f(i);
    return;
  }
  // indices are taken in chunks (one shared counter, few updates of it)
  const int chunk = std::max(1, std::max(std::min(grain, n), n / (8 * host_threads())));
  std::atomic<int> next{0};
  const std::function<void()> body = [&]() {
    for (int i0; (i0 = next.fetch_add(chunk, std::memory_order_relaxed)) < n;)
      for (int i = i0, i1 = std::min(n, i0 + chunk); i < i1; ++i) f(i);
  };
  if (!HostPool::get().run(body)) body();
}

}  // namespace fds
