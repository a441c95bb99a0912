// Host-side parallel loop over independent cells (index bookkeeping of the
// factorisation: proxy disks, near sets, block requests).
#pragma once

#include <algorithm>
#include <atomic>
#include <cstdlib>
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

// f(i) for i in [0, n); f must not throw.
template <typename F>
void parallel_for(int n, F&& f, int grain = 8) {
  const int nt = std::min(host_threads(), (n + grain - 1) / grain);
  if (nt <= 1) {
    for (int i = 0; i < n; ++i) f(i);
    return;
  }
  std::atomic<int> next{0};
  auto body = [&]() {
    for (int i; (i = next.fetch_add(1, std::memory_order_relaxed)) < n;) f(i);
  };
  std::vector<std::thread> th;
  th.reserve(nt - 1);
  for (int t = 1; t < nt; ++t) th.emplace_back(body);
  body();
  for (auto& x : th) x.join();
}

}  // namespace fds
