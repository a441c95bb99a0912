// Process-wide cache of device blocks (see devmem.hpp).
#include <algorithm>
#include <cstdlib>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "devmem.hpp"

namespace fds {

namespace {

thread_local hipStream_t t_alloc_stream = nullptr;
thread_local bool t_alloc_scoped = false;

// block sizes: powers of two up to 1 MiB, then multiples of 2 MiB
size_t round_block(size_t bytes) {
  if (bytes <= (1u << 20)) {
    size_t b = 512;
    while (b < bytes) b <<= 1;
    return b;
  }
  const size_t g = size_t(2) << 20;
  return (bytes + g - 1) / g * g;
}

struct FreeBlock {
  void* p;
  hipStream_t s;      // stream of the last owner
  hipEvent_t ev;      // recorded on s when the block was returned
};

struct DeviceCache {
  std::multimap<size_t, FreeBlock> free;   // by block size
  size_t cached = 0;                       // bytes held in ``free``
};

class BlockCache {
 public:
  static BlockCache& get() {
    static BlockCache* c = new BlockCache();   // never destroyed: frees at exit would race the runtime's teardown
    return *c;
  }

  void* alloc(size_t bytes, hipStream_t s, size_t* got) {
    int dev = 0;
    FDS_HIP(hipGetDevice(&dev));
    UserAllocator u;
    {
      std::lock_guard<std::mutex> g(mu_);
      u = user_;
    }
    if (u.alloc) {   // the caller's allocator (called outside the lock): no caching
      const size_t b = std::max<size_t>(bytes, 1);
      void* p = u.alloc(b, dev, (void*)s, u.ctx);
      if (!p) throw Error(3, "the allocator set by fds_set_allocator returned NULL");
      std::lock_guard<std::mutex> g(mu_);
      live_[p] = Live{b, dev, true, s};
      *got = b;
      return p;
    }
    const size_t b = round_block(std::max<size_t>(bytes, 1));
    {
      std::lock_guard<std::mutex> g(mu_);
      DeviceCache& dc = devs_[dev];
      // exact size class; a block freed on another stream only once its event has completed
      auto range = dc.free.equal_range(b);
      auto pick = dc.free.end();
      for (auto it = range.first; it != range.second; ++it) {
        if (it->second.s == s) {
          pick = it;
          break;
        }
        if (pick == dc.free.end() && hipEventQuery(it->second.ev) == hipSuccess) pick = it;
      }
      if (pick != dc.free.end()) {
        void* p = pick->second.p;
        events_.push_back(pick->second.ev);
        dc.free.erase(pick);
        dc.cached -= b;
        live_[p] = Live{b, dev, false, s};
        *got = b;
        return p;
      }
    }
    void* p = nullptr;
    if (hipMalloc(&p, b) != hipSuccess) {
      (void)hipGetLastError();
      release_device(dev);
      if (hipMalloc(&p, b) != hipSuccess) {
        (void)hipGetLastError();
        throw Error(3, "hipMalloc failed");
      }
    }
    std::lock_guard<std::mutex> g(mu_);
    live_[p] = Live{b, dev, false, s};
    *got = b;
    return p;
  }

  void free(void* p, hipStream_t s) {
    if (!p) return;
    std::unique_lock<std::mutex> g(mu_);
    auto it = live_.find(p);
    if (it == live_.end()) {
      (void)hipFree(p);
      return;
    }
    const Live l = it->second;
    live_.erase(it);
    if (l.user) {
      // a stream-ordered allocator may hand the block out again for work on
      // the stream it was allocated for; work queued on another stream must
      // have finished first
      const UserAllocator u = user_;
      g.unlock();
      if (s != l.stream) (void)hipStreamSynchronize(s);
      u.free(p, l.bytes, l.dev, (void*)l.stream, u.ctx);
      return;
    }
    hipEvent_t ev = nullptr;
    if (!events_.empty()) {
      ev = events_.back();
      events_.pop_back();
    } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
      ev = nullptr;
    }
    if (!ev || hipEventRecord(ev, s) != hipSuccess) {
      // no way to order a later reuse: give the block back to the runtime
      (void)hipGetLastError();
      if (ev) events_.push_back(ev);
      (void)hipFree(p);
      return;
    }
    DeviceCache& dc = devs_[l.dev];
    dc.free.emplace(l.bytes, FreeBlock{p, s, ev});
    dc.cached += l.bytes;
    if (dc.cached > limit()) trim_locked(dc, limit() / 2);
  }

  size_t cached_bytes() {
    std::lock_guard<std::mutex> g(mu_);
    size_t t = 0;
    for (auto& kv : devs_) t += kv.second.cached;
    return t;
  }

  void release_all() {
    std::lock_guard<std::mutex> g(mu_);
    for (auto& kv : devs_) trim_locked(kv.second, 0);
  }

  // false while any block is live (it must go back to the allocator that made it)
  bool set_user(const UserAllocator& u) {
    std::lock_guard<std::mutex> g(mu_);
    if (!live_.empty()) return false;
    for (auto& kv : devs_) trim_locked(kv.second, 0);
    user_ = u;
    return true;
  }

 private:
  struct Live {
    size_t bytes;
    int dev;
    bool user;          // made by the caller's allocator
    hipStream_t stream; // stream named at allocation
  };

  void release_device(int dev) {
    std::lock_guard<std::mutex> g(mu_);
    trim_locked(devs_[dev], 0);
  }

  // hipFree waits for the device, so blocks still in use by queued work
  // are safe to hand back; the largest go first.
  void trim_locked(DeviceCache& dc, size_t target) {
    while (dc.cached > target && !dc.free.empty()) {
      auto it = std::prev(dc.free.end());
      (void)hipFree(it->second.p);
      events_.push_back(it->second.ev);
      dc.cached -= it->first;
      dc.free.erase(it);
    }
  }

  static size_t limit() {
    static const size_t lim = [] {
      const char* e = std::getenv("FDS_CACHE_LIMIT_MB");
      const long long mb = e ? std::atoll(e) : 65536;   // 64 GiB of the 288 GB per GPU
      return (size_t)std::max(0LL, mb) << 20;
    }();
    return lim;
  }

  std::mutex mu_;
  std::map<int, DeviceCache> devs_;
  std::unordered_map<void*, Live> live_;
  std::vector<hipEvent_t> events_;
  UserAllocator user_{};
};

// Pinned host blocks of the workspaces' upload staging, kept across
// factorisations: pinning pages (hipHostMalloc) costs milliseconds for the
// multi-megabyte assembly tables, and hipHostFree waits for the device, so
// each factorisation after the first reuses the blocks of earlier ones.
class PinnedCache {
 public:
  static PinnedCache& get() {
    static PinnedCache* c = new PinnedCache();   // never destroyed (runtime teardown order)
    return *c;
  }

  void* alloc(size_t bytes, size_t* got) {
    const size_t g = size_t(1) << 20;
    const size_t b = (std::max<size_t>(bytes, 1) + g - 1) / g * g;
    {
      std::lock_guard<std::mutex> lk(mu_);
      // the smallest cached block that holds the request, if not far larger
      auto it = free_.lower_bound(b);
      if (it != free_.end() && it->first <= 4 * b) {
        void* p = it->second;
        *got = it->first;
        cached_ -= it->first;
        free_.erase(it);
        return p;
      }
    }
    void* p = nullptr;
    FDS_HIP(hipHostMalloc(&p, b, hipHostMallocDefault));
    *got = b;
    return p;
  }

  // the block must be idle (no copy from it still queued)
  void free(void* p, size_t bytes) {
    if (!p) return;
    std::unique_lock<std::mutex> lk(mu_);
    if (cached_ + bytes > kLimit) {
      lk.unlock();
      (void)hipHostFree(p);
      return;
    }
    free_.emplace(bytes, p);
    cached_ += bytes;
  }

  void release_all() {
    std::lock_guard<std::mutex> lk(mu_);
    for (auto& kv : free_) (void)hipHostFree(kv.second);
    free_.clear();
    cached_ = 0;
  }

 private:
  static constexpr size_t kLimit = size_t(512) << 20;
  std::mutex mu_;
  std::multimap<size_t, void*> free_;   // by block size
  size_t cached_ = 0;
};

}  // namespace

void* pinned_alloc(size_t bytes, size_t* block_bytes) { return PinnedCache::get().alloc(bytes, block_bytes); }

void pinned_free(void* p, size_t block_bytes) { PinnedCache::get().free(p, block_bytes); }

void set_alloc_stream(hipStream_t s, bool scoped) {
  t_alloc_stream = s;
  t_alloc_scoped = scoped;
}
hipStream_t alloc_stream() { return t_alloc_stream; }
bool alloc_scoped() { return t_alloc_scoped; }

void* cache_alloc(size_t bytes, size_t* block_bytes) {
  size_t got = 0;
  void* p = BlockCache::get().alloc(bytes, t_alloc_stream, &got);
  if (block_bytes) *block_bytes = got;
  return p;
}

void cache_free(void* p, hipStream_t s) { BlockCache::get().free(p, s); }

size_t cache_bytes() { return BlockCache::get().cached_bytes(); }

void cache_release() {
  BlockCache::get().release_all();
  PinnedCache::get().release_all();
}

bool set_user_allocator(const UserAllocator& u) { return BlockCache::get().set_user(u); }

}  // namespace fds
