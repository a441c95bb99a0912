// Device memory helpers: an owning buffer and a grow-only workspace of named
// device buffers that keeps per-level temporaries, descriptor arrays and
// scratch alive across launches, so launchers never allocate, free or
// synchronise.
//
// Both take their memory from a process-wide cache of device blocks, so a
// factorisation after the first reuses the blocks of those before it
// instead of calling hipMalloc / hipFree (hipFree also waits for the whole
// device).  Ordering: every entry point runs its work on one stream, named
// for the calling thread by an AllocScope.  A block given back inside an
// entry point is marked with an event on that stream; it is handed out again
// at once for work on the same stream (stream order protects it) and for
// another stream only once the event has completed.  Entry points end by
// synchronising their stream, so blocks freed afterwards are idle.
// Size classes: powers of two up to 1 MiB, then multiples of 2 MiB.  The
// cache holds at most FDS_CACHE_LIMIT_MB (default 65536) MiB per device and
// gives everything back on fds_release_cache().  A caller can replace the
// cache by an allocator of its own (fds_set_allocator).
#pragma once

#include <cstring>
#include <functional>
#include <map>
#include <string>
#include <vector>

#include "common.hpp"

namespace fds {

// A caller's allocator (fds_set_allocator): when set, every device block
// comes from it and goes back to it, bypassing the cache.
struct UserAllocator {
  void* (*alloc)(size_t bytes, int device, void* stream, void* ctx) = nullptr;
  void (*free)(void* p, size_t bytes, int device, void* stream, void* ctx) = nullptr;
  void* ctx = nullptr;
};
// false (nothing changed) while blocks are live
bool set_user_allocator(const UserAllocator& u);

void set_alloc_stream(hipStream_t s, bool scoped);
hipStream_t alloc_stream();
bool alloc_scoped();
void* cache_alloc(size_t bytes, size_t* block_bytes = nullptr);
void cache_free(void* p, hipStream_t s);
// Pinned host blocks (upload staging), cached process-wide; pinned_free takes
// an idle block and the size pinned_alloc reported.
void* pinned_alloc(size_t bytes, size_t* block_bytes);
void pinned_free(void* p, size_t block_bytes);
size_t cache_bytes();
void cache_release();

// names the stream of the calling entry point for the block cache
struct AllocScope {
  hipStream_t prev;
  bool prev_scoped;
  explicit AllocScope(hipStream_t s) : prev(alloc_stream()), prev_scoped(alloc_scoped()) { set_alloc_stream(s, true); }
  ~AllocScope() { set_alloc_stream(prev, prev_scoped); }
  AllocScope(const AllocScope&) = delete;
  AllocScope& operator=(const AllocScope&) = delete;
};

template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  explicit DevBuf(size_t count) { alloc(count); }
  // inside an AllocScope: stream-ordered upload on the scope's stream (the
  // host data is staged before the call returns); otherwise synchronous
  explicit DevBuf(const std::vector<T>& h) {
    alloc(h.size());
    if (h.empty()) return;
    if (alloc_scoped())
      FDS_HIP(hipMemcpyAsync(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, alloc_stream()));
    else
      FDS_HIP(hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n) {
    o.p = nullptr;
    o.n = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      n = o.n;
      o.p = nullptr;
      o.n = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t count) {
    release();
    n = count;
    if (count) {
      try {
        p = static_cast<T*>(cache_alloc(count * sizeof(T)));
      } catch (...) {
        p = nullptr;
        n = 0;
        throw;
      }
    }
  }
  void release() {
    if (p) cache_free(p, alloc_stream());
    p = nullptr;
    n = 0;
  }
  std::vector<T> download(size_t count, hipStream_t s) const {
    std::vector<T> h(count);
    if (count) {
      FDS_HIP(hipMemcpyAsync(h.data(), p, count * sizeof(T), hipMemcpyDeviceToHost, s));
      FDS_HIP(hipStreamSynchronize(s));
    }
    return h;
  }
};

// A device array inside an arena (not owning).
template <typename T>
struct DevView {
  T* p = nullptr;
  size_t n = 0;
};

// Many small host arrays placed in one device allocation and sent with one
// copy: each allocation through a caller's allocator and each copy from
// pageable memory costs tens of microseconds, and a solve plan has a hundred
// arrays.  add() records an array and the view to point at it; finish()
// allocates the arena (256-byte aligned slices), uploads it and sets the
// views.
class ArenaBuilder {
 public:
  template <typename T>
  void add(DevView<T>& v, const std::vector<T>& h) {
    v.n = h.size();
    v.p = nullptr;   // an empty array stays null
    if (h.empty()) return;
    const size_t off = (data_.size() + 255) / 256 * 256;
    data_.resize(off + h.size() * sizeof(T));
    std::memcpy(data_.data() + off, h.data(), h.size() * sizeof(T));
    T** where = &v.p;
    fix_.push_back([where, off](unsigned char* base) { *where = reinterpret_cast<T*>(base + off); });
  }
  // inside an AllocScope: a stream-ordered upload on its stream
  void finish(DevBuf<unsigned char>& arena) {
    arena = DevBuf<unsigned char>(data_);
    for (auto& f : fix_) f(arena.p);
    data_.clear();
    fix_.clear();
  }

 private:
  std::vector<unsigned char> data_;
  std::vector<std::function<void(unsigned char*)>> fix_;
};

// Named grow-only device buffers.  A buffer is reallocated only when a
// larger size is requested; the old block goes back to the cache marked
// with the workspace stream, so kernels still queued on that stream keep
// it.  Uploads are stream ordered (hipMemcpyAsync on the workspace stream).
class Workspace {
 public:
  explicit Workspace(hipStream_t s = nullptr) : s_(s) {}
  Workspace(const Workspace&) = delete;
  Workspace& operator=(const Workspace&) = delete;
  // destroyed after the owner's last synchronisation: the blocks are idle,
  // and the stream they were used on may no longer exist
  ~Workspace() {
    for (auto& kv : bufs_)
      if (kv.second.p) cache_free(kv.second.p, alloc_stream());
    for (Pinned& b : pin_) {
      if (b.ev) {
        if (b.pending) (void)hipEventSynchronize(b.ev);
        (void)hipEventDestroy(b.ev);
      }
      pinned_free(b.p, b.bytes);
    }
  }
  void set_stream(hipStream_t s) { s_ = s; }
  hipStream_t stream() const { return s_; }

  template <typename T>
  T* get(const std::string& key, size_t count) {
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    Buf& b = bufs_[key];
    if (b.bytes < bytes) {
      const size_t nb = std::max(bytes, b.bytes + b.bytes / 2);
      if (b.p) {
        cache_free(b.p, s_);
        b.p = nullptr;
        b.bytes = 0;
      }
      AllocScope scope(s_);
      try {
        b.p = cache_alloc(nb, &b.bytes);
      } catch (const Error&) {
        b.p = nullptr;
        b.bytes = 0;
        throw Error(3, "hipMalloc failed for workspace buffer " + key);
      }
    }
    return reinterpret_cast<T*>(b.p);
  }

  template <typename T>
  T* upload(const std::string& key, const std::vector<T>& h) {
    T* p = get<T>(key, h.size());
    if (!h.empty()) FDS_HIP(hipMemcpyAsync(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s_));
    return p;
  }

  // Pinned host staging for uploads, two slots used in turn: pinned(bytes)
  // returns the next slot (waiting for the copies of its previous contents,
  // two uploads back, to complete), the caller fills it, and
  // pinned_upload(dst, bytes) enqueues one copy of it to dst on the
  // workspace stream.  A copy from pinned memory does not hold the host.
  void* pinned(size_t bytes) {
    pin_cur_ ^= 1;
    Pinned& b = pin_[pin_cur_];
    if (b.pending) {
      FDS_HIP(hipEventSynchronize(b.ev));
      b.pending = false;
    }
    if (b.bytes < bytes) {
      const size_t nb = std::max(bytes, b.bytes + b.bytes / 2);
      pinned_free(b.p, b.bytes);
      b.p = nullptr;
      b.bytes = 0;
      b.p = pinned_alloc(nb, &b.bytes);
    }
    if (!b.ev) FDS_HIP(hipEventCreateWithFlags(&b.ev, hipEventDisableTiming));
    return b.p;
  }
  void pinned_upload(void* dst, size_t bytes) {
    Pinned& b = pin_[pin_cur_];
    if (bytes) FDS_HIP(hipMemcpyAsync(dst, b.p, bytes, hipMemcpyHostToDevice, s_));
    FDS_HIP(hipEventRecord(b.ev, s_));
    b.pending = true;
  }

  size_t bytes() const {
    size_t t = 0;
    for (auto& kv : bufs_) t += kv.second.bytes;
    return t;
  }

 private:
  struct Buf {
    void* p = nullptr;
    size_t bytes = 0;
  };
  struct Pinned {
    void* p = nullptr;
    size_t bytes = 0;
    hipEvent_t ev = nullptr;
    bool pending = false;
  };
  std::map<std::string, Buf> bufs_;
  Pinned pin_[2];
  int pin_cur_ = 0;
  hipStream_t s_;
};

}  // namespace fds
