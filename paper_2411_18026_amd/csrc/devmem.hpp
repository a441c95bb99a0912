// Device memory helpers: an owning buffer and a grow-only workspace of named
// device buffers that keeps per-level temporaries, descriptor arrays and
// scratch alive across launches, so launchers never allocate, free or
// synchronise.
#pragma once

#include <map>
#include <string>
#include <vector>

#include "common.hpp"

namespace fds {

template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  explicit DevBuf(size_t count) { alloc(count); }
  explicit DevBuf(const std::vector<T>& h) {
    alloc(h.size());
    if (!h.empty()) FDS_HIP(hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
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
      hipError_t e = hipMalloc((void**)&p, count * sizeof(T));
      if (e != hipSuccess) {
        p = nullptr;
        n = 0;
        throw Error(3, "hipMalloc failed");
      }
    }
  }
  void release() {
    if (p) (void)hipFree(p);
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

// Named grow-only device buffers.  A buffer is reallocated only when a
// larger size is requested; the stream is synchronised first so that no
// in-flight kernel still uses the old allocation.  Uploads are stream
// ordered (hipMemcpyAsync on the workspace stream).
class Workspace {
 public:
  explicit Workspace(hipStream_t s = nullptr) : s_(s) {}
  Workspace(const Workspace&) = delete;
  Workspace& operator=(const Workspace&) = delete;
  ~Workspace() {
    for (auto& kv : bufs_)
      if (kv.second.p) (void)hipFree(kv.second.p);
  }
  void set_stream(hipStream_t s) { s_ = s; }
  hipStream_t stream() const { return s_; }

  template <typename T>
  T* get(const std::string& key, size_t count) {
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    Buf& b = bufs_[key];
    if (b.bytes < bytes) {
      if (b.p) {
        FDS_HIP(hipStreamSynchronize(s_));
        FDS_HIP(hipFree(b.p));
        b.p = nullptr;
        b.bytes = 0;
      }
      const size_t nb = std::max(bytes, b.bytes + b.bytes / 2);
      if (hipMalloc(&b.p, nb) != hipSuccess) {
        b.p = nullptr;
        throw Error(3, "hipMalloc failed for workspace buffer " + key);
      }
      b.bytes = nb;
    }
    return reinterpret_cast<T*>(b.p);
  }

  template <typename T>
  T* upload(const std::string& key, const std::vector<T>& h) {
    T* p = get<T>(key, h.size());
    if (!h.empty()) FDS_HIP(hipMemcpyAsync(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s_));
    return p;
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
  std::map<std::string, Buf> bufs_;
  hipStream_t s_;
};

}  // namespace fds
