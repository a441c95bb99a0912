// Device memory helpers: an owning buffer and a grow-only arena for the
// per-level temporaries of the factorisation.
#pragma once

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
  void upload(const std::vector<T>& h, hipStream_t s) {
    if (h.size() > n) alloc(h.size());
    if (!h.empty()) FDS_HIP(hipMemcpyAsync(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
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

}  // namespace fds
