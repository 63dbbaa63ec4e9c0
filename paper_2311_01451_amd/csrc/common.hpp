// Shared host-side helpers of the HIP library: status propagation and device buffers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <utility>
#include <vector>

#include "../../include/rsrs.h"

namespace rsrs {

void set_error(const std::string& msg);
void set_required_s(int64_t s);

struct Status {
  rsrs_status code = RSRS_OK;
  bool ok() const { return code == RSRS_OK; }
};

#define RSRS_HIP(expr)                                                          \
  do {                                                                          \
    hipError_t e_ = (expr);                                                     \
    if (e_ != hipSuccess) {                                                     \
      ::rsrs::set_error(std::string("HIP error ") + hipGetErrorString(e_) +     \
                        " at " __FILE__ ":" + std::to_string(__LINE__) + ": " #expr); \
      return e_ == hipErrorOutOfMemory ? RSRS_E_NOMEM : RSRS_E_HIP;             \
    }                                                                           \
  } while (0)

#define RSRS_TRY(...)                      \
  do {                                     \
    rsrs_status s_ = (__VA_ARGS__);        \
    if (s_ != RSRS_OK) return s_;          \
  } while (0)

// Owning device allocation.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; bytes = o.bytes; o.p = nullptr; o.bytes = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  rsrs_status alloc(size_t nbytes) {
    if (nbytes <= bytes && p) return RSRS_OK;
    release();
    if (nbytes == 0) return RSRS_OK;
    hipError_t e = hipMalloc(&p, nbytes);
    if (e != hipSuccess) {
      p = nullptr;
      set_error(std::string("hipMalloc of ") + std::to_string(nbytes) + " bytes failed: " +
                hipGetErrorString(e));
      return RSRS_E_NOMEM;
    }
    bytes = nbytes;
    return RSRS_OK;
  }
  template <class T> T* as() const { return reinterpret_cast<T*>(p); }
};

// Pinned host staging buffer (allocated, never registered).
struct HostBuf {
  void* p = nullptr;
  size_t bytes = 0;
  HostBuf() = default;
  HostBuf(const HostBuf&) = delete;
  HostBuf& operator=(const HostBuf&) = delete;
  ~HostBuf() { release(); }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
  }
  rsrs_status alloc(size_t nbytes) {
    if (nbytes <= bytes && p) return RSRS_OK;
    release();
    if (nbytes == 0) return RSRS_OK;
    hipError_t e = hipHostMalloc(&p, nbytes, hipHostMallocDefault);
    if (e != hipSuccess) {
      p = nullptr;
      set_error(std::string("hipHostMalloc failed: ") + hipGetErrorString(e));
      return RSRS_E_NOMEM;
    }
    bytes = nbytes;
    return RSRS_OK;
  }
  template <class T> T* as() const { return reinterpret_cast<T*>(p); }
};

// Scratch reuse across factorizations (pool.hip): pool_alloc takes a kept
// buffer of a similar size on the current device, or allocates;
// pool_return keeps the buffer for a later call.  A buffer may be returned
// only once no queued work uses it.
rsrs_status pool_alloc(DevBuf& b, size_t nbytes);
rsrs_status pool_alloc(HostBuf& b, size_t nbytes);
void pool_return(DevBuf& b);
void pool_return(HostBuf& b);
// Device bytes the pool keeps for device `dev`, and a trim of them (oldest
// first) down to at most `keep` bytes.
size_t pool_cached_device_bytes(int dev);
void pool_trim_device(int dev, size_t keep);

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

}  // namespace rsrs
