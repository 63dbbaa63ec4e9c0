// Reuse of the scratch allocations of finished factorizations.
//
// A factorization needs gigabytes of workspace and pinned staging for its
// descriptor and index uploads; allocating and releasing them costs
// milliseconds per call (hipFree and hipHostFree also wait for the device).
// Buffers handed back here are kept, and the next request of a similar size
// on the same device takes one of them.  Only buffers that no queued work
// still uses may be handed back (the caller synchronises first).
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "common.hpp"
#include "../../include/rsrs.h"

namespace rsrs {
namespace {

struct Entry {
  void* p;
  size_t bytes;
  int dev;     // device of a device buffer (-1: pinned host memory)
};

constexpr size_t kMaxEntries = 16;
constexpr size_t kMaxCachedBytes = (size_t)32 << 30;   // device and host together

std::mutex g_mu;
std::vector<Entry>& cached() {
  static auto* v = new std::vector<Entry>();   // never destroyed: no HIP calls at exit
  return *v;
}

void free_entry(const Entry& e) {
  if (e.dev < 0) {
    (void)hipHostFree(e.p);
  } else {
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != e.dev) (void)hipSetDevice(e.dev);
    (void)hipFree(e.p);
    if (cur != e.dev) (void)hipSetDevice(cur);
  }
}

// Takes the smallest cached buffer of at least n bytes (and at most twice
// that, so a small request does not pin a large block) for device dev.
bool take(size_t n, int dev, void** p, size_t* bytes) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto& v = cached();
  size_t best = v.size();
  for (size_t i = 0; i < v.size(); ++i) {
    const Entry& e = v[i];
    if (e.dev != dev || e.bytes < n || e.bytes > 2 * n + ((size_t)1 << 20)) continue;
    if (best == v.size() || e.bytes < v[best].bytes) best = i;
  }
  if (best == v.size()) return false;
  *p = v[best].p;
  *bytes = v[best].bytes;
  v.erase(v.begin() + (std::ptrdiff_t)best);
  return true;
}

void give(void* p, size_t bytes, int dev) {
  std::vector<Entry> evict;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto& v = cached();
    v.push_back(Entry{p, bytes, dev});
    size_t total = 0;
    for (const auto& e : v) total += e.bytes;
    // the oldest entries go first
    while (!v.empty() && (v.size() > kMaxEntries || total > kMaxCachedBytes)) {
      total -= v.front().bytes;
      evict.push_back(v.front());
      v.erase(v.begin());
    }
  }
  for (const auto& e : evict) free_entry(e);
}

}  // namespace

size_t pool_cached_device_bytes(int dev) {
  std::lock_guard<std::mutex> lk(g_mu);
  size_t t = 0;
  for (const auto& e : cached())
    if (e.dev == dev) t += e.bytes;
  return t;
}

void pool_trim_device(int dev, size_t keep) {
  std::vector<Entry> evict;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto& v = cached();
    size_t t = 0;
    for (const auto& e : v)
      if (e.dev == dev) t += e.bytes;
    // the oldest buffers of this device go first
    for (size_t i = 0; i < v.size() && t > keep;) {
      if (v[i].dev == dev) {
        t -= v[i].bytes;
        evict.push_back(v[i]);
        v.erase(v.begin() + (std::ptrdiff_t)i);
      } else {
        ++i;
      }
    }
  }
  for (const auto& e : evict) free_entry(e);
}

rsrs_status pool_alloc(DevBuf& b, size_t nbytes) {
  b.release();
  if (nbytes == 0) return RSRS_OK;
  int dev = 0;
  RSRS_HIP(hipGetDevice(&dev));
  if (take(nbytes, dev, &b.p, &b.bytes)) return RSRS_OK;
  return b.alloc(nbytes);
}

rsrs_status pool_alloc(HostBuf& b, size_t nbytes) {
  b.release();
  if (nbytes == 0) return RSRS_OK;
  if (take(nbytes, -1, &b.p, &b.bytes)) return RSRS_OK;
  return b.alloc(nbytes);
}

void pool_return(DevBuf& b) {
  if (!b.p) return;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) { b.release(); return; }
  give(b.p, b.bytes, dev);
  b.p = nullptr;
  b.bytes = 0;
}

void pool_return(HostBuf& b) {
  if (!b.p) return;
  give(b.p, b.bytes, -1);
  b.p = nullptr;
  b.bytes = 0;
}

}  // namespace rsrs

extern "C" void rsrs_release_cached(void) {
  std::vector<rsrs::Entry> all;
  {
    std::lock_guard<std::mutex> lk(rsrs::g_mu);
    all.swap(rsrs::cached());
  }
  for (const auto& e : all) rsrs::free_entry(e);
}
