// Event-based launch accounting (rsrs_profile_*).
#include "profile.hpp"

#include <hip/hip_runtime.h>

#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/rsrs.h"

namespace rsrs {
namespace {

struct Rec {
  hipEvent_t a, b;
  std::string tag;
  double flops, bytes;
  bool done;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
std::string g_filter;   // kernel-name prefix of the launches to record ("" = all)

hipEvent_t get_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

}  // namespace

bool prof_on() { return g_on; }

int prof_begin(hipStream_t st, const char* tag) {
  if (!g_on) return -1;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_filter.empty() && std::strncmp(tag, g_filter.c_str(), g_filter.size()) != 0) return -1;
  Rec r{get_event(), get_event(), std::string(), 0.0, 0.0, false};
  if (!r.a || !r.b) return -1;
  if (hipEventRecord(r.a, st) != hipSuccess) return -1;
  g_recs.push_back(r);
  return (int)g_recs.size() - 1;
}

int prof_begin_ext(const char* tag, hipEvent_t* start, hipEvent_t* stop) {
  *start = *stop = nullptr;
  if (!g_on) return -1;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_filter.empty() && std::strncmp(tag, g_filter.c_str(), g_filter.size()) != 0) return -1;
  Rec r{get_event(), get_event(), std::string(), 0.0, 0.0, false};
  if (!r.a || !r.b) return -1;
  g_recs.push_back(r);
  *start = r.a;
  *stop = r.b;
  return (int)g_recs.size() - 1;
}

void prof_end_ext(int slot, const char* tag, double flops, double bytes) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (slot < 0 || slot >= (int)g_recs.size()) return;
  Rec& r = g_recs[slot];
  r.tag = tag;
  r.flops = flops;
  r.bytes = bytes;
  r.done = true;
}

void prof_end(int slot, hipStream_t st, const char* tag, double flops, double bytes) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (slot < 0 || slot >= (int)g_recs.size()) return;
  Rec& r = g_recs[slot];
  (void)hipEventRecord(r.b, st);
  r.tag = tag;
  r.flops = flops;
  r.bytes = bytes;
  r.done = true;
}

}  // namespace rsrs

extern "C" {

void rsrs_profile_enable(int on) { rsrs::g_on = on != 0; }

void rsrs_profile_filter(const char* prefix) {
  std::lock_guard<std::mutex> lk(rsrs::g_mu);
  rsrs::g_filter = prefix ? prefix : "";
}

void rsrs_profile_reset(void) {
  std::lock_guard<std::mutex> lk(rsrs::g_mu);
  (void)hipDeviceSynchronize();
  for (auto& r : rsrs::g_recs) {
    rsrs::g_pool.push_back(r.a);
    rsrs::g_pool.push_back(r.b);
  }
  rsrs::g_recs.clear();
}

int rsrs_profile_read(rsrs_profile_entry* out, int max) {
  std::lock_guard<std::mutex> lk(rsrs::g_mu);
  if (hipDeviceSynchronize() != hipSuccess) return -1;
  std::map<std::string, rsrs_profile_entry> acc;
  for (auto& r : rsrs::g_recs) {
    if (!r.done) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) continue;
    auto& e = acc[r.tag];
    std::strncpy(e.tag, r.tag.c_str(), sizeof(e.tag) - 1);
    e.launches += 1;
    e.ms += ms;
    e.flops += r.flops;
    e.bytes += r.bytes;
  }
  int i = 0;
  for (auto& kv : acc) {
    if (out && i < max) out[i] = kv.second;
    ++i;
  }
  return i;
}

}  // extern "C"
