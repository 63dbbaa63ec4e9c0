// Launch accounting for measurement (see rsrs_profile_* in include/rsrs.h).
#pragma once
#include <hip/hip_runtime.h>

#include <string>

namespace rsrs {

bool prof_on();
// Returns an opaque slot (or -1 when profiling is off); call prof_end after the launch.
int prof_begin(hipStream_t st, const char* tag);
void prof_end(int slot, hipStream_t st, const char* tag, double flops, double bytes);
// For launches that time themselves (hipExtLaunchKernel with start / stop
// events, no separate event records): the events to pass to the launch, or
// -1 (events null) when the tag is not recorded; prof_end_ext after it.
int prof_begin_ext(const char* tag, hipEvent_t* start, hipEvent_t* stop);
void prof_end_ext(int slot, const char* tag, double flops, double bytes);

// RAII helper around one launch.
struct ProfScope {
  int slot;
  hipStream_t st;
  const char* tag;
  double flops, bytes;
  ProfScope(hipStream_t s, const char* t, double f = 0.0, double b = 0.0)
      : slot(prof_begin(s, t)), st(s), tag(t), flops(f), bytes(b) {}
  ~ProfScope() { if (slot >= 0) prof_end(slot, st, tag, flops, bytes); }
};

}  // namespace rsrs
