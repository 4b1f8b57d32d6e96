// roctx ranges over the library's host calls, so that a trace taken with
// `rocprofv3 --marker-trace` shows each call (its argument checks, planning,
// uploads and kernel launches) by name beside the kernels it enqueued.  The
// ranges cost a call into the roctx library each way when no tool listens.
#pragma once
#include <rocprofiler-sdk-roctx/roctx.h>

namespace cfog {

struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

}  // namespace cfog
