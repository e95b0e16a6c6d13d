// lbm_trace.h -- named ranges for profilers: each stepping and tuning entry
// point of the C ABI opens a roctx range for its duration (rocprofv3
// --marker-trace shows them beside the kernels they launch).  Without a
// profiler attached a range costs a call into the roctx library and nothing
// else.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

namespace lbm {

struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

}  // namespace lbm
