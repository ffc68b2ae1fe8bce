// trace.h -- named host ranges (roctx) around the entry points and the phases
// of an update, so that a rocprofv3 trace (--marker-trace) can be cut into
// updates and phases.  The ranges mark when the host enqueues the work; the
// kernels they launch fall inside them.  Without a profiler attached a range
// costs a call into the roctx library and nothing else.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

namespace eigupd {

struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

}  // namespace eigupd
