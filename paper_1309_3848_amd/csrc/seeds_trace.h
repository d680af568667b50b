// roctx ranges around the library's host-side steps (a refinement, each level
// of its schedule, an initialisation, a warm start, a server tick), so that a
// profiler's marker trace (rocprofv3 --marker-trace) shows where a timeline's
// kernels come from. Without a profiler attached the calls do nothing.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

#include <cstdio>

namespace seeds {

// A range from construction to destruction.
class TraceRange {
  public:
    explicit TraceRange(const char *what) { roctxRangePushA(what); }
    TraceRange(const char *fmt, int a) {
        char buf[64];
        snprintf(buf, sizeof(buf), fmt, a);
        roctxRangePushA(buf);
    }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

}  // namespace seeds
