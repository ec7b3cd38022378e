// Named ranges of the library's calls on a profiler's timeline.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

namespace vg {

// A range around each call that does device work, shown by rocprofv3
// --marker-trace; with no profiler attached the two calls return at once.
struct TimelineRange {
    explicit TimelineRange(const char* name) { roctxRangePushA(name); }
    ~TimelineRange() { roctxRangePop(); }
    TimelineRange(const TimelineRange&) = delete;
    TimelineRange& operator=(const TimelineRange&) = delete;
};

}  // namespace vg
