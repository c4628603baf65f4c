// roctx ranges around the solver's phases (the five phase timers of the
// Results tables: setup, right-hand side, preconditioner, GMRES, Delta G).
// A profiler that records markers (rocprofv3 --marker-trace) shows them on
// the calling thread's timeline; without one each push/pop costs a call.
#pragma once
#include <rocprofiler-sdk-roctx/roctx.h>

namespace pbm {

// Pushes a range on construction and pops it on destruction (exceptions
// included), so ranges nest and always close.
struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

}  // namespace pbm
