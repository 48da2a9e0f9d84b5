// roctx ranges around the library's calls and their passes, so that a
// profiler's marker trace (rocprofv3 --marker-trace) shows which call and
// which pass of section 2.1 / 2.2 enqueued each kernel.  The ranges are
// host-side: they cover argument checks and launches, not device time.
// RZ_ROCTX=0 in the environment turns them off (read once per process).
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

namespace rz {

bool roctx_on();

struct Range {
    bool on;
    explicit Range(const char *name) : on(roctx_on())
    {
        if (on)
            roctxRangePushA(name);
    }
    ~Range()
    {
        if (on)
            roctxRangePop();
    }
    Range(const Range &) = delete;
    Range &operator=(const Range &) = delete;
};

}  // namespace rz
