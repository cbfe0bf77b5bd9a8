// Host-side trace ranges of the library's calls and serving iterations.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

// A roctx range over a host-side scope (visible with rocprofv3 --marker-trace).
struct RoctxRange {
    explicit RoctxRange(const char* name) { roctxRangePushA(name); }
    ~RoctxRange() { roctxRangePop(); }
    RoctxRange(const RoctxRange&) = delete;
    RoctxRange& operator=(const RoctxRange&) = delete;
};
