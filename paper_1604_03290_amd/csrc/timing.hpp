// Diagnostic timing of hot kernels (see timing.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace sph {

bool timing_on();

// Records a start event at construction and a stop event at destruction on
// the given stream, when timing is enabled (a null name records nothing).
struct TimedRegion {
    hipStream_t stream;
    hipEvent_t start = nullptr, stop = nullptr;
    TimedRegion(const char *name, hipStream_t s);
    ~TimedRegion();
    TimedRegion(const TimedRegion &) = delete;
    TimedRegion &operator=(const TimedRegion &) = delete;
};

}  // namespace sph
