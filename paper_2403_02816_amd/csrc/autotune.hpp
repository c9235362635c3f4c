// Plan-time selection of kernel tile shapes by measurement.
#pragma once

#include <hip/hip_runtime.h>

#include <functional>
#include <string>

namespace cgl {

// Returns the candidate in [0, ncand) whose launch is fastest: every
// candidate is launched once to warm up, then `reps` times between two events
// on stream s, and the smallest mean wins.  Results are cached per key for the
// process and, when the environment variable CGL_AUTOTUNE_CACHE names a file,
// in that file ("key choice" lines), so later processes skip the timing.
// A candidate whose launch fails is never chosen; if all fail, returns 0.
// weight (optional, ncand entries) multiplies each measured time before the
// comparison: a known cost that the isolated launch does not show.
int autotune_pick(const std::string& key, int ncand,
                  const std::function<hipError_t(int)>& launch, hipStream_t s, int reps,
                  const double* weight = nullptr);

// Short identifier of the current device (its gfx architecture name).
std::string device_tag();

}  // namespace cgl
