// Diagnostics beside the boundary relation's step (not part of it).
#pragma once
#include <hip/hip_runtime.h>

namespace sbim {

constexpr int kCheckThreads = 256;
constexpr int kCheckBlocks = 1024;   // partial counts written per call

// Count the non-finite values (infinities, NaNs) of n reals, float or double,
// into partial[kCheckBlocks] (one count per work-group; the caller sums them).
hipError_t launch_count_nonfinite(bool fp64, const void *x, long long n, long long *partial,
                                  hipStream_t st);

}  // namespace sbim
