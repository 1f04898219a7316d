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

// Device address of this file's static partial-count array on `device` (the
// current device when called); looked up once per device and kept.
hipError_t count_scratch_address(int device, long long **out);

// The same count with the partials in that static array (`scratch`, the
// address count_scratch_address returned for the current device) and their
// sum written by a second one-work-group kernel to *count_dev (device memory).
// Nothing is allocated; concurrent calls on one device share the array.
hipError_t launch_count_nonfinite_static(bool fp64, const void *x, long long n,
                                         long long *scratch, long long *count_dev,
                                         hipStream_t st);

}  // namespace sbim
