// Non-finite count of a field: a grid-stride pass, a work-group tree sum in LDS,
// one partial count per work-group (plain stores; no atomics).
#include <cstdint>

#include "checks.h"

namespace sbim {
namespace {

// Exponent bits all set: an infinity or a NaN (independent of floating-point flags).
__device__ __forceinline__ int nonfinite(float x) {
  return (__float_as_uint(x) & 0x7f800000u) == 0x7f800000u;
}
__device__ __forceinline__ int nonfinite(double x) {
  const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(x));
  return (b & 0x7ff0000000000000ull) == 0x7ff0000000000000ull;
}

template <typename R>
__global__ __launch_bounds__(kCheckThreads) void count_nonfinite_kernel(
    const R *__restrict__ x, long long n, long long *__restrict__ partial) {
  __shared__ long long s[kCheckThreads];
  long long c = 0;
  const long long stride = static_cast<long long>(gridDim.x) * kCheckThreads;
  for (long long i = static_cast<long long>(blockIdx.x) * kCheckThreads + threadIdx.x; i < n;
       i += stride)
    c += nonfinite(x[i]);
  s[threadIdx.x] = c;
  __syncthreads();
  for (int off = kCheckThreads / 2; off > 0; off >>= 1) {
    if (static_cast<int>(threadIdx.x) < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = s[0];
}

}  // namespace

hipError_t launch_count_nonfinite(bool fp64, const void *x, long long n, long long *partial,
                                  hipStream_t st) {
  if (fp64)
    count_nonfinite_kernel<double><<<kCheckBlocks, kCheckThreads, 0, st>>>(
        static_cast<const double *>(x), n, partial);
  else
    count_nonfinite_kernel<float><<<kCheckBlocks, kCheckThreads, 0, st>>>(
        static_cast<const float *>(x), n, partial);
  return hipGetLastError();
}

}  // namespace sbim
