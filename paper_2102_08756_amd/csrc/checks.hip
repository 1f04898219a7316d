// Non-finite count of a field: a grid-stride pass, a work-group tree sum in LDS,
// one partial count per work-group (plain stores; no atomics).
#include <cstdint>
#include <mutex>

#include "checks.h"

namespace sbim {
namespace {

// Partial counts of the allocation-free count (one per work-group of the
// first pass).  Each GPU the library runs on holds its own copy until the
// process ends; host code reaches it only through the address
// hipGetSymbolAddress gives for that device (count_scratch_address).
static __device__ __align__(256) long long scratch[kCheckBlocks];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
long long *g_scratch_ptr[kMaxDevices] = {};

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

// One work-group: the kCheckBlocks partial counts summed in a fixed order.
__global__ __launch_bounds__(kCheckThreads) void sum_partials_kernel(
    const long long *__restrict__ partial, long long *__restrict__ out) {
  __shared__ long long s[kCheckThreads];
  long long c = 0;
  for (int i = threadIdx.x; i < kCheckBlocks; i += kCheckThreads) c += partial[i];
  s[threadIdx.x] = c;
  __syncthreads();
  for (int off = kCheckThreads / 2; off > 0; off >>= 1) {
    if (static_cast<int>(threadIdx.x) < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s[0];
}

}  // namespace

hipError_t count_scratch_address(int device, long long **out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = static_cast<long long *>(p);
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

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

hipError_t launch_count_nonfinite_static(bool fp64, const void *x, long long n,
                                         long long *scratch_dev, long long *count_dev,
                                         hipStream_t st) {
  const hipError_t e = launch_count_nonfinite(fp64, x, n, scratch_dev, st);
  if (e != hipSuccess) return e;
  sum_partials_kernel<<<1, kCheckThreads, 0, st>>>(scratch_dev, count_dev);
  return hipGetLastError();
}

}  // namespace sbim
