// Host helpers shared by the C-ABI translation units (sbim_api.cpp defines them):
// error reporting, device allocation, buffer sizes and the per-step launch
// sequences that the fault and the strip reuse.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "internal.h"

namespace sbim_api {

// Record a message on the handle (or, without one, for sbim_last_error(NULL)) and return `code`.
int fail(sbim_handle *h, int code, const char *fmt, ...);
// SBIM_E_DEVICE with the HIP error string.
int hip_fail(sbim_handle *h, hipError_t e, const char *what);

template <typename T>
hipError_t dev_alloc(T **p, size_t count) {
  *p = nullptr;
  if (count == 0) return hipSuccess;
  return hipMalloc(reinterpret_cast<void **>(p), count * sizeof(T));
}
hipError_t dev_alloc_bytes(void **p, size_t bytes);
hipError_t upload(void *dst, const void *src, size_t bytes, hipStream_t st);
int check_ptr(sbim_handle *h, const void *p, const char *name);

// Device bytes of one material group's buffers and of the traction spectrum.
long long ring_bytes(const sbim_handle *h, const sbim::Group &g);
long long table_bytes(const sbim_handle *h, const sbim::Group &g);
long long state_bytes_g(const sbim::Group &g);
long long pending_bytes(const sbim_handle *h, const sbim::Group &g);
long long out_spec_bytes(const sbim_handle *h);

// Forward transform of a [P][3][n1][n3] field into a spectrum buffer; inverse of a
// traction spectrum (intact) into a field, with `scratch` for the intermediate.
hipError_t fft_forward(sbim_handle *h, const void *field, void *spec);
hipError_t fft_inverse(sbim_handle *h, const void *spec, void *scratch, void *field,
                       const void *add);
// One forward step: transform u (and v for VEL_INPUT), then the step launch of
// every material group with the given rule for the damping term's velocity.
int push_fields(sbim_handle *h, const void *u, const void *v, int vel_rule);

}  // namespace sbim_api
