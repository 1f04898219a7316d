// C ABI of the frictional fault between the two half-spaces (Sec. 2.2
// friction laws on the boundary relation of Sec. 2.3): state, parameter checks
// and the per-step launch sequence; the arithmetic runs in fault.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "api_internal.h"

using namespace sbim_api;

// ---------------------------------------------------------------- fault

// Frictional fault between the half-space of plane 0 (above) and the one below
// it (plane 1, or the mirror image of plane 0).  Float64 state in one block of
// [kFaultRows][cells]: u (6 rows: upper side x1..x3, lower side x1..x3), v (6),
// slip (2), slip rate (2), traction (3).
struct sbim_fault {
  sbim_handle *h = nullptr;
  long long cells = 0;
  bool mirror = false;
  double zp[3] = {0, 0, 0}, zm[3] = {0, 0, 0};
  double *prm = nullptr;     // tau0 (3 rows), mu_s, mu_k, d_c
  double *st = nullptr;      // state rows as above
  void *push = nullptr;      // [P][3][cells] working precision: input of the next push
  void *func = nullptr;      // [P][3][cells] working precision: tractions without damping
  long long *bad = nullptr;  // parameter check result
  long long steps = 0;
};

namespace {

constexpr int kFaultRows = 19;
constexpr int kRowU = 0, kRowV = 6, kRowSlip = 12, kRowRate = 14, kRowTau = 16;

void free_fault(sbim_fault *f) {
  if (!f) return;
  if (f->h) (void)hipStreamSynchronize(f->h->stream);
  void *ptrs[] = {f->prm, f->st, f->push, f->func, f->bad};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  delete f;
}

int fault_clear(sbim_fault *f) {
  sbim_handle *h = f->h;
  const size_t field = static_cast<size_t>(h->cfg.nplanes) * 3 * f->cells * h->rsize;
  hipError_t e = hipMemsetAsync(f->st, 0, sizeof(double) * kFaultRows * f->cells, h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(f->push, 0, field, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "clearing the fault state");
  f->steps = 0;
  return SBIM_OK;
}

}  // namespace

extern "C" {

int sbim_fault_create(sbim_handle *h, const sbim_fault_params *prm, sbim_fault **out) {
  if (!out) return fail(h, SBIM_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!h) return fail(nullptr, SBIM_E_INVALID, "handle is NULL");
  if (!prm || !prm->tau0 || !prm->mu_s || !prm->mu_k || !prm->d_c)
    return fail(h, SBIM_E_INVALID, "fault parameters: a pointer is NULL");
  const sbim_config &c = h->cfg;
  const bool one = c.nplanes == 1 && c.plane[0].side == 1;
  const bool two = c.nplanes == 2 && c.plane[0].side == 1 && c.plane[1].side == -1;
  if (!one && !two)
    return fail(h, SBIM_E_INVALID,
                "a fault needs plane 0 with side +1 and, if present, plane 1 with side -1");
  if (h->step != 0) return fail(h, SBIM_E_STATE, "a fault starts from a handle at step 0");
  sbim_fault *f = new (std::nothrow) sbim_fault;
  if (!f) return fail(h, SBIM_E_OOM, "host allocation failed");
  f->h = h;
  f->cells = static_cast<long long>(h->n1) * h->n3;
  f->mirror = one;
  const sbim_plane &pu = c.plane[0];
  const sbim_plane &pl = one ? c.plane[0] : c.plane[1];
  const double zu[3] = {pu.mu / pu.cs, (pu.cp / pu.cs) * pu.mu / pu.cs, pu.mu / pu.cs};
  const double zl[3] = {pl.mu / pl.cs, (pl.cp / pl.cs) * pl.mu / pl.cs, pl.mu / pl.cs};
  for (int i = 0; i < 3; ++i) {
    f->zp[i] = zu[i];
    f->zm[i] = zl[i];
  }
  const size_t n = static_cast<size_t>(f->cells);
  const size_t field = static_cast<size_t>(c.nplanes) * 3 * n * h->rsize;
  hipError_t e;
  if ((e = dev_alloc(&f->prm, 6 * n)) != hipSuccess ||
      (e = dev_alloc(&f->st, kFaultRows * n)) != hipSuccess ||
      (e = dev_alloc_bytes(&f->push, field)) != hipSuccess ||
      (e = dev_alloc_bytes(&f->func, field)) != hipSuccess ||
      (e = dev_alloc(&f->bad, 1)) != hipSuccess) {
    f->h = nullptr;
    free_fault(f);
    return fail(h, SBIM_E_OOM, "fault allocation failed: %s", hipGetErrorString(e));
  }
  const size_t b = n * sizeof(double);
  if ((e = hipMemcpyAsync(f->prm, prm->tau0, 3 * b, hipMemcpyDeviceToDevice, h->stream)) ||
      (e = hipMemcpyAsync(f->prm + 3 * n, prm->mu_s, b, hipMemcpyDeviceToDevice, h->stream)) ||
      (e = hipMemcpyAsync(f->prm + 4 * n, prm->mu_k, b, hipMemcpyDeviceToDevice, h->stream)) ||
      (e = hipMemcpyAsync(f->prm + 5 * n, prm->d_c, b, hipMemcpyDeviceToDevice, h->stream)) ||
      (e = hipMemsetAsync(f->bad, 0, sizeof(long long), h->stream)) ||
      (e = sbim::launch_fault_check(f->prm, f->prm + 3 * n, f->prm + 4 * n, f->prm + 5 * n,
                                    f->cells, f->bad, h->stream))) {
    free_fault(f);
    return hip_fail(h, e, "fault parameter upload");
  }
  long long bad = 0;
  if ((e = hipMemcpyAsync(&bad, f->bad, sizeof bad, hipMemcpyDeviceToHost, h->stream)) ||
      (e = hipStreamSynchronize(h->stream))) {
    free_fault(f);
    return hip_fail(h, e, "fault parameter check");
  }
  if (bad) {
    const long long cell = bad - 1;
    free_fault(f);
    return fail(h, SBIM_E_INVALID,
                "fault parameters at cell (i1=%lld, i3=%lld): need finite values, d_c > 0, "
                "0 <= mu_k <= mu_s",
                cell / h->n3, cell % h->n3);
  }
  int rc = fault_clear(f);
  if (rc) {
    free_fault(f);
    return rc;
  }
  *out = f;
  return SBIM_OK;
}

int sbim_fault_step(sbim_fault *f, double *tau_out, double *rate_out) {
  if (!f) return fail(nullptr, SBIM_E_INVALID, "fault is NULL");
  sbim_handle *h = f->h;
  if (h->step != f->steps)
    return fail(h, SBIM_E_STATE, "the handle was stepped outside its fault (%lld vs %lld steps)",
                h->step, f->steps);
  int rc = push_fields(h, f->push, nullptr, sbim::VEL_ZERO);
  if (rc) return rc;
  hipError_t e = fft_inverse(h, h->out_spec, h->spec, f->func, nullptr);
  if (e != hipSuccess) return hip_fail(h, e, "inverse FFT of the fault tractions");
  const long long n = f->cells;
  sbim::FaultArgs a;
  a.functional = f->func;
  a.tau0 = f->prm;
  a.mu_s = f->prm + 3 * n;
  a.mu_k = f->prm + 4 * n;
  a.d_c = f->prm + 5 * n;
  a.u = f->st + kRowU * n;
  a.v = f->st + kRowV * n;
  a.slip = f->st + kRowSlip * n;
  a.rate = f->st + kRowRate * n;
  a.tau = f->st + kRowTau * n;
  a.tau_out = tau_out;
  a.rate_out = rate_out;
  a.push = f->push;
  a.cells = n;
  for (int i = 0; i < 3; ++i) {
    a.zp[i] = f->zp[i];
    a.zm[i] = f->zm[i];
  }
  a.dt = h->cfg.dt;
  a.increment = h->cfg.input_kind == SBIM_INCREMENT;
  e = sbim::launch_fault_step(h->fp64, f->mirror, a, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "fault kernel");
  f->steps += 1;
  return SBIM_OK;
}

int sbim_fault_read(const sbim_fault *f, int field, double *dst) {
  if (!f) return fail(nullptr, SBIM_E_INVALID, "fault is NULL");
  sbim_handle *h = f->h;
  if (!dst) return fail(h, SBIM_E_INVALID, "dst is NULL");
  int row, rows;
  switch (field) {
    case SBIM_FAULT_TRACTION: row = kRowTau, rows = 3; break;
    case SBIM_FAULT_SLIP_RATE: row = kRowRate, rows = 2; break;
    case SBIM_FAULT_SLIP: row = kRowSlip, rows = 2; break;
    case SBIM_FAULT_DISPLACEMENT: row = kRowU, rows = 6; break;
    case SBIM_FAULT_VELOCITY: row = kRowV, rows = 6; break;
    default: return fail(h, SBIM_E_INVALID, "unknown fault field %d", field);
  }
  hipError_t e = hipMemcpyAsync(dst, f->st + static_cast<long long>(row) * f->cells,
                                sizeof(double) * rows * f->cells, hipMemcpyDeviceToDevice,
                                h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "fault read");
  return SBIM_OK;
}

int sbim_fault_reset(sbim_fault *f) {
  if (!f) return fail(nullptr, SBIM_E_INVALID, "fault is NULL");
  int rc = sbim_reset(f->h);
  if (rc) return rc;
  return fault_clear(f);
}

int sbim_fault_destroy(sbim_fault *f) {
  free_fault(f);
  return SBIM_OK;
}

}  // extern "C"
