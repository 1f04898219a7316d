// Interface solve of a frictional fault between two half-spaces: one thread
// per grid cell, float64 arithmetic, fields in the [component][cell] layout of
// the library's tractions.  The inputs are the two sides' traction functionals
// (the boundary relation of Sec. 2.3 with its damping term left out); the
// interface conditions are those of Sec. 2.2 (traction continuity, Eqs. stick
// and slip chosen per cell as in Eq. stickslip, strength = normal stress x the
// slip-weakening coefficient of Eq. slipweak at the amplitude of the slip
// vector before the step), with the damping coefficients of
// Eq. SBI as the impedances that tie each side's velocity to its traction.
#include <hip/hip_runtime.h>

#include "internal.h"

// Products and sums are rounded one at a time, like a plain float64 evaluation
// of the same formulas: the stick/slip choice compares two such results.
#pragma clang fp contract(off)

namespace sbim {
namespace {

constexpr int kFaultThreads = 256;

template <typename R, bool MIRROR>
__global__ __launch_bounds__(kFaultThreads) void fault_step_kernel(FaultArgs a) {
  const long long c = static_cast<long long>(blockIdx.x) * kFaultThreads + threadIdx.x;
  if (c >= a.cells) return;
  const long long n = a.cells;
  const R *__restrict__ s = static_cast<const R *>(a.functional);

  // traction functionals of the two sides, background included
  double fp[3], fm[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double t0 = a.tau0[i * n + c];
    const double sp = static_cast<double>(s[i * n + c]);
    fp[i] = t0 + sp;
    if (MIRROR)
      fm[i] = i == 1 ? t0 - sp : t0 + sp;   // the lower side is the mirror image x2 -> -x2
    else
      fm[i] = t0 + static_cast<double>(s[(3 + i) * n + c]);
  }

  double tau[3];
  // normal: no opening, so both sides share the normal velocity
  tau[1] = (a.zm[1] * fp[1] + a.zp[1] * fm[1]) / (a.zp[1] + a.zm[1]);
  // shear: the traction that holds the slip rate at zero
  const double zs = a.zp[0] + a.zm[0];
  const double st0 = (a.zm[0] * fp[0] + a.zp[0] * fm[0]) / zs;
  const double st2 = (a.zm[0] * fp[2] + a.zp[0] * fm[2]) / zs;
  const double mag = sqrt(st0 * st0 + st2 * st2);

  const double d0 = a.slip[c], d2 = a.slip[n + c];
  const double delta = sqrt(d0 * d0 + d2 * d2);
  const double mus = a.mu_s[c], muk = a.mu_k[c], dc = a.d_c[c];
  const double mu = delta < dc ? mus - (mus - muk) * delta / dc : muk;
  const double strength = fmax(-tau[1], 0.0) * mu;
  double V0 = 0.0, V2 = 0.0;
  if (mag > strength) {
    const double sc = strength / mag;
    tau[0] = st0 * sc;
    tau[2] = st2 * sc;
    const double cz = 1.0 / a.zp[0] + 1.0 / a.zm[0];
    V0 = (st0 - tau[0]) * cz;
    V2 = (st2 - tau[2]) * cz;
  } else {
    tau[0] = st0;
    tau[2] = st2;
  }

  const double dt = a.dt;
  R *__restrict__ push = static_cast<R *>(a.push);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double vp = (fp[i] - tau[i]) / a.zp[i];
    const double vm = (tau[i] - fm[i]) / a.zm[i];
    const double up = a.u[i * n + c] + dt * vp;
    const double um = a.u[(3 + i) * n + c] + dt * vm;
    a.u[i * n + c] = up;
    a.u[(3 + i) * n + c] = um;
    a.v[i * n + c] = vp;
    a.v[(3 + i) * n + c] = vm;
    // what the next push receives: the displacement, or its increment
    push[i * n + c] = static_cast<R>(a.increment ? dt * vp : up);
    if (!MIRROR) push[(3 + i) * n + c] = static_cast<R>(a.increment ? dt * vm : um);
    a.tau[i * n + c] = tau[i];
    if (a.tau_out) a.tau_out[i * n + c] = tau[i];
  }
  a.slip[c] = d0 + dt * V0;
  a.slip[n + c] = d2 + dt * V2;
  a.rate[c] = V0;
  a.rate[n + c] = V2;
  if (a.rate_out) {
    a.rate_out[c] = V0;
    a.rate_out[n + c] = V2;
  }
}

// Flags parameter cells outside the law's domain: d_c <= 0, mu_k < 0,
// mu_s < mu_k, or any non-finite value.  Every offending thread stores its
// own cell index + 1 (plain stores; any one of them is a valid report).
__global__ __launch_bounds__(kFaultThreads) void fault_check_kernel(const double *__restrict__ tau0,
                                                                   const double *__restrict__ mu_s,
                                                                   const double *__restrict__ mu_k,
                                                                   const double *__restrict__ d_c,
                                                                   long long n,
                                                                   long long *__restrict__ bad) {
  const long long c = static_cast<long long>(blockIdx.x) * kFaultThreads + threadIdx.x;
  if (c >= n) return;
  const double s = mu_s[c], k = mu_k[c], d = d_c[c];
  bool ok = isfinite(s) && isfinite(k) && isfinite(d) && d > 0.0 && k >= 0.0 && s >= k;
#pragma unroll
  for (int i = 0; i < 3; ++i) ok = ok && isfinite(tau0[i * n + c]);
  if (!ok) *bad = c + 1;
}

}  // namespace

hipError_t launch_fault_step(bool fp64, bool mirror, const FaultArgs &a, hipStream_t st) {
  if (a.cells <= 0) return hipSuccess;
  const unsigned blocks = static_cast<unsigned>((a.cells + kFaultThreads - 1) / kFaultThreads);
  if (fp64) {
    if (mirror)
      fault_step_kernel<double, true><<<blocks, kFaultThreads, 0, st>>>(a);
    else
      fault_step_kernel<double, false><<<blocks, kFaultThreads, 0, st>>>(a);
  } else {
    if (mirror)
      fault_step_kernel<float, true><<<blocks, kFaultThreads, 0, st>>>(a);
    else
      fault_step_kernel<float, false><<<blocks, kFaultThreads, 0, st>>>(a);
  }
  return hipGetLastError();
}

hipError_t launch_fault_check(const double *tau0, const double *mu_s, const double *mu_k,
                              const double *d_c, long long cells, long long *bad, hipStream_t st) {
  if (cells <= 0) return hipSuccess;
  const unsigned blocks = static_cast<unsigned>((cells + kFaultThreads - 1) / kFaultThreads);
  fault_check_kernel<<<blocks, kFaultThreads, 0, st>>>(tau0, mu_s, mu_k, d_c, cells, bad);
  return hipGetLastError();
}

}  // namespace sbim
