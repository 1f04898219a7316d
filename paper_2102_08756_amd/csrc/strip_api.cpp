// C ABI of the hybrid finite-element strip (Sec. 2.2 and 2.4): host assembly
// of the element stiffness stencil, device state and the per-step launch
// sequence; the arithmetic of a step runs in strip.hip.
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

// ---------------------------------------------------------------- strip

// Finite-element strip of the hybrid scheme on the fault, closed at S+ (and
// S-) by the handle's planes.  Float64 node state [12][nodes], 3 components
// each: two displacement buffers (u_{t+1} read by the next step's stencil, the
// other one written with u_{t+2}; `cur` names the first), the half-step velocity
// and the velocity v_{t+1}; fault outputs [8][cells] (traction 3, slip rate 2,
// slip 2, sliding 1).  Each step ends with the predictor of the next one, so
// the push inputs of S+ (S-) are ready when the step begins.
struct sbim_strip {
  sbim_handle *h = nullptr;
  int n2 = 0;                 // index of the top storage node layer (S+)
  int fault_lo = -1;          // two-sided: storage layer of the lower fault copy
  long long cells = 0, nodes = 0;
  double *node = nullptr;     // u (two buffers), half-step velocity, velocity
  int cur = 0;                // displacement buffer the next step's stencil reads
  double dt_pred = 0;         // step size of the prediction held for the next step
  double *cell = nullptr;     // fault outputs
  double *prm = nullptr;      // tau0 (3), mu_s, mu_k, d_c
  double *stencil = nullptr;  // [n2+1][27][9]
  double *mass = nullptr;     // [n2+1]
  void *push_u = nullptr, *push_v = nullptr, *tau_sbi = nullptr;  // [P][3][cells] working precision
  double *r_fault = nullptr;  // two-sided: [2][3][cells]
  long long *bad = nullptr;
  long long steps = 0;
};

namespace {

constexpr int kCellTau = 0, kCellRate = 3, kCellSlip = 5, kCellSliding = 7, kCellRows = 8;

// Stiffness of a cube of side h with Lame constants (lam, mu): trilinear shape
// functions, 2x2x2 Gauss points; dofs node-major (corner a = a1 + 2 a2 + 4 a3),
// then x1, x2, x3.
void cube_stiffness(double h, double lam, double mu, std::vector<double> &K) {
  K.assign(24 * 24, 0.0);
  const double g = 1.0 / std::sqrt(3.0);
  const double pts[2] = {-g, g};
  double D[6][6] = {};
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) D[i][j] = lam;
    D[i][i] = lam + 2.0 * mu;
    D[3 + i][3 + i] = mu;
  }
  const double jac = (h / 2.0) * (h / 2.0) * (h / 2.0);
  for (double p0 : pts)
    for (double p1 : pts)
      for (double p2 : pts) {
        const double p[3] = {p0, p1, p2};
        double B[6][24] = {};
        for (int a = 0; a < 8; ++a) {
          double sgn[3], d[3];
          for (int k = 0; k < 3; ++k) sgn[k] = ((a >> k) & 1) ? 1.0 : -1.0;
          for (int k = 0; k < 3; ++k) {
            double prod = sgn[k] / 8.0;
            for (int m = 0; m < 3; ++m)
              if (m != k) prod *= 1.0 + sgn[m] * p[m];
            d[k] = prod * (2.0 / h);
          }
          // Voigt order (11, 22, 33, 23, 13, 12), engineering shear strains
          B[0][3 * a] = d[0];
          B[1][3 * a + 1] = d[1];
          B[2][3 * a + 2] = d[2];
          B[3][3 * a + 1] = d[2];
          B[3][3 * a + 2] = d[1];
          B[4][3 * a] = d[2];
          B[4][3 * a + 2] = d[0];
          B[5][3 * a] = d[1];
          B[5][3 * a + 1] = d[0];
        }
        for (int i = 0; i < 24; ++i)
          for (int j = 0; j < 24; ++j) {
            double acc = 0.0;
            for (int r = 0; r < 6; ++r) {
              double db = 0.0;
              for (int c = 0; c < 6; ++c) db += D[r][c] * B[c][j];
              acc += B[r][i] * db;
            }
            K[i * 24 + j] += acc * jac;
          }
      }
}

void free_strip(sbim_strip *s) {
  if (!s) return;
  if (s->h) (void)hipStreamSynchronize(s->h->stream);
  void *ptrs[] = {s->node, s->cell, s->prm, s->stencil, s->mass, s->push_u, s->push_v,
                  s->tau_sbi, s->r_fault, s->bad};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  delete s;
}

int strip_clear(sbim_strip *s) {
  sbim_handle *h = s->h;
  // at rest: u_1 = 0 and v_{1/2} = 0, so the first push inputs are zero too
  const size_t fb = static_cast<size_t>(h->cfg.nplanes) * 3 * s->cells * h->rsize;
  hipError_t e = hipMemsetAsync(s->node, 0, sizeof(double) * 12 * s->nodes, h->stream);
  if (e == hipSuccess)
    e = hipMemsetAsync(s->cell, 0, sizeof(double) * kCellRows * s->cells, h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(s->push_u, 0, fb, h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(s->push_v, 0, fb, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "clearing the strip state");
  s->cur = 0;
  s->dt_pred = h->cfg.dt;
  s->steps = 0;
  return SBIM_OK;
}

}  // namespace

extern "C" {

int sbim_strip_create(sbim_handle *h, const sbim_strip_config *sc, const sbim_fault_params *prm,
                      sbim_strip **out) {
  if (!out) return fail(h, SBIM_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!h) return fail(nullptr, SBIM_E_INVALID, "handle is NULL");
  if (!sc || !sc->rho || !sc->cp || !sc->cs)
    return fail(h, SBIM_E_INVALID, "strip configuration: a pointer is NULL");
  if (!prm || !prm->tau0 || !prm->mu_s || !prm->mu_k || !prm->d_c)
    return fail(h, SBIM_E_INVALID, "fault parameters: a pointer is NULL");
  const sbim_config &c = h->cfg;
  const int La = sc->layers, Lb = sc->layers_below;
  if (Lb == 0 && (c.nplanes != 1 || c.plane[0].side != 1))
    return fail(h, SBIM_E_INVALID, "a strip needs a handle with one plane of side +1 (S+)");
  if (Lb > 0 && (c.nplanes != 2 || c.plane[0].side != 1 || c.plane[1].side != -1))
    return fail(h, SBIM_E_INVALID,
                "a two-sided strip needs a handle with planes of sides +1 (S+) and -1 (S-)");
  if (c.dx1 != c.dx3)
    return fail(h, SBIM_E_INVALID, "strip elements are cubes: dx1 must equal dx3");
  if (La < 1 || La > 4096 || Lb < 0 || Lb > 4096)
    return fail(h, SBIM_E_INVALID, "strip layers must be in [1, 4096] above and [0, 4096] below, "
                "got %d and %d", La, Lb);
  if (Lb > 0 && (!sc->rho_below || !sc->cp_below || !sc->cs_below))
    return fail(h, SBIM_E_INVALID, "strip configuration: a pointer of the lower side is NULL");
  for (int side = 0; side < 2; ++side) {
    const int L = side ? Lb : La;
    const double *R = side ? sc->rho_below : sc->rho, *P = side ? sc->cp_below : sc->cp,
                 *Q = side ? sc->cs_below : sc->cs;
    for (int l = 0; l < L; ++l) {
      const double r = R[l], p = P[l], q = Q[l];
      if (!(r > 0 && q > 0 && p > q * std::sqrt(4.0 / 3.0)) || !std::isfinite(r) ||
          !std::isfinite(p))
        return fail(h, SBIM_E_INVALID,
                    "strip layer %d%s: need rho > 0, cs > 0, cp > cs sqrt(4/3) (got %g, %g, %g)",
                    l, side ? " below the fault" : "", r, p, q);
    }
  }
  if (h->step != 0) return fail(h, SBIM_E_STATE, "a strip starts from a handle at step 0");
  sbim_strip *s = new (std::nothrow) sbim_strip;
  if (!s) return fail(h, SBIM_E_OOM, "host allocation failed");
  s->h = h;
  // storage node layers: [0, Lb] the block below the fault (S- first; empty when
  // one-sided), then the block above it from the fault to S+
  const int base = Lb > 0 ? Lb + 1 : 0;
  s->fault_lo = Lb > 0 ? Lb : -1;
  s->n2 = base + La;
  s->cells = static_cast<long long>(h->n1) * h->n3;
  s->nodes = (s->n2 + 1LL) * s->cells;
  const double hx = c.dx1;
  // element layers in storage order: (first storage node layer, material)
  struct ELayer { int j0; double rho, cp, cs; };
  std::vector<ELayer> el;
  for (int l = 0; l < Lb; ++l) {      // listed from the fault outwards: storage bottom-up
    const int k = Lb - 1 - l;
    el.push_back({l, sc->rho_below[k], sc->cp_below[k], sc->cs_below[k]});
  }
  for (int l = 0; l < La; ++l) el.push_back({base + l, sc->rho[l], sc->cp[l], sc->cs[l]});
  // stencil and lumped mass per node layer (no element crosses the split fault)
  std::vector<double> st(static_cast<size_t>(s->n2 + 1) * 27 * 9, 0.0), ms(s->n2 + 1, 0.0);
  std::vector<double> K;
  for (const ELayer &E : el) {
    const double rho = E.rho;
    const double mu = rho * E.cs * E.cs;
    const double lam = rho * E.cp * E.cp - 2.0 * mu;
    cube_stiffness(hx, lam, mu, K);
    for (int a2 = 0; a2 < 2; ++a2) {
      const int j = E.j0 + a2;             // node layer of the element's corners with this a2
      ms[j] += 4.0 * rho * hx * hx * hx / 8.0;
      for (int a1 = 0; a1 < 2; ++a1)
        for (int a3 = 0; a3 < 2; ++a3) {
          const int a = a1 + 2 * a2 + 4 * a3;
          for (int b = 0; b < 8; ++b) {
            const int o1 = (b & 1) - a1, o2 = ((b >> 1) & 1) - a2, o3 = ((b >> 2) & 1) - a3;
            const int o = (o1 + 1) + 3 * (o2 + 1) + 9 * (o3 + 1);
            double *blk = &st[(static_cast<size_t>(j) * 27 + o) * 9];
            for (int p = 0; p < 3; ++p)
              for (int q = 0; q < 3; ++q) blk[3 * p + q] += K[(3 * a + p) * 24 + 3 * b + q];
          }
        }
    }
  }
  const size_t n = static_cast<size_t>(s->cells);
  const size_t fb = static_cast<size_t>(c.nplanes) * 3 * n * h->rsize;
  hipError_t e;
  if ((e = dev_alloc(&s->node, 12 * static_cast<size_t>(s->nodes))) != hipSuccess ||
      (Lb > 0 && (e = dev_alloc(&s->r_fault, 6 * n)) != hipSuccess) ||
      (e = dev_alloc(&s->cell, kCellRows * n)) != hipSuccess ||
      (e = dev_alloc(&s->prm, 6 * n)) != hipSuccess ||
      (e = dev_alloc(&s->stencil, st.size())) != hipSuccess ||
      (e = dev_alloc(&s->mass, ms.size())) != hipSuccess ||
      (e = dev_alloc_bytes(&s->push_u, fb)) != hipSuccess ||
      (e = dev_alloc_bytes(&s->push_v, fb)) != hipSuccess ||
      (e = dev_alloc_bytes(&s->tau_sbi, fb)) != hipSuccess ||
      (e = dev_alloc(&s->bad, 1)) != hipSuccess) {
    s->h = nullptr;
    free_strip(s);
    return fail(h, SBIM_E_OOM, "strip allocation failed: %s", hipGetErrorString(e));
  }
  const size_t b = n * sizeof(double);
  long long bad = 0;
  if ((e = upload(s->stencil, st.data(), st.size() * sizeof(double), h->stream)) ||
      (e = upload(s->mass, ms.data(), ms.size() * sizeof(double), h->stream)) ||
      (e = hipMemcpyAsync(s->prm, prm->tau0, 3 * b, hipMemcpyDeviceToDevice, h->stream)) ||
      (e = hipMemcpyAsync(s->prm + 3 * n, prm->mu_s, b, hipMemcpyDeviceToDevice, h->stream)) ||
      (e = hipMemcpyAsync(s->prm + 4 * n, prm->mu_k, b, hipMemcpyDeviceToDevice, h->stream)) ||
      (e = hipMemcpyAsync(s->prm + 5 * n, prm->d_c, b, hipMemcpyDeviceToDevice, h->stream)) ||
      (e = hipMemsetAsync(s->bad, 0, sizeof(long long), h->stream)) ||
      (e = sbim::launch_fault_check(s->prm, s->prm + 3 * n, s->prm + 4 * n, s->prm + 5 * n,
                                    s->cells, s->bad, h->stream)) ||
      (e = hipMemcpyAsync(&bad, s->bad, sizeof bad, hipMemcpyDeviceToHost, h->stream)) ||
      (e = hipStreamSynchronize(h->stream))) {
    free_strip(s);
    return hip_fail(h, e, "strip set-up");
  }
  if (bad) {
    const long long cell = bad - 1;
    free_strip(s);
    return fail(h, SBIM_E_INVALID,
                "fault parameters at cell (i1=%lld, i3=%lld): need finite values, d_c > 0, "
                "0 <= mu_k <= mu_s",
                cell / h->n3, cell % h->n3);
  }
  int rc = strip_clear(s);
  if (rc) {
    free_strip(s);
    return rc;
  }
  *out = s;
  return SBIM_OK;
}

int sbim_strip_step(sbim_strip *s, double *tau_out, double *rate_out) {
  if (!s) return fail(nullptr, SBIM_E_INVALID, "strip is NULL");
  sbim_handle *h = s->h;
  if (h->step != s->steps)
    return fail(h, SBIM_E_STATE, "the handle was stepped outside its strip (%lld vs %lld steps)",
                h->step, s->steps);
  const long long n = s->cells;
  sbim::StripArgs a;
  a.u = s->node + 3 * s->cur * s->nodes;
  a.u_next = s->node + 3 * (1 - s->cur) * s->nodes;
  a.vh = s->node + 6 * s->nodes;
  a.v = s->node + 9 * s->nodes;
  a.stencil = s->stencil;
  a.mass = s->mass;
  a.tau_sbi = s->tau_sbi;
  a.push_u = s->push_u;
  a.push_v = s->push_v;
  a.tau0 = s->prm;
  a.mu_s = s->prm + 3 * n;
  a.mu_k = s->prm + 4 * n;
  a.d_c = s->prm + 5 * n;
  a.tau = s->cell + kCellTau * n;
  a.rate = s->cell + kCellRate * n;
  a.slip = s->cell + kCellSlip * n;
  a.sliding = s->cell + kCellSliding * n;
  a.tau_out = tau_out;
  a.rate_out = rate_out;
  a.nodes = s->nodes;
  a.cells = n;
  a.n1 = h->n1;
  a.n3 = h->n3;
  a.n2 = s->n2;
  a.fault_lo = s->fault_lo;
  a.r_fault = s->r_fault;
  a.dt = h->cfg.dt;
  a.area = h->cfg.dx1 * h->cfg.dx3;
  a.increment = h->cfg.input_kind == SBIM_INCREMENT;
  // push of u_{t+1} (or its increment) and the predicted velocity, written by
  // the previous step's predictor, redone first if the step size has changed
  // since (sbim_set_dt on a quasi-dynamic handle)
  if (h->cfg.dt != s->dt_pred) {
    hipError_t e0 = sbim::launch_strip_repredict(
        h->fp64, s->node + 3 * s->cur * s->nodes, s->node + 3 * (1 - s->cur) * s->nodes,
        s->node + 6 * s->nodes, s->node + 9 * s->nodes, s->push_u, s->push_v, s->nodes,
        s->cells, s->fault_lo >= 0, h->cfg.input_kind == SBIM_INCREMENT, h->cfg.dt,
        s->dt_pred, h->stream);
    if (e0 != hipSuccess) return hip_fail(h, e0, "strip predictor for the new step size");
    s->dt_pred = h->cfg.dt;
  }
  int rc = push_fields(h, s->push_u, s->push_v, sbim::VEL_INPUT);
  if (rc) return rc;
  hipError_t e = fft_inverse(h, h->out_spec, h->spec, s->tau_sbi, nullptr);
  if (e != hipSuccess) return hip_fail(h, e, "inverse FFT of the S+ (and S-) tractions");
  e = sbim::launch_strip_correct(h->fp64, a, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "strip corrector");
  if (s->fault_lo >= 0) {
    e = sbim::launch_strip_fault2(a, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "strip fault nodes");
  }
  s->cur = 1 - s->cur;
  s->steps += 1;
  return SBIM_OK;
}

int sbim_strip_read(const sbim_strip *s, int field, double *dst) {
  if (!s) return fail(nullptr, SBIM_E_INVALID, "strip is NULL");
  sbim_handle *h = s->h;
  if (!dst) return fail(h, SBIM_E_INVALID, "dst is NULL");
  const double *src;
  long long count;
  switch (field) {
    case SBIM_STRIP_TRACTION: src = s->cell + kCellTau * s->cells, count = 3 * s->cells; break;
    case SBIM_STRIP_SLIP_RATE: src = s->cell + kCellRate * s->cells, count = 2 * s->cells; break;
    case SBIM_STRIP_SLIP: src = s->cell + kCellSlip * s->cells, count = 2 * s->cells; break;
    case SBIM_STRIP_SLIDING: src = s->cell + kCellSliding * s->cells, count = s->cells; break;
    case SBIM_STRIP_DISPLACEMENT:   // u_{t+1}: the buffer the last step's stencil read
      src = s->node + 3 * (1 - s->cur) * s->nodes, count = 3 * s->nodes;
      break;
    case SBIM_STRIP_VELOCITY: src = s->node + 9 * s->nodes, count = 3 * s->nodes; break;
    default: return fail(h, SBIM_E_INVALID, "unknown strip field %d", field);
  }
  hipError_t e = hipMemcpyAsync(dst, src, sizeof(double) * count, hipMemcpyDeviceToDevice,
                                h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "strip read");
  return SBIM_OK;
}

int sbim_strip_reset(sbim_strip *s) {
  if (!s) return fail(nullptr, SBIM_E_INVALID, "strip is NULL");
  int rc = sbim_reset(s->h);
  if (rc) return rc;
  return strip_clear(s);
}

int sbim_strip_destroy(sbim_strip *s) {
  free_strip(s);
  return SBIM_OK;
}

}  // extern "C"
