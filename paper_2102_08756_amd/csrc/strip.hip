// Finite-element strip of the hybrid scheme: 8-node hexahedra on a regular grid
// between the fault (node layer 0) and the boundary S+ (node layer N2), periodic
// in x1 and x3 with the boundary-integral grid; explicit central differences in
// the predictor-corrector form of Sec. 2.2 (Eqs. fepred, feintdisp, tintf,
// fecorr); the traction of the half-space above S+ from the boundary relation
// (Eq. SBI, Sec. 2.4 items 2-4); the fault either as a symmetry plane or, in
// the two-sided strip, as split nodes between two element blocks, with the
// stick traction of the forward Lagrange multiplier (Eqs. freeslip,
// sticktraction) limited by the slip-weakening strength (Eqs. stickslip,
// slipweak).
//
// Fields are float64 [component][node layer][x1][x3] (x3 fastest); one thread
// per node in the predictor, per four nodes along x1 in each of three node
// layers in the corrector, per fault cell for the split nodes.  The
// stiffness is applied node by node as a 27-point stencil of 3x3 blocks, one
// stencil per node layer (the element layers above and below it may differ),
// precomputed on the host from the element stiffness.
#include <hip/hip_runtime.h>

#include "internal.h"

// Plain float64 rounding of each product and sum, as in the interface solve of
// the fault kernel: the stick/slip choice compares two such results.  The
// stencil sums alone are contracted into fused multiply-adds.
#pragma clang fp contract(off)

namespace sbim {
namespace {

constexpr int kStripThreads = 256;
constexpr int kStripRows = 4;        // nodes along x1 per thread of the corrector (divides n1)
constexpr int kStripLayers = 3;      // node layers per thread of the corrector

// The predictor of the next step from a node's new acceleration and velocity
// (Eq. fepred and the displacement update), with the push inputs of S+ (plane
// 0) or S- (plane 1) when the node lies on one of them.
template <typename R>
__device__ __forceinline__ void strip_predict(const StripArgs &a, long long k, int push_plane,
                                              long long cell, int c, double vn, double acc) {
  const double dt = a.dt;
  const double vh = vn + 0.5 * dt * acc;        // v_{t+3/2}
  const double un = a.u[k] + dt * vh;           // u_{t+2}
  a.v[k] = vn;
  a.vh[k] = vh;
  a.u_next[k] = un;
  if (push_plane >= 0) {
    R *__restrict__ pu = static_cast<R *>(a.push_u);
    R *__restrict__ pv = static_cast<R *>(a.push_v);
    const long long t = (push_plane * 3 + c) * a.cells + cell;
    pu[t] = static_cast<R>(a.increment ? dt * vh : un);
    pv[t] = static_cast<R>(vn + dt * acc);      // predicted velocity of Eq. fepred
  }
}

// Everything after the stiffness forces for one node: the S+ (S-) traction,
// the fault solve on layer 0 of the one-sided strip, the corrector and the
// fault outputs, then the predictor of the next step.
template <typename R>
__device__ __forceinline__ void strip_finish(const StripArgs &a, int layer, long long id,
                                             long long cell, double r[3]) {
  const long long nodes = a.nodes, cells = a.cells;
  const double A = a.area;
  const R *__restrict__ ts = static_cast<const R *>(a.tau_sbi);
  if (layer == a.n2) {                           // S+: traction of the half-space above
#pragma unroll
    for (int p = 0; p < 3; ++p) r[p] += A * static_cast<double>(ts[p * cells + cell]);
  }
  const bool two = a.fault_lo >= 0;
  if (two && layer == 0) {                       // S-: outward normal -e2
#pragma unroll
    for (int p = 0; p < 3; ++p) r[p] -= A * static_cast<double>(ts[(3 + p) * cells + cell]);
  }
  if (two && (layer == a.fault_lo || layer == a.fault_lo + 1)) {
    // split fault nodes: the two copies are solved together by strip_fault2
    const int side = layer == a.fault_lo ? 1 : 0;
#pragma unroll
    for (int p = 0; p < 3; ++p) a.r_fault[(side * 3 + p) * cells + cell] = r[p];
    return;
  }
  const double M = a.mass[layer];
  const double dt = a.dt;
  if (!two && layer == 0) {                      // fault node: stick traction and strength
    const double t00 = a.tau0[cell], t01 = a.tau0[cells + cell], t02 = a.tau0[2 * cells + cell];
    const double vs0 = a.vh[id] + dt * r[0] / M;
    const double vs2 = a.vh[2 * nodes + id] + dt * r[2] / M;
    const double st0 = t00 + M * vs0 / (dt * A);
    const double st2 = t02 + M * vs2 / (dt * A);
    const double mag = sqrt(st0 * st0 + st2 * st2);
    const double s0 = 2.0 * a.u[id], s2 = 2.0 * a.u[2 * nodes + id];
    const double delta = sqrt(s0 * s0 + s2 * s2);
    const double mus = a.mu_s[cell], muk = a.mu_k[cell], dc = a.d_c[cell];
    const double mu = delta < dc ? mus - (mus - muk) * delta / dc : muk;
    const double strength = fmax(-t01, 0.0) * mu;
    double tau0 = st0, tau2 = st2;
    const bool sliding = mag > strength;
    if (sliding) {
      const double sc = strength / mag;
      tau0 = st0 * sc;
      tau2 = st2 * sc;
    }
    r[0] -= A * (tau0 - t00);
    r[2] -= A * (tau2 - t02);
    a.tau[cell] = tau0;
    a.tau[cells + cell] = t01;
    a.tau[2 * cells + cell] = tau2;
    a.slip[cell] = s0;
    a.slip[cells + cell] = s2;
    a.sliding[cell] = sliding ? 1.0 : 0.0;
    if (a.tau_out) {
      a.tau_out[cell] = tau0;
      a.tau_out[cells + cell] = t01;
      a.tau_out[2 * cells + cell] = tau2;
    }
  }
  const int push_plane = layer == a.n2 ? 0 : (two && layer == 0 ? 1 : -1);
  double vn[3];
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    const long long k = p * nodes + id;
    const double acc = r[p] / M;
    vn[p] = a.vh[k] + 0.5 * dt * acc;            // v_{t+1} (Eqs. tintf, fecorr)
    strip_predict<R>(a, k, push_plane, cell, p, vn[p], acc);
  }
  if (!two && layer == 0) {
    a.rate[cell] = 2.0 * vn[0];
    a.rate[cells + cell] = 2.0 * vn[2];
    if (a.rate_out) {
      a.rate_out[cell] = 2.0 * vn[0];
      a.rate_out[cells + cell] = 2.0 * vn[2];
    }
  }
}

// One thread per kStripRows consecutive nodes along x1 (same x3) in each of
// kStripLayers consecutive node layers: each row of u that the 27-point
// stencils of those nodes need (node layers l0-1 .. l0+kStripLayers) is loaded
// once and serves up to three of the thread's layers and three of its rows.
// UNIFORM: every wavefront lies in one layer chunk, so the stencils are read
// through the scalar cache once per wavefront.
template <typename R, bool UNIFORM>
__global__ __launch_bounds__(kStripThreads) void strip_correct_kernel(StripArgs a) {
  const long long nodes = a.nodes, cells = a.cells;
  const int n1 = a.n1, n3 = a.n3, n2 = a.n2;
  const long long tid = static_cast<long long>(blockIdx.x) * kStripThreads + threadIdx.x;
  const long long per_chunk = cells / kStripRows;
  const int nchunks = (n2 + kStripLayers) / kStripLayers;
  if (tid >= per_chunk * nchunks) return;
  const int chunk = UNIFORM ? __builtin_amdgcn_readfirstlane(static_cast<int>(tid / per_chunk))
                            : static_cast<int>(tid / per_chunk);
  const int l0 = chunk * kStripLayers;
  const long long g = tid - chunk * per_chunk;
  const int ib = static_cast<int>(g / n3);
  const int i3 = static_cast<int>(g - static_cast<long long>(ib) * n3);
  const int i10 = ib * kStripRows;
  const int col[3] = {i3 == 0 ? n3 - 1 : i3 - 1, i3, i3 == n3 - 1 ? 0 : i3 + 1};

  double r[kStripLayers][kStripRows][3];
#pragma unroll
  for (int lo = 0; lo < kStripLayers; ++lo)
#pragma unroll
    for (int k = 0; k < kStripRows; ++k) r[lo][k][0] = r[lo][k][1] = r[lo][k][2] = 0.0;
#pragma unroll 1
  for (int li = -1; li <= kStripLayers; ++li) {   // u of node layer l0 + li
#pragma clang fp contract(fast)
    const int l = l0 + li;
    if (l < 0 || l > n2) continue;
    const long long base = static_cast<long long>(l) * cells;
#pragma unroll
    for (int q = 0; q < kStripRows + 2; ++q) {     // neighbour row i10 - 1 + q
      int jr = i10 - 1 + q;
      jr = jr < 0 ? jr + n1 : (jr >= n1 ? jr - n1 : jr);
      const long long rb = base + static_cast<long long>(jr) * n3;
      double u[3][3];
#pragma unroll
      for (int o3 = 0; o3 < 3; ++o3) {
        const long long nb = rb + col[o3];
        u[o3][0] = a.u[nb];
        u[o3][1] = a.u[nodes + nb];
        u[o3][2] = a.u[2 * nodes + nb];
      }
      // the row is the neighbour at offset o2 = li - lo of the thread's layer lo
#pragma unroll
      for (int lo = 0; lo < kStripLayers; ++lo) {
        const int o2 = li - lo;
        if (o2 < -1 || o2 > 1 || l0 + lo > n2) continue;
        const double *__restrict__ Cl =
            a.stencil + static_cast<long long>(l0 + lo) * 27 * 9 + 3 * (o2 + 1) * 9;
        // row q is the neighbour at offset o1 = q - 1 - k of node k
#pragma unroll
        for (int k = 0; k < kStripRows; ++k) {
          const int o1 = q - 1 - k;
          if (o1 < -1 || o1 > 1) continue;
#pragma unroll
          for (int o3 = 0; o3 < 3; ++o3) {
            const double *B = Cl + ((o1 + 1) + 9 * o3) * 9;
#pragma unroll
            for (int p = 0; p < 3; ++p) {
              r[lo][k][p] -= B[3 * p] * u[o3][0];
              r[lo][k][p] -= B[3 * p + 1] * u[o3][1];
              r[lo][k][p] -= B[3 * p + 2] * u[o3][2];
            }
          }
        }
      }
    }
  }
#pragma unroll
  for (int lo = 0; lo < kStripLayers; ++lo) {
    const int layer = l0 + lo;
    if (layer > n2) break;
#pragma unroll
    for (int k = 0; k < kStripRows; ++k) {
      const long long cell = static_cast<long long>(i10 + k) * n3 + i3;
      strip_finish<R>(a, layer, layer * cells + cell, cell, r[lo][k]);
    }
  }
}

// Split fault nodes (two-sided strip), one thread per cell: the traction change
// that closes the jump of the next half-step velocities of the two copies
// (Eqs. freeslip, sticktraction), applied in full to the normal component (no
// opening) and limited on the shear pair by the slip-weakening strength at the
// current normal traction (Eqs. stickslip, slipweak); then both copies' corrector
// and the predictor of the next step.
__global__ __launch_bounds__(kStripThreads) void strip_fault2_kernel(StripArgs a) {
  const long long cell = static_cast<long long>(blockIdx.x) * kStripThreads + threadIdx.x;
  const long long cells = a.cells, nodes = a.nodes;
  if (cell >= cells) return;
  const long long im = static_cast<long long>(a.fault_lo) * cells + cell;   // lower copy
  const long long ip = im + cells;                                          // upper copy
  const double Mm = a.mass[a.fault_lo], Mp = a.mass[a.fault_lo + 1];
  const double dt = a.dt, A = a.area;
  double rp[3], rm[3], t0[3], stick[3];
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    rp[p] = a.r_fault[p * cells + cell];
    rm[p] = a.r_fault[(3 + p) * cells + cell];
    t0[p] = a.tau0[p * cells + cell];
  }
  const double zinv = dt * A * (1.0 / Mp + 1.0 / Mm);
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    const double vsp = a.vh[p * nodes + ip] + dt * rp[p] / Mp;
    const double vsm = a.vh[p * nodes + im] + dt * rm[p] / Mm;
    stick[p] = t0[p] + (vsp - vsm) / zinv;
  }
  double tau[3] = {stick[0], stick[1], stick[2]};
  const double mag = sqrt(stick[0] * stick[0] + stick[2] * stick[2]);
  const double s0 = a.u[ip] - a.u[im], s2 = a.u[2 * nodes + ip] - a.u[2 * nodes + im];
  const double delta = sqrt(s0 * s0 + s2 * s2);
  const double mus = a.mu_s[cell], muk = a.mu_k[cell], dc = a.d_c[cell];
  const double mu = delta < dc ? mus - (mus - muk) * delta / dc : muk;
  const double strength = fmax(-tau[1], 0.0) * mu;
  const bool sliding = mag > strength;
  if (sliding) {
    const double sc = strength / mag;
    tau[0] = stick[0] * sc;
    tau[2] = stick[2] * sc;
  }
  double vp[3], vm[3];
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    const double dtau = A * (tau[p] - t0[p]);
    const double ap = (rp[p] - dtau) / Mp;
    const double am = (rm[p] + dtau) / Mm;
    vp[p] = a.vh[p * nodes + ip] + 0.5 * dt * ap;
    vm[p] = a.vh[p * nodes + im] + 0.5 * dt * am;
    // the split copies lie on neither S+ nor S-
    strip_predict<double>(a, p * nodes + ip, -1, cell, p, vp[p], ap);
    strip_predict<double>(a, p * nodes + im, -1, cell, p, vm[p], am);
    a.tau[p * cells + cell] = tau[p];
    if (a.tau_out) a.tau_out[p * cells + cell] = tau[p];
  }
  a.slip[cell] = s0;
  a.slip[cells + cell] = s2;
  a.sliding[cell] = sliding ? 1.0 : 0.0;
  a.rate[cell] = vp[0] - vm[0];
  a.rate[cells + cell] = vp[2] - vm[2];
  if (a.rate_out) {
    a.rate_out[cell] = vp[0] - vm[0];
    a.rate_out[cells + cell] = vp[2] - vm[2];
  }
}

// A new step size before a step (the quasi-dynamic boundary relation allows
// one): the predictor that the last step ran with its own size dt_old is redone
// with the new size dt, one thread per node, from u_{t+1}, v_{t+1} and the
// stored half-step velocity v_{t+1} + dt_old/2 a_{t+1}; the push inputs of S+
// (and S-) follow.
template <typename R>
__global__ __launch_bounds__(kStripThreads) void strip_repredict_kernel(
    double *u_pred, const double *u_prev, double *vh, const double *v, R *push_u, R *push_v,
    long long nodes, long long cells, int two_sided, int increment, double dt, double dt_old) {
  const long long id = static_cast<long long>(blockIdx.x) * kStripThreads + threadIdx.x;
  if (id >= nodes) return;
  const long long top0 = nodes - cells;
  const int plane = id >= top0 ? 0 : (two_sided && id < cells ? 1 : -1);
  const long long cell = plane == 0 ? id - top0 : id;
  const double ratio = dt / dt_old;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const long long k = c * nodes + id;
    const double vn = v[k];
    const double half = vh[k] - vn;             // dt_old/2 a_{t+1}
    const double h2 = vn + ratio * half;        // v_{t+3/2} with the new size
    const double un = u_prev[k] + dt * h2;
    vh[k] = h2;
    u_pred[k] = un;
    if (plane >= 0) {
      const long long t = (plane * 3 + c) * cells + cell;
      push_u[t] = static_cast<R>(increment ? dt * h2 : un);
      push_v[t] = static_cast<R>(vn + 2.0 * ratio * half);
    }
  }
}

}  // namespace

hipError_t launch_strip_repredict(bool fp64, double *u_pred, const double *u_prev, double *vh,
                                  const double *v, void *push_u, void *push_v, long long nodes,
                                  long long cells, bool two_sided, bool increment, double dt,
                                  double dt_old, hipStream_t st) {
  const unsigned blocks = static_cast<unsigned>((nodes + kStripThreads - 1) / kStripThreads);
  if (fp64)
    strip_repredict_kernel<double><<<blocks, kStripThreads, 0, st>>>(
        u_pred, u_prev, vh, v, static_cast<double *>(push_u), static_cast<double *>(push_v),
        nodes, cells, two_sided, increment, dt, dt_old);
  else
    strip_repredict_kernel<float><<<blocks, kStripThreads, 0, st>>>(
        u_pred, u_prev, vh, v, static_cast<float *>(push_u), static_cast<float *>(push_v),
        nodes, cells, two_sided, increment, dt, dt_old);
  return hipGetLastError();
}

hipError_t launch_strip_fault2(const StripArgs &a, hipStream_t st) {
  const unsigned blocks = static_cast<unsigned>((a.cells + kStripThreads - 1) / kStripThreads);
  strip_fault2_kernel<<<blocks, kStripThreads, 0, st>>>(a);
  return hipGetLastError();
}

hipError_t launch_strip_correct(bool fp64, const StripArgs &a, hipStream_t st) {
  const long long threads = a.cells / kStripRows * ((a.n2 + kStripLayers) / kStripLayers);
  const unsigned blocks = static_cast<unsigned>((threads + kStripThreads - 1) / kStripThreads);
  const bool uniform = (a.cells / kStripRows) % 64 == 0;
  if (fp64) {
    if (uniform)
      strip_correct_kernel<double, true><<<blocks, kStripThreads, 0, st>>>(a);
    else
      strip_correct_kernel<double, false><<<blocks, kStripThreads, 0, st>>>(a);
  } else {
    if (uniform)
      strip_correct_kernel<float, true><<<blocks, kStripThreads, 0, st>>>(a);
    else
      strip_correct_kernel<float, false><<<blocks, kStripThreads, 0, st>>>(a);
  }
  return hipGetLastError();
}

}  // namespace sbim
