// Mode-space kernels of the boundary-integral step on gfx950:
//   push_kernel      rotate a new spectrum into the wavevector frame, update the
//                    float64 running state, store the history ring slot and the
//                    velocity spectrum used by the damping term;
//   conv_kernel      the truncated history convolution (the nonlocal term of
//                    Eq. SBI, Sec. 2.3) fused with the damping and instantaneous
//                    terms and the rotation back to (x1, x2, x3);
//   tabulate_kernel  float64 quadrature of the per-lag kernel weights.
//
// Layouts (one material group; modes sorted by (W desc, q asc), 64 per block):
//   ring    [record][plane][component L,N,T][64 lanes] complex.  Step n of
//           block b lives in record blk_off[b] + (n mod blk_cap[b]) * blk_stride[b]:
//           consecutive blocks of equal capacity form a run laid out slot-major
//           (stride = run length), so one history slot of a run is contiguous;
//   table   lag-major rows: entry lag_off[j] + class holds (w11, w12, w22, w33);
//           classes are sorted by W desc, so the classes alive at lag j are a
//           prefix of the row.
#include <cmath>

#include "internal.h"

namespace sbim {
namespace {

template <typename R> struct C2;
template <> struct C2<float> { using T = float2; };
template <> struct C2<double> { using T = double2; };
template <typename R> using cplx = typename C2<R>::T;

template <typename R> struct W4;
template <> struct W4<float> { using T = float4; };
template <> struct W4<double> { using T = double4; };

// ------------------------------------------------------------------ push

template <typename R>
__global__ __launch_bounds__(256) void push_kernel(
    const double2 *__restrict__ spec, const double2 *__restrict__ spec_v,
    cplx<R> *__restrict__ ring, double2 *__restrict__ state, cplx<R> *__restrict__ vel,
    const int *__restrict__ nat, const double *__restrict__ geom,
    const long long *__restrict__ blk_off, const int *__restrict__ blk_cap,
    const int *__restrict__ blk_stride, long long M, long long nh, int np, int plane0, int plane1,
    long long step, double inv_dt, int vel_rule, int state_rule) {
  // one thread per (mode, plane); consecutive threads take consecutive modes
  const long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= M * np) return;
  const int p = static_cast<int>(t / M);
  const long long s = t - p * M;
  const long long natural = nat[s];
  const double kh1 = geom[4 * s + 1];
  const double kh3 = geom[4 * s + 2];
  const long long b = s >> 6;
  const int lane = static_cast<int>(s & 63);
  const int cap = blk_cap[b];
  const long long rec = cap > 0 ? blk_off[b] + (step % cap) * blk_stride[b] : 0;
  {
    const int pg = p == 0 ? plane0 : plane1;
    double2 x[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) x[c] = spec[(pg * 3 + c) * nh + natural];
    // (1, 2, 3) -> (L, N, T)
    const double2 xr[3] = {{kh1 * x[0].x + kh3 * x[2].x, kh1 * x[0].y + kh3 * x[2].y},
                           x[1],
                           {-kh3 * x[0].x + kh1 * x[2].x, -kh3 * x[0].y + kh1 * x[2].y}};
    double2 vr[3];
    if (vel_rule == VEL_INPUT) {
      double2 y[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) y[c] = spec_v[(pg * 3 + c) * nh + natural];
      vr[0] = double2{kh1 * y[0].x + kh3 * y[2].x, kh1 * y[0].y + kh3 * y[2].y};
      vr[1] = y[1];
      vr[2] = double2{-kh3 * y[0].x + kh1 * y[2].x, -kh3 * y[0].y + kh1 * y[2].y};
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const long long si = (static_cast<long long>(p) * 3 + c) * M + s;
      const double2 prev = state[si];
      double2 now;
      if (state_rule == STATE_ACCUM)
        now = double2{prev.x + xr[c].x, prev.y + xr[c].y};
      else
        now = xr[c];
      state[si] = now;
      double2 v;
      if (vel_rule == VEL_DIFF)
        v = double2{(now.x - prev.x) * inv_dt, (now.y - prev.y) * inv_dt};
      else if (vel_rule == VEL_SCALE)
        v = double2{xr[c].x * inv_dt, xr[c].y * inv_dt};
      else if (vel_rule == VEL_INPUT)
        v = vr[c];
      else
        v = xr[c];
      vel[si] = cplx<R>{static_cast<R>(v.x), static_cast<R>(v.y)};
      if (cap > 0)
        ring[((rec * np + p) * 3 + c) * kLanes + lane] =
            cplx<R>{static_cast<R>(now.x), static_cast<R>(now.y)};
    }
  }
}

// ------------------------------------------------------------------ conv

// Neumaier's compensated addition: s + x with the rounding error kept in c.
__device__ __forceinline__ void neumaier(float &s, float &c, float x) {
  const float t = s + x;
  if (fabsf(s) >= fabsf(x))
    c += (s - t) + x;
  else
    c += (x - t) + s;
  s = t;
}

// Accumulator of one real history sum: plain (T = R) or compensated (float pair).
template <typename R, bool COMP> struct Acc;
template <typename R> struct Acc<R, false> {
  R s = R(0);
  __device__ __forceinline__ void fold(R x) { s += x; }
  __device__ __forceinline__ void fold_pair(R x, R) { s += x; }
  __device__ __forceinline__ R value() const { return s; }
  __device__ __forceinline__ R comp() const { return R(0); }
};
template <> struct Acc<float, true> {
  float s = 0.f, c = 0.f;
  __device__ __forceinline__ void fold(float x) { neumaier(s, c, x); }
  __device__ __forceinline__ void fold_pair(float x, float xc) {
    neumaier(s, c, x);
    c += xc;
  }
  __device__ __forceinline__ float value() const { return s + c; }
  __device__ __forceinline__ float comp() const { return c; }
};

// Five complex history sums per plane: C11[U_L], C12[U_N], C22[U_N], C12[U_L], C33[U_T].
constexpr int kSums = 10;  // real accumulators per plane

// Lags handled per unrolled chunk: loads of U lags are issued before their FMAs.
// (Measured on gfx950: 4 for plain float32; 2 for float64 and for the
// compensated form, whose extra registers otherwise cost a wave per SIMD.)
template <typename R, bool COMP> constexpr int conv_unroll() {
  return (sizeof(R) == 8 || COMP) ? 2 : 4;
}

// One lag for all planes of the lane's mode: weights of the lane's kernel row
// (zero once the lag passes the lane's own window W(q): such lanes read the
// row of class 0, which is alive at every lag of the block, and discard it).
template <typename R, int NP>
__device__ __forceinline__ void load_lag(const cplx<R> *__restrict__ ring,
                                         const typename W4<R>::T *__restrict__ table,
                                         const long long *__restrict__ lag_off, long long record,
                                         int lane, int j, int llane, int cl,
                                         typename W4<R>::T &w, cplx<R> (&u)[NP][3]) {
  const bool on = j < llane;
  w = table[lag_off[j] + (on ? cl : 0)];
  if (!on) w = typename W4<R>::T{R(0), R(0), R(0), R(0)};
  // the history is read once per step: non-temporal loads keep it from
  // displacing the kernel rows and indices in the caches
  const cplx<R> *r = ring + record * NP * 3 * kLanes + lane;
  typedef R nv2 __attribute__((ext_vector_type(2)));
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const nv2 v =
          __builtin_nontemporal_load(reinterpret_cast<const nv2 *>(r + (p * 3 + c) * kLanes));
      u[p][c] = cplx<R>{v.x, v.y};
    }
}

// part[p][.] += w * u for the five history sums of each plane.
template <typename R, int NP>
__device__ __forceinline__ void fma_lag(R (&part)[NP][kSums], const typename W4<R>::T &w,
                                        const cplx<R> (&u)[NP][3]) {
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    part[p][0] = fma(w.x, u[p][0].x, part[p][0]);
    part[p][1] = fma(w.x, u[p][0].y, part[p][1]);
    part[p][2] = fma(w.y, u[p][1].x, part[p][2]);
    part[p][3] = fma(w.y, u[p][1].y, part[p][3]);
    part[p][4] = fma(w.z, u[p][1].x, part[p][4]);
    part[p][5] = fma(w.z, u[p][1].y, part[p][5]);
    part[p][6] = fma(w.y, u[p][0].x, part[p][6]);
    part[p][7] = fma(w.y, u[p][0].y, part[p][7]);
    part[p][8] = fma(w.w, u[p][2].x, part[p][8]);
    part[p][9] = fma(w.w, u[p][2].y, part[p][9]);
  }
}

// Work-item split of the history sums.  Item (b, c) = block b of 64 modes and
// chunk c of its lags; one wavefront per item streams the chunk's history
// records and kernel rows and writes its ten partial sums per plane:
//   partial[(c * NP * 10 + k) * M + s],  k = plane * 10 + sum index.
// Items are small and uniform, so the dispatch has no long tail.
template <typename R, int NP, bool COMP>
__global__ __launch_bounds__(kLanes) void conv_stream_kernel(
    const cplx<R> *__restrict__ ring, const typename W4<R>::T *__restrict__ table,
    R *__restrict__ partial, const int *__restrict__ cls, const int *__restrict__ win,
    const long long *__restrict__ blk_off, const int *__restrict__ blk_cap,
    const int *__restrict__ blk_stride, const long long *__restrict__ lag_off, long long M,
    long long step, int chunks, int nblocks) {
  constexpr int U = conv_unroll<R, COMP>();
  // chunk-major item order: the waves in flight at any time work on the same
  // lag range of consecutive blocks, whose records are adjacent in memory
  const int ch = blockIdx.x / nblocks;
  const int b = blockIdx.x - ch * nblocks;
  const int lane = threadIdx.x;
  const long long s = static_cast<long long>(b) * kLanes + lane;
  const bool valid = s < M;
  const int cap = blk_cap[b];
  const long long navail = step + 1;
  const int lblk = static_cast<int>(min(static_cast<long long>(cap), navail));
  const int wl = valid ? win[s] : 0;
  const int llane = static_cast<int>(min(static_cast<long long>(wl), navail));
  const int cl = valid ? cls[s] : 0;
  const int per = (lblk + chunks - 1) / chunks;
  const int j0 = min(lblk, ch * per);
  const int j1 = min(lblk, j0 + per);
  const long long base = cap > 0 ? blk_off[b] : 0;
  const long long stride = blk_stride[b];

  Acc<R, COMP> acc[NP][kSums];
  if (j0 < j1) {
    int rec = static_cast<int>((step - j0) % cap);  // ring slot of lag j0
    int j = j0;
    if (cap >= U) {
      for (; j + U <= j1; j += U) {
        typename W4<R>::T w[U];
        cplx<R> u[U][NP][3];
#pragma unroll
        for (int t = 0; t < U; ++t) {
          const int rr = rec - t < 0 ? rec - t + cap : rec - t;
          load_lag<R, NP>(ring, table, lag_off, base + rr * stride, lane, j + t, llane, cl, w[t],
                          u[t]);
        }
        if constexpr (COMP) {
          R part[NP][kSums];
#pragma unroll
          for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int k = 0; k < kSums; ++k) part[p][k] = R(0);
#pragma unroll
          for (int t = 0; t < U; ++t) fma_lag<R, NP>(part, w[t], u[t]);
#pragma unroll
          for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int k = 0; k < kSums; ++k) acc[p][k].fold(part[p][k]);
        } else {
          R sums[NP][kSums];
#pragma unroll
          for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int k = 0; k < kSums; ++k) sums[p][k] = acc[p][k].s;
#pragma unroll
          for (int t = 0; t < U; ++t) fma_lag<R, NP>(sums, w[t], u[t]);
#pragma unroll
          for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int k = 0; k < kSums; ++k) acc[p][k].s = sums[p][k];
        }
        rec -= U;
        if (rec < 0) rec += cap;
      }
    }
    for (; j < j1; ++j) {  // remaining lags one at a time
      typename W4<R>::T w;
      cplx<R> u[NP][3];
      load_lag<R, NP>(ring, table, lag_off, base + rec * stride, lane, j, llane, cl, w, u);
      R part[NP][kSums];
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int k = 0; k < kSums; ++k) part[p][k] = COMP ? R(0) : acc[p][k].s;
      fma_lag<R, NP>(part, w, u);
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int k = 0; k < kSums; ++k) {
          if constexpr (COMP)
            acc[p][k].fold(part[p][k]);
          else
            acc[p][k].s = part[p][k];
        }
      rec = rec == 0 ? cap - 1 : rec - 1;
    }
  }
  if (!valid) return;
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int k = 0; k < kSums; ++k)
      __builtin_nontemporal_store(  // read once, by the epilogue
          acc[p][k].value(),
          partial + (static_cast<long long>(ch) * NP * kSums + p * kSums + k) * M + s);
}

// Per mode: fold the chunk partials in chunk order (compensated for the
// compensated form), add damping and instantaneous terms, rotate back to
// (x1, x2, x3) and scatter into the natural half-spectrum layout.
template <typename R, int NP, bool COMP>
__global__ __launch_bounds__(256) void conv_epilogue_kernel(
    const R *__restrict__ partial, const cplx<R> *__restrict__ ring,
    const cplx<R> *__restrict__ vel, double2 *__restrict__ lam, cplx<R> *__restrict__ out_a,
    cplx<R> *__restrict__ out_b, const int *__restrict__ nat, const int *__restrict__ win,
    const double *__restrict__ geom, const long long *__restrict__ blk_off,
    const int *__restrict__ blk_cap, const int *__restrict__ blk_stride, long long M, long long nh,
    long long step, int chunks, PlaneParams p0, PlaneParams p1) {
  // one thread per (mode, plane); consecutive threads take consecutive modes
  const long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= M * NP) return;
  const int p = static_cast<int>(t / M);
  const long long s = t - p * M;
  const long long b = s >> 6;
  const int lane = static_cast<int>(s & 63);
  const int cap = blk_cap[b];
  const int wl = win[s];
  const double q = geom[4 * s + 0];
  const R kh1 = static_cast<R>(geom[4 * s + 1]);
  const R kh3 = static_cast<R>(geom[4 * s + 2]);
  const long long natural = nat[s];
  const long long rec0 = cap > 0 ? blk_off[b] + (step % cap) * blk_stride[b] : 0;
  // fold the chunk partials in chunk order (ten sums of a chunk loaded together)
  R cs[kSums];
  {
    Acc<R, COMP> a[kSums];
#pragma unroll 4
    for (int c = 0; c < chunks; ++c) {
      const R *pc = partial + (static_cast<long long>(c) * NP + p) * kSums * M + s;
      R v[kSums];
#pragma unroll
      for (int k = 0; k < kSums; ++k) v[k] = pc[k * M];
#pragma unroll
      for (int k = 0; k < kSums; ++k) a[k].fold(v[k]);
    }
#pragma unroll
    for (int k = 0; k < kSums; ++k) cs[k] = a[k].value();
  }
  {
    const PlaneParams &pp = p == 0 ? p0 : p1;
    const R sg = static_cast<R>(pp.side);
    const R muq = static_cast<R>(pp.mu * q);
    const R damp = static_cast<R>(pp.mu / pp.cs);
    const R inst = static_cast<R>((2.0 - pp.eta) * pp.mu * q);
    const R eta = static_cast<R>(pp.eta);
    cplx<R> u[3] = {{R(0), R(0)}, {R(0), R(0)}, {R(0), R(0)}};
    if (cap > 0 && wl > 0) {
      const cplx<R> *r = ring + (rec0 * NP + p) * 3 * kLanes + lane;
      u[0] = r[0];
      u[1] = r[kLanes];
      u[2] = r[2 * kLanes];
    }
    cplx<R> v[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c] = vel[(static_cast<long long>(p) * 3 + c) * M + s];
    // conv + instantaneous (rotated frame):
    //   A_L = -sg mu q C11 + i (2-eta) mu q U_N - i mu q C12[U_N]
    //   A_N = -sg mu q C22 - i (2-eta) mu q U_L + i mu q C12[U_L]
    //   A_T = -sg mu q C33
    cplx<R> a[3];
    a[0] = cplx<R>{-sg * muq * cs[0] - inst * u[1].y + muq * cs[3],
                   -sg * muq * cs[1] + inst * u[1].x - muq * cs[2]};
    a[1] = cplx<R>{-sg * muq * cs[4] + inst * u[0].y - muq * cs[7],
                   -sg * muq * cs[5] - inst * u[0].x + muq * cs[6]};
    a[2] = cplx<R>{-sg * muq * cs[8], -sg * muq * cs[9]};
    // damping: -sg (mu/c_s) diag(1, eta, 1) V
    cplx<R> d[3] = {{-sg * damp * v[0].x, -sg * damp * v[0].y},
                    {-sg * damp * eta * v[1].x, -sg * damp * eta * v[1].y},
                    {-sg * damp * v[2].x, -sg * damp * v[2].y}};
    if (lam) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const long long si = (static_cast<long long>(p) * 3 + c) * M + s;
        double2 l = lam[si];
        l.x += static_cast<double>(a[c].x);
        l.y += static_cast<double>(a[c].y);
        lam[si] = l;
        a[c] = cplx<R>{static_cast<R>(l.x), static_cast<R>(l.y)};
      }
    }
    if (!out_b) {
#pragma unroll
      for (int c = 0; c < 3; ++c) a[c] = cplx<R>{a[c].x + d[c].x, a[c].y + d[c].y};
    }
    const int pg = pp.index;
    // (L, N, T) -> (1, 2, 3)
    out_a[(pg * 3 + 0) * nh + natural] =
        cplx<R>{kh1 * a[0].x - kh3 * a[2].x, kh1 * a[0].y - kh3 * a[2].y};
    out_a[(pg * 3 + 1) * nh + natural] = a[1];
    out_a[(pg * 3 + 2) * nh + natural] =
        cplx<R>{kh3 * a[0].x + kh1 * a[2].x, kh3 * a[0].y + kh1 * a[2].y};
    if (out_b) {
      out_b[(pg * 3 + 0) * nh + natural] =
          cplx<R>{kh1 * d[0].x - kh3 * d[2].x, kh1 * d[0].y - kh3 * d[2].y};
      out_b[(pg * 3 + 1) * nh + natural] = d[1];
      out_b[(pg * 3 + 2) * nh + natural] =
          cplx<R>{kh3 * d[0].x + kh1 * d[2].x, kh3 * d[0].y + kh1 * d[2].y};
    }
  }
}

// -------------------------------------------------------------- tabulate

// Piece A (0 < y < 1): y = sin(t).  Piece B (1 < y < eta): y^2 = 1 + (eta^2-1) sin^2(t).
// Both map t in [0, pi/2] and remove the square-root end points of the
// branch-cut densities D_ab (see the oracle-independent derivation in the
// library notes): the substituted integrands are analytic.
struct Node {
  double y, g11, g12, g22, g33, ph_hi, ph_lo;
};

__device__ Node make_node(int i, int npan, double eta, double dT, const double *gl_x,
                          const double *gl_w) {
  const int per_piece = npan * kGaussN;
  const int piece = i / per_piece;
  const int r = i - piece * per_piece;
  const int pan = r / kGaussN;
  const int g = r - pan * kGaussN;
  const double half_pi = 1.5707963267948966;
  const double h = half_pi / npan;
  const double t = (pan + 0.5 * (gl_x[g] + 1.0)) * h;
  const double wt = 0.5 * gl_w[g] * h;
  const double e2 = eta * eta;
  const double st = sin(t), ct = cos(t);
  Node n;
  double d11, d12, d22, d33, jac, y;
  if (piece == 0) {
    y = st;
    const double as = ct;
    const double ap = sqrt(1.0 - y * y / e2);
    const double d = e2 + 1.0 - y * y;
    jac = ct * wt;
    d11 = 2.0 * (as * (e2 - y * y) + e2 * ap) / d;
    d22 = 2.0 * e2 * ((1.0 - y * y) * ap + as) / d;
    d12 = 0.0;
    d33 = 2.0 * as;
  } else {
    y = sqrt(1.0 + (e2 - 1.0) * st * st);
    const double bs = sqrt(e2 - 1.0) * st;
    const double ap = sqrt(e2 - 1.0) * ct / eta;
    const double d = e2 + 1.0 - y * y;
    jac = (e2 - 1.0) * st * ct / y * wt;
    d11 = 2.0 * e2 * ap / d;
    d22 = 2.0 * e2 * (1.0 - y * y) * ap / d;
    d12 = -2.0 * e2 * bs * ap / d;
    d33 = 0.0;
  }
  // (2/pi) * sin(y dT / 2) / y * density * jacobian
  const double f = 0.63661977236758134 * sin(0.5 * y * dT) / y * jac;
  n.y = y;
  n.g11 = f * d11;
  n.g12 = f * d12;
  n.g22 = f * d22;
  n.g33 = f * d33;
  n.ph_hi = y * dT;                    // y dT = ph_hi + ph_lo exactly
  n.ph_lo = fma(y, dT, -n.ph_hi);
  return n;
}

// w_ab,j = sum_nodes g_ab cos or sin((j + 1/2) y dT).  The phase is formed as a
// double-double and reduced by 2 pi in two parts (Cody-Waite), so it is
// accurate to ~1e-16 absolute however many periods it spans.
template <typename R>
__global__ __launch_bounds__(256) void tabulate_kernel(
    typename W4<R>::T *__restrict__ table, const long long *__restrict__ lag_off,
    const double *__restrict__ cls_q, const int *__restrict__ cls_w, double cs, double dt,
    double eta, double rate, const double *__restrict__ gl_x, const double *__restrict__ gl_w) {
  __shared__ Node nodes[256];
  const int c = blockIdx.x;
  const int W = cls_w[c];
  const double q = cls_q[c];
  const double dT = q * cs * dt;
  const double tmax = dT * W * rate;
  const int npan = max(1, static_cast<int>(ceil(tmax / 40.0)));
  const int nnodes = 2 * npan * kGaussN;
  const double two_pi_hi = 6.283185307179586;      // nearest double to 2 pi
  const double two_pi_lo = 2.4492935982947064e-16;  // 2 pi - two_pi_hi
  const double inv_two_pi = 0.15915494309189535;
  for (int jb = 0; jb < W; jb += 256) {
    const int j = jb + threadIdx.x;
    const double m = j + 0.5;
    double w11 = 0, w12 = 0, w22 = 0, w33 = 0;
    for (int nb = 0; nb < nnodes; nb += 256) {
      __syncthreads();
      if (nb + threadIdx.x < nnodes)
        nodes[threadIdx.x] = make_node(nb + threadIdx.x, npan, eta, dT, gl_x, gl_w);
      __syncthreads();
      const int cnt = min(256, nnodes - nb);
      if (j < W) {
        for (int i = 0; i < cnt; ++i) {
          const Node &nd = nodes[i];
          const double p_hi = m * nd.ph_hi;
          const double p_lo = fma(m, nd.ph_lo, fma(m, nd.ph_hi, -p_hi));
          const double k = rint(p_hi * inv_two_pi);
          double r = fma(-k, two_pi_hi, p_hi);  // exact
          r = fma(-k, two_pi_lo, r) + p_lo;
          double sn, cn;
          sincos(r, &sn, &cn);
          w11 = fma(nd.g11, cn, w11);
          w12 = fma(nd.g12, sn, w12);
          w22 = fma(nd.g22, cn, w22);
          w33 = fma(nd.g33, cn, w33);
        }
      }
    }
    if (j < W) {
      typename W4<R>::T o;
      o.x = static_cast<R>(w11);
      o.y = static_cast<R>(w12);
      o.z = static_cast<R>(w22);
      o.w = static_cast<R>(w33);
      table[lag_off[j] + c] = o;
    }
  }
}

template <typename R, int NP, bool COMP>
hipError_t conv_launch_np(const sbim_handle *h, const Group &g, const ConvLaunch &a,
                          hipEvent_t ev0, hipEvent_t ev1) {
  const PlaneParams p1 = g.np > 1 ? g.pl[1] : g.pl[0];
  const int chunks = h->lag_split;
  const long long items = g.nblocks * chunks;
  if (ev0) (void)hipEventRecord(ev0, h->stream);
  hipLaunchKernelGGL((conv_stream_kernel<R, NP, COMP>), dim3(static_cast<unsigned>(items)),
                     dim3(kLanes), 0, h->stream, static_cast<const cplx<R> *>(a.ring),
                     static_cast<const typename W4<R>::T *>(g.table), static_cast<R *>(g.partial),
                     g.cls, g.win, g.blk_off, g.blk_cap, g.blk_stride, g.lag_off, g.M, a.step,
                     chunks, static_cast<int>(g.nblocks));
  if (ev1) (void)hipEventRecord(ev1, h->stream);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((conv_epilogue_kernel<R, NP, COMP>),
                     dim3(static_cast<unsigned>((g.M * NP + 255) / 256)),
                     dim3(256), 0, h->stream, static_cast<const R *>(g.partial),
                     static_cast<const cplx<R> *>(a.ring), static_cast<const cplx<R> *>(a.vel),
                     reinterpret_cast<double2 *>(a.lam), static_cast<cplx<R> *>(a.out_a),
                     static_cast<cplx<R> *>(a.out_b), g.nat, g.win, g.geom, g.blk_off, g.blk_cap,
                     g.blk_stride, g.M, a.nh, a.step, chunks, g.pl[0], p1);
  return hipGetLastError();
}

template <typename R, bool COMP>
hipError_t conv_launch_r(const sbim_handle *h, const Group &g, const ConvLaunch &a,
                         hipEvent_t ev0, hipEvent_t ev1) {
  return g.np == 2 ? conv_launch_np<R, 2, COMP>(h, g, a, ev0, ev1)
                   : conv_launch_np<R, 1, COMP>(h, g, a, ev0, ev1);
}

}  // namespace

hipError_t launch_push(const sbim_handle *h, const Group &g, const PushLaunch &a) {
  const unsigned grid = static_cast<unsigned>((g.M * g.np + 255) / 256);
  const int p0 = g.pl[0].index;
  const int p1 = g.np > 1 ? g.pl[1].index : p0;
  if (h->fp64) {
    hipLaunchKernelGGL(push_kernel<double>, dim3(grid), dim3(256), 0, h->stream,
                       static_cast<const double2 *>(a.spec), static_cast<const double2 *>(a.spec_v),
                       static_cast<double2 *>(a.ring), reinterpret_cast<double2 *>(a.state),
                       static_cast<double2 *>(a.vel), g.nat, g.geom, g.blk_off, g.blk_cap, g.blk_stride, g.M,
                       a.nh, g.np, p0, p1, a.step, 1.0 / a.dt, a.vel_rule, a.state_rule);
  } else {
    hipLaunchKernelGGL(push_kernel<float>, dim3(grid), dim3(256), 0, h->stream,
                       static_cast<const double2 *>(a.spec), static_cast<const double2 *>(a.spec_v),
                       static_cast<float2 *>(a.ring), reinterpret_cast<double2 *>(a.state),
                       static_cast<float2 *>(a.vel), g.nat, g.geom, g.blk_off, g.blk_cap, g.blk_stride, g.M,
                       a.nh, g.np, p0, p1, a.step, 1.0 / a.dt, a.vel_rule, a.state_rule);
  }
  return hipGetLastError();
}

hipError_t launch_conv(const sbim_handle *h, const Group &g, const ConvLaunch &a, hipEvent_t ev0,
                       hipEvent_t ev1) {
  if (h->fp64) return conv_launch_r<double, false>(h, g, a, ev0, ev1);
  if (h->comp) return conv_launch_r<float, true>(h, g, a, ev0, ev1);
  return conv_launch_r<float, false>(h, g, a, ev0, ev1);
}

hipError_t launch_tabulate(bool fp64, const Group &g, double dt, const double *gl_x,
                           const double *gl_w, hipStream_t st) {
  if (g.nclasses == 0) return hipSuccess;
  const double rate = fmax(1.0, (g.eta * g.eta - 1.0) / 2.0);
  if (fp64) {
    hipLaunchKernelGGL(tabulate_kernel<double>, dim3(static_cast<unsigned>(g.nclasses)), dim3(256),
                       0, st, static_cast<double4 *>(g.table), g.lag_off, g.cls_q, g.cls_w, g.cs, dt,
                       g.eta, rate, gl_x, gl_w);
  } else {
    hipLaunchKernelGGL(tabulate_kernel<float>, dim3(static_cast<unsigned>(g.nclasses)), dim3(256),
                       0, st, static_cast<float4 *>(g.table), g.lag_off, g.cls_q, g.cls_w, g.cs, dt,
                       g.eta, rate, gl_x, gl_w);
  }
  return hipGetLastError();
}

}  // namespace sbim
