// Real 2-D FFT of boundary fields on gfx950: row real-to-complex / complex-to-real
// transforms and strided column transforms, each done by one work-group in LDS
// with Stockham autosort radix-4 passes (one radix-2 pass when log2 N is odd).
//
// Conventions (the paper fixes none): forward exp(-i k.x), stored half spectrum
// [n1][n3/2+1]; the inverse drops the imaginary parts of the i3 = 0 and
// i3 = n3/2 columns and applies the caller's scale (1/(n1 n3) for tractions).
#include <cmath>

#include "internal.h"

namespace sbim {
namespace {

template <typename R> struct C2;
template <> struct C2<float> { using T = float2; };
template <> struct C2<double> { using T = double2; };
template <typename R> using cplx = typename C2<R>::T;

template <typename R>
__device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename R>
__device__ __forceinline__ cplx<R> cadd(cplx<R> a, cplx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ cplx<R> csub(cplx<R> a, cplx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ cplx<R> cconj(cplx<R> a) { return {a.x, -a.y}; }

// exp(dir * 2 pi i m / 4096) from the table of exp(-2 pi i m / 4096).
template <typename R>
__device__ __forceinline__ cplx<R> twiddle(const cplx<R> *__restrict__ tw, int m, int dir) {
  cplx<R> t = tw[m & (kTwiddleN - 1)];
  if (dir > 0) t.y = -t.y;
  return t;
}

// In-place FFT of nseq contiguous sequences of length N = 2^logN held in LDS.
// Every thread of the work-group must call it.  Each pass stages its inputs
// in registers, synchronises, then writes the Stockham-ordered outputs.
template <typename R, int NT, int MAXV>
__device__ void lds_fft(cplx<R> *buf, int N, int logN, int nseq, int dir,
                        const cplx<R> *__restrict__ tw) {
  const int total = N * nseq;
  int logNs = 0;
  // radix-4 passes
  for (; logNs + 2 <= logN; logNs += 2) {
    const int q4 = N >> 2;
    const int nbf = total >> 2;
    cplx<R> v[MAXV / 4][4];
#pragma unroll
    for (int t = 0; t < MAXV / 4; ++t) {
      const int g = threadIdx.x + t * NT;
      if (g < nbf) {
        const int b = g >> (logN - 2);
        const int j = g & (q4 - 1);
        const int base = b * N + j;
#pragma unroll
        for (int r = 0; r < 4; ++r) v[t][r] = buf[base + r * q4];
      }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < MAXV / 4; ++t) {
      const int g = threadIdx.x + t * NT;
      if (g < nbf) {
        const int b = g >> (logN - 2);
        const int j = g & (q4 - 1);
        const int Ns = 1 << logNs;
        const int k = j & (Ns - 1);
        const int step = kTwiddleN >> (logNs + 2);  // 4096 / (4 Ns)
        cplx<R> a0 = v[t][0];
        cplx<R> a1 = cmul<R>(v[t][1], twiddle<R>(tw, k * step, dir));
        cplx<R> a2 = cmul<R>(v[t][2], twiddle<R>(tw, 2 * k * step, dir));
        cplx<R> a3 = cmul<R>(v[t][3], twiddle<R>(tw, 3 * k * step, dir));
        cplx<R> t0 = cadd<R>(a0, a2), t1 = csub<R>(a0, a2);
        cplx<R> t2 = cadd<R>(a1, a3), d = csub<R>(a1, a3);
        // t3 = dir * i * (a1 - a3): -i for the forward transform, +i for the inverse
        cplx<R> t3 = (dir < 0) ? cplx<R>{d.y, -d.x} : cplx<R>{-d.y, d.x};
        const int out = b * N + ((j >> logNs) << (logNs + 2)) + k;
        buf[out] = cadd<R>(t0, t2);
        buf[out + Ns] = cadd<R>(t1, t3);
        buf[out + 2 * Ns] = csub<R>(t0, t2);
        buf[out + 3 * Ns] = csub<R>(t1, t3);
      }
    }
    __syncthreads();
  }
  // final radix-2 pass when log2 N is odd
  if (logNs < logN) {
    const int h2 = N >> 1;
    const int nbf = total >> 1;
    cplx<R> v[MAXV / 2][2];
#pragma unroll
    for (int t = 0; t < MAXV / 2; ++t) {
      const int g = threadIdx.x + t * NT;
      if (g < nbf) {
        const int b = g >> (logN - 1);
        const int j = g & (h2 - 1);
        v[t][0] = buf[b * N + j];
        v[t][1] = buf[b * N + j + h2];
      }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < MAXV / 2; ++t) {
      const int g = threadIdx.x + t * NT;
      if (g < nbf) {
        const int b = g >> (logN - 1);
        const int j = g & (h2 - 1);
        const int Ns = 1 << logNs;
        const int k = j & (Ns - 1);
        const int step = kTwiddleN >> (logNs + 1);
        cplx<R> a1 = cmul<R>(v[t][1], twiddle<R>(tw, k * step, dir));
        const int out = b * N + ((j >> logNs) << (logNs + 1)) + k;
        buf[out] = cadd<R>(v[t][0], a1);
        buf[out + Ns] = csub<R>(v[t][0], a1);
      }
    }
    __syncthreads();
  }
}

template <typename R>
constexpr int lds_elems() { return static_cast<int>(kFftLdsBytes / sizeof(cplx<R>)); }

// Rows of n3 reals -> n3/2+1 complex bins.  Pairs (x[2m], x[2m+1]) form a
// half-length complex sequence; its FFT Z gives
//   X[k] = (Z[k] + conj Z[Nh-k]) / 2 - i e^{-2 pi i k/n3} (Z[k] - conj Z[Nh-k]) / 2.
template <typename R>
__global__ __launch_bounds__(kFftThreads) void r2c_rows_kernel(
    const R *__restrict__ in, cplx<R> *__restrict__ out, long long rows, int n3, int logNh,
    int rows_per_wg, const cplx<R> *__restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  cplx<R> *buf = reinterpret_cast<cplx<R> *>(smem_raw);
  const int Nh = n3 >> 1;
  const int h3 = Nh + 1;
  const long long row0 = static_cast<long long>(blockIdx.x) * rows_per_wg;
  const int nb = static_cast<int>(min(static_cast<long long>(rows_per_wg), rows - row0));
  const cplx<R> *src = reinterpret_cast<const cplx<R> *>(in + row0 * n3);
  for (int e = threadIdx.x; e < nb * Nh; e += kFftThreads) buf[e] = src[e];
  __syncthreads();
  lds_fft<R, kFftThreads, lds_elems<R>() / kFftThreads>(buf, Nh, logNh, nb, -1, tw);
  const int step = kTwiddleN / n3;
  for (int e = threadIdx.x; e < nb * h3; e += kFftThreads) {
    const int r = e / h3;
    const int k = e - r * h3;
    const cplx<R> zk = buf[r * Nh + (k == Nh ? 0 : k)];
    const cplx<R> zc = cconj<R>(buf[r * Nh + (k == 0 ? 0 : Nh - k)]);
    const cplx<R> ev = {(zk.x + zc.x) * R(0.5), (zk.y + zc.y) * R(0.5)};
    const cplx<R> od = {(zk.x - zc.x) * R(0.5), (zk.y - zc.y) * R(0.5)};
    const cplx<R> t = cmul<R>(od, twiddle<R>(tw, k * step, -1));
    out[(row0 + r) * h3 + k] = cplx<R>{ev.x + t.y, ev.y - t.x};  // ev - i t
  }
}

// n3/2+1 complex bins -> n3 reals (unnormalised inverse, then * scale, + add).
template <typename R>
__global__ __launch_bounds__(kFftThreads) void c2r_rows_kernel(
    const cplx<R> *__restrict__ in, R *__restrict__ out, const R *__restrict__ add,
    long long rows, int n3, int logNh, int rows_per_wg, R scale,
    const cplx<R> *__restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  cplx<R> *buf = reinterpret_cast<cplx<R> *>(smem_raw);
  const int Nh = n3 >> 1;
  const int h3 = Nh + 1;
  const long long row0 = static_cast<long long>(blockIdx.x) * rows_per_wg;
  const int nb = static_cast<int>(min(static_cast<long long>(rows_per_wg), rows - row0));
  const int step = kTwiddleN / n3;
  for (int e = threadIdx.x; e < nb * Nh; e += kFftThreads) {
    const int r = e / Nh;
    const int k = e - r * Nh;
    const cplx<R> *row = in + (row0 + r) * h3;
    cplx<R> yk = row[k];
    cplx<R> ym = row[Nh - k];
    if (k == 0) {  // the i3 = 0 and i3 = n3/2 bins enter through their real parts only
      yk.y = R(0);
      ym.y = R(0);
    }
    const cplx<R> yc = cconj<R>(ym);
    const cplx<R> a = cadd<R>(yk, yc);
    const cplx<R> b = cmul<R>(csub<R>(yk, yc), twiddle<R>(tw, k * step, +1));
    buf[e] = cplx<R>{a.x - b.y, a.y + b.x};  // a + i b
  }
  __syncthreads();
  lds_fft<R, kFftThreads, lds_elems<R>() / kFftThreads>(buf, Nh, logNh, nb, +1, tw);
  cplx<R> *dst = reinterpret_cast<cplx<R> *>(out + row0 * n3);
  const cplx<R> *addp = add ? reinterpret_cast<const cplx<R> *>(add + row0 * n3) : nullptr;
  for (int e = threadIdx.x; e < nb * Nh; e += kFftThreads) {
    cplx<R> z = buf[e];
    z.x *= scale;
    z.y *= scale;
    if (addp) {
      const cplx<R> s = addp[e];
      z.x += s.x;
      z.y += s.y;
    }
    dst[e] = z;
  }
}

// In-place FFT along n1 of every column of [outer][n1][h3]; a work-group takes
// a tile of up to `tile` adjacent columns of one outer slice.
template <typename R>
__global__ __launch_bounds__(kFftThreads) void col_fft_kernel(
    cplx<R> *__restrict__ data, int n1, int logn1, int h3, int tile, int ntiles, int dir,
    const cplx<R> *__restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  cplx<R> *buf = reinterpret_cast<cplx<R> *>(smem_raw);
  const long long o = blockIdx.x / ntiles;
  const int c0 = (blockIdx.x - static_cast<int>(o) * ntiles) * tile;
  const int tc = min(tile, h3 - c0);
  cplx<R> *base = data + o * static_cast<long long>(n1) * h3 + c0;
  for (int e = threadIdx.x; e < n1 * tc; e += kFftThreads) {
    const int r = e / tc;
    const int c = e - r * tc;
    buf[c * n1 + r] = base[static_cast<long long>(r) * h3 + c];
  }
  __syncthreads();
  lds_fft<R, kFftThreads, lds_elems<R>() / kFftThreads>(buf, n1, logn1, tc, dir, tw);
  for (int e = threadIdx.x; e < n1 * tc; e += kFftThreads) {
    const int r = e / tc;
    const int c = e - r * tc;
    base[static_cast<long long>(r) * h3 + c] = buf[c * n1 + r];
  }
}

int ilog2(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

template <typename R>
hipError_t r2c_impl(const void *in, void *out, long long rows, int n3, const void *tw,
                    hipStream_t st) {
  const int Nh = n3 / 2;
  const int per = max(1, lds_elems<R>() / Nh);
  const long long grid = (rows + per - 1) / per;
  const size_t lds = static_cast<size_t>(per) * Nh * sizeof(cplx<R>);
  hipLaunchKernelGGL(r2c_rows_kernel<R>, dim3(static_cast<unsigned>(grid)), dim3(kFftThreads),
                     lds, st, static_cast<const R *>(in), static_cast<cplx<R> *>(out), rows, n3,
                     ilog2(Nh), per, static_cast<const cplx<R> *>(tw));
  return hipGetLastError();
}

template <typename R>
hipError_t c2r_impl(const void *in, void *out, const void *add, long long rows, int n3,
                    double scale, const void *tw, hipStream_t st) {
  const int Nh = n3 / 2;
  const int per = max(1, lds_elems<R>() / Nh);
  const long long grid = (rows + per - 1) / per;
  const size_t lds = static_cast<size_t>(per) * Nh * sizeof(cplx<R>);
  hipLaunchKernelGGL(c2r_rows_kernel<R>, dim3(static_cast<unsigned>(grid)), dim3(kFftThreads),
                     lds, st, static_cast<const cplx<R> *>(in), static_cast<R *>(out),
                     static_cast<const R *>(add), rows, n3, ilog2(Nh), per, static_cast<R>(scale),
                     static_cast<const cplx<R> *>(tw));
  return hipGetLastError();
}

template <typename R>
hipError_t col_impl(void *data, long long outer, int n1, int h3, int dir, const void *tw,
                    hipStream_t st) {
  const int tile = max(1, min(16, lds_elems<R>() / n1));
  const int ntiles = (h3 + tile - 1) / tile;
  const long long grid = outer * ntiles;
  const size_t lds = static_cast<size_t>(tile) * n1 * sizeof(cplx<R>);
  hipLaunchKernelGGL(col_fft_kernel<R>, dim3(static_cast<unsigned>(grid)), dim3(kFftThreads), lds,
                     st, static_cast<cplx<R> *>(data), n1, ilog2(n1), h3, tile, ntiles, dir,
                     static_cast<const cplx<R> *>(tw));
  return hipGetLastError();
}

}  // namespace

hipError_t launch_r2c_rows(bool fp64, const void *in, void *out, long long rows, int n3,
                           const void *tw, hipStream_t st) {
  return fp64 ? r2c_impl<double>(in, out, rows, n3, tw, st)
              : r2c_impl<float>(in, out, rows, n3, tw, st);
}

hipError_t launch_c2r_rows(bool fp64, const void *in, void *out, const void *add, long long rows,
                           int n3, double scale, const void *tw, hipStream_t st) {
  return fp64 ? c2r_impl<double>(in, out, add, rows, n3, scale, tw, st)
              : c2r_impl<float>(in, out, add, rows, n3, scale, tw, st);
}

hipError_t launch_col_fft(bool fp64, void *data, long long outer, int n1, int h3, int dir,
                          const void *tw, hipStream_t st) {
  return fp64 ? col_impl<double>(data, outer, n1, h3, dir, tw, st)
              : col_impl<float>(data, outer, n1, h3, dir, tw, st);
}

// Twiddles exp(-2 pi i m / 4096), m = 0..4095, from long-double sin/cos on the host.
hipError_t upload_twiddles(bool fp64, void *dst, hipStream_t st) {
  const long double two_pi = 2.0L * 3.141592653589793238462643383279502884L;
  if (fp64) {
    std::vector<double2> t(kTwiddleN);
    for (int m = 0; m < kTwiddleN; ++m) {
      const long double a = two_pi * m / kTwiddleN;
      t[m] = double2{static_cast<double>(cosl(a)), static_cast<double>(-sinl(a))};
    }
    hipError_t e = hipMemcpyAsync(dst, t.data(), t.size() * sizeof(double2), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(st);
  }
  std::vector<float2> t(kTwiddleN);
  for (int m = 0; m < kTwiddleN; ++m) {
    const long double a = two_pi * m / kTwiddleN;
    t[m] = float2{static_cast<float>(cosl(a)), static_cast<float>(-sinl(a))};
  }
  hipError_t e = hipMemcpyAsync(dst, t.data(), t.size() * sizeof(float2), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(st);
}

}  // namespace sbim
