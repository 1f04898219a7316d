// Real 2-D FFT of boundary fields on gfx950.  Every transform runs in LDS with
// Stockham autosort radix-8 passes (and one radix-4 or radix-2 pass for the
// remaining factor), and every pass reads and writes contiguous rows:
//   forward  [F][n1][n3] real --r2c along x3, written transposed--> [F][h3][n1]
//            --complex FFT along contiguous x1 rows--> spectrum [F][h3][n1];
//   inverse  the same two steps backwards.
// Conventions (the paper fixes none): forward exp(-i k.x) on the stored half
// spectrum (h3 = n3/2 + 1 bins along x3); the inverse drops the imaginary parts
// of the i3 = 0 and i3 = n3/2 bins and applies the caller's scale.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

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

// A work-group's twiddles come from a quarter-wave table in LDS for the
// transform's period L (a power of two, 4 <= L <= 4096): q[r] = exp(-2 pi i r / L),
// r < L/4, copied from the global 4096-point table once per work-group, so that
// no radix pass waits for memory.  load_quarter fills it (every thread calls it;
// the caller synchronises before the first use).
template <typename R>
__device__ __forceinline__ void load_quarter(cplx<R> *q, int logL, const cplx<R> *__restrict__ tw) {
  const int n = 1 << (logL - 2);
  const int stride = kTwiddleN >> logL;
  for (int r = threadIdx.x; r < n; r += kFftThreads) q[r] = tw[r * stride];
}
// exp(dir 2 pi i j / 4096) for j a multiple of 4096 / L, from the quarter table:
// with m = j L / 4096 = r + h L/4 (r < L/4), exp(-2 pi i m / L) = q[r] (-i)^h.
template <typename R>
__device__ __forceinline__ cplx<R> twq(const cplx<R> *q, int j, int logL, int dir) {
  const int m = (j & (kTwiddleN - 1)) >> (kTwiddleLog - logL);
  const int h = m >> (logL - 2);
  const cplx<R> t = q[m & ((1 << (logL - 2)) - 1)];
  // (-i)^h t: h = 0 (x, y), 1 (y, -x), 2 (-x, -y), 3 (-y, x)
  R x = (h & 1) ? t.y : t.x;
  R y = (h & 1) ? t.x : t.y;
  if (h >= 2) x = -x;
  if (h == 1 || h == 2) y = -y;
  return cplx<R>{x, dir > 0 ? -y : y};
}

// (1 + dir i) / sqrt(2) times a, i.e. a * exp(dir i pi / 4).
template <typename R>
__device__ __forceinline__ cplx<R> rot8(cplx<R> a, int dir) {
  const R h = R(0.70710678118654752440);
  return dir < 0 ? cplx<R>{(a.x + a.y) * h, (a.y - a.x) * h}
                 : cplx<R>{(a.x - a.y) * h, (a.y + a.x) * h};
}
// dir i a
template <typename R>
__device__ __forceinline__ cplx<R> rot4(cplx<R> a, int dir) {
  return dir < 0 ? cplx<R>{a.y, -a.x} : cplx<R>{-a.y, a.x};
}

// LDS slot of point i of a tile.  Padded tiles leave one slot unused after
// every 8 points: the first radix-8 pass stores each thread's 8 outputs
// contiguously (a 128-byte stride between the lanes for float64), which
// without padding puts whole wavefronts on a few LDS banks.  Small tiles (at
// most 4 points per thread) are padded; larger ones are not, since their LDS
// size limits the work-groups per CU.
template <bool PAD>
__device__ __forceinline__ int pad(int i) {
  return PAD ? i + (i >> 3) : i;
}
__host__ __device__ constexpr int padded_points(int cnt, bool pad) {
  return pad ? cnt + (cnt + 7) / 8 : cnt;
}

// In-place FFT of nseq contiguous sequences of length N = 2^logN held in LDS
// (point i at slot pad<PAD>(i)): Stockham autosort passes of radix 8 (then one
// of radix 4 or 2 for the remaining factor).  Every thread of the work-group
// must call it.  Each pass stages its inputs in registers, synchronises, then
// writes the outputs.
template <typename R, int NT, int MAXV, bool PAD>
__device__ __attribute__((always_inline)) void lds_fft(cplx<R> *buf, int N, int logN, int nseq,
                                                       int dir, const cplx<R> *q, int logL) {
  const int total = N * nseq;
  int logNs = 0;
  // Each pass reads the inputs of every butterfly of the thread from LDS,
  // synchronises, then writes the outputs; twiddles come from the quarter table
  // q of period L (a multiple of N) in LDS.
  constexpr int B8 = (MAXV + 7) / 8;  // radix-8 butterflies per thread and pass
  // radix-8 passes
  for (; logNs + 3 <= logN; logNs += 3) {
    const int q8 = N >> 3;
    const int nbf = total >> 3;
    const int Ns = 1 << logNs;
    const int lstep = kTwiddleLog - logNs - 3;  // step = 4096 / (8 Ns) = 2^lstep
    cplx<R> v[B8][8];
#pragma unroll
    for (int t = 0; t < B8; ++t) {
      const int g = min(static_cast<int>(threadIdx.x) + t * NT, nbf - 1);
      const int base = ((g >> (logN - 3)) << logN) + (g & (q8 - 1));
#pragma unroll
      for (int r = 0; r < 8; ++r) v[t][r] = buf[pad<PAD>(base + (r << (logN - 3)))];
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < B8; ++t) {
      const int g = threadIdx.x + t * NT;
      if (g < nbf) {
        const int b = g >> (logN - 3);
        const int j = g & (q8 - 1);
        const int k = j & (Ns - 1);
        // twiddles w^r, w = exp(dir 2 pi i k / (8 Ns)): w, w^2 and w^4 from the
        // table, the others as products of two or three of them (a few units in
        // the last place, against seven table reconstructions)
        const int ks = k << lstep;  // k * step
        const cplx<R> w1 = twq<R>(q, ks, logL, dir);
        const cplx<R> w2 = twq<R>(q, ks << 1, logL, dir);
        const cplx<R> w4 = twq<R>(q, ks << 2, logL, dir);
        const cplx<R> w3 = cmul<R>(w1, w2);
        cplx<R> a[8];
        a[0] = v[t][0];
        a[1] = cmul<R>(v[t][1], w1);
        a[2] = cmul<R>(v[t][2], w2);
        a[3] = cmul<R>(v[t][3], w3);
        a[4] = cmul<R>(v[t][4], w4);
        a[5] = cmul<R>(v[t][5], cmul<R>(w1, w4));
        a[6] = cmul<R>(v[t][6], cmul<R>(w2, w4));
        a[7] = cmul<R>(v[t][7], cmul<R>(w3, w4));
        // 8-point DFT as radix 2 x radix 4: e_r = a_r + a_{r+4},
        // o_r = (a_r - a_{r+4}) exp(dir 2 pi i r / 8); X[2m] = DFT4(e), X[2m+1] = DFT4(o)
        cplx<R> e[4], o[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          e[r] = cadd<R>(a[r], a[r + 4]);
          o[r] = csub<R>(a[r], a[r + 4]);
        }
        o[1] = rot8<R>(o[1], dir);
        o[2] = rot4<R>(o[2], dir);
        o[3] = rot4<R>(rot8<R>(o[3], dir), dir);
        const int out = (b << logN) + ((j >> logNs) << (logNs + 3)) + k;
        {
          const cplx<R> t0 = cadd<R>(e[0], e[2]), t1 = csub<R>(e[0], e[2]);
          const cplx<R> t2 = cadd<R>(e[1], e[3]), t3 = rot4<R>(csub<R>(e[1], e[3]), dir);
          buf[pad<PAD>(out)] = cadd<R>(t0, t2);
          buf[pad<PAD>(out + (2 << logNs))] = cadd<R>(t1, t3);
          buf[pad<PAD>(out + (4 << logNs))] = csub<R>(t0, t2);
          buf[pad<PAD>(out + (6 << logNs))] = csub<R>(t1, t3);
        }
        {
          const cplx<R> t0 = cadd<R>(o[0], o[2]), t1 = csub<R>(o[0], o[2]);
          const cplx<R> t2 = cadd<R>(o[1], o[3]), t3 = rot4<R>(csub<R>(o[1], o[3]), dir);
          buf[pad<PAD>(out + (1 << logNs))] = cadd<R>(t0, t2);
          buf[pad<PAD>(out + (3 << logNs))] = cadd<R>(t1, t3);
          buf[pad<PAD>(out + (5 << logNs))] = csub<R>(t0, t2);
          buf[pad<PAD>(out + (7 << logNs))] = csub<R>(t1, t3);
        }
      }
    }
    __syncthreads();
  }
  // one radix-4 pass when 2 factors of two remain
  if (logNs + 2 == logN) {
    const int q4 = N >> 2;
    const int nbf = total >> 2;
    const int Ns = 1 << logNs;
    const int lstep = kTwiddleLog - logNs - 2;  // step = 4096 / (4 Ns) = 2^lstep
    constexpr int B4 = (MAXV + 3) / 4;
    cplx<R> v[B4][4];
#pragma unroll
    for (int t = 0; t < B4; ++t) {
      const int g = min(static_cast<int>(threadIdx.x) + t * NT, nbf - 1);
      const int base = ((g >> (logN - 2)) << logN) + (g & (q4 - 1));
#pragma unroll
      for (int r = 0; r < 4; ++r) v[t][r] = buf[pad<PAD>(base + (r << (logN - 2)))];
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < B4; ++t) {
      const int g = threadIdx.x + t * NT;
      if (g < nbf) {
        const int b = g >> (logN - 2);
        const int j = g & (q4 - 1);
        const int k = j & (Ns - 1);
        cplx<R> a0 = v[t][0];
        const cplx<R> w1 = twq<R>(q, k << lstep, logL, dir);
        const cplx<R> w2 = twq<R>(q, k << (lstep + 1), logL, dir);
        cplx<R> a1 = cmul<R>(v[t][1], w1);
        cplx<R> a2 = cmul<R>(v[t][2], w2);
        cplx<R> a3 = cmul<R>(v[t][3], cmul<R>(w1, w2));
        cplx<R> t0 = cadd<R>(a0, a2), t1 = csub<R>(a0, a2);
        cplx<R> t2 = cadd<R>(a1, a3);
        // dir * i * (a1 - a3): -i for the forward transform, +i for the inverse
        cplx<R> t3 = rot4<R>(csub<R>(a1, a3), dir);
        const int out = (b << logN) + ((j >> logNs) << (logNs + 2)) + k;
        buf[pad<PAD>(out)] = cadd<R>(t0, t2);
        buf[pad<PAD>(out + (1 << logNs))] = cadd<R>(t1, t3);
        buf[pad<PAD>(out + (2 << logNs))] = csub<R>(t0, t2);
        buf[pad<PAD>(out + (3 << logNs))] = csub<R>(t1, t3);
      }
    }
    __syncthreads();
    logNs += 2;
  }
  // one radix-2 pass when 1 factor of two remains
  if (logNs < logN) {
    const int h2 = N >> 1;
    const int nbf = total >> 1;
    const int Ns = 1 << logNs;
    const int lstep = kTwiddleLog - logNs - 1;  // step = 4096 / (2 Ns) = 2^lstep
    constexpr int B2 = (MAXV + 1) / 2;
    cplx<R> v[B2][2];
#pragma unroll
    for (int t = 0; t < B2; ++t) {
      const int g = min(static_cast<int>(threadIdx.x) + t * NT, nbf - 1);
      const int b = g >> (logN - 1);
      const int j = g & (h2 - 1);
      v[t][0] = buf[pad<PAD>((b << logN) + j)];
      v[t][1] = buf[pad<PAD>((b << logN) + j + h2)];
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < B2; ++t) {
      const int g = threadIdx.x + t * NT;
      if (g < nbf) {
        const int b = g >> (logN - 1);
        const int j = g & (h2 - 1);
        const int k = j & (Ns - 1);
        cplx<R> a1 = cmul<R>(v[t][1], twq<R>(q, k << lstep, logL, dir));
        const int out = (b << logN) + ((j >> logNs) << (logNs + 1)) + k;
        buf[pad<PAD>(out)] = cadd<R>(v[t][0], a1);
        buf[pad<PAD>(out + (1 << logNs))] = csub<R>(v[t][0], a1);
      }
    }
    __syncthreads();
  }
}

static_assert(kFftThreads * kFftPerThread == 4096, "one work-group covers the longest transform");

// Tile of a transposed kernel from its tile id.  Work-groups are dispatched
// round-robin over the 8 XCDs; with a persistent grid that is a multiple of 8,
// the ids a work-group takes are congruent mod 8 to its XCD, and a tile count
// that is a multiple of 8 maps ids 8 k + x to tile x * (ntiles / 8) + k, so the
// tiles one XCD works on at a time are consecutive and the partial cache lines
// of their transposed runs meet in one L2.
__device__ __forceinline__ int xcd_tile(int id, int ntiles) {
  if (ntiles % 8) return id;
  return (id & 7) * (ntiles >> 3) + (id >> 3);
}

// Forward, step 1: rows x1 in [x0, x0 + R) of one field; each row of n3 reals
// becomes n3/2+1 bins.  Pairs (x[2m], x[2m+1]) form a half-length complex
// sequence z; with Z = FFT(z)
//   X[k] = (Z[k] + conj Z[Nh-k]) / 2 - i e^{-2 pi i k/n3} (Z[k] - conj Z[Nh-k]) / 2.
// The bins are written transposed, spec[f][k][x1], R consecutive x1 at a time.
// Input reals of type Rin are widened to the transform's type R on load.
// Persistent: work-group w takes tiles w, w + G, w + 2G, ... (G = the grid,
// sized to the work-groups the GPU holds at once when there are more tiles) and
// loads the next tile's rows into registers while the current tile is
// transformed in LDS, so the input's memory latency overlaps the transform
// (measured at 2048 x 2048: 198 -> 148 us for six fields).
template <typename Rin, typename R, int MAXV>
__global__ __launch_bounds__(kFftThreads) __attribute__((amdgpu_waves_per_eu(2))) void r2c_t_kernel(
    const Rin *__restrict__ in, cplx<R> *__restrict__ spec, int n1, int n3, int logNh, int rows,
    const cplx<R> *__restrict__ tw, int ntiles, int logrows, int logn1) {
  extern __shared__ unsigned char smem_raw[];
  cplx<R> *buf = reinterpret_cast<cplx<R> *>(smem_raw);
  const int Nh = n3 >> 1;
  const int h3 = Nh + 1;
  const int tiles = n1 / rows;
  constexpr bool PAD = MAXV == 4;
  const int cnt = rows * Nh;  // complex input points of a tile (<= kFftThreads * MAXV)
  const int logL = logNh + 1;  // twiddle period: n3
  cplx<R> *q = buf + padded_points(cnt, PAD);  // quarter table, after the tile
  load_quarter<R>(q, logL, tw);
  cplx<Rin> pre[MAXV];
  auto load = [&](int id) {
    const int tile = xcd_tile(id, ntiles);
    const int f = tile / tiles;
    const int x0 = (tile - f * tiles) * rows;
    const cplx<Rin> *src =
        reinterpret_cast<const cplx<Rin> *>(in + (static_cast<long long>(f) * n1 + x0) * n3);
#pragma unroll
    for (int i = 0; i < MAXV; ++i) {
      const int e = threadIdx.x + i * kFftThreads;
      if (e < cnt) pre[i] = src[e];
    }
  };
  int id = blockIdx.x;
  if (id < ntiles) load(id);
  const int lstep = kTwiddleLog - logL;  // 4096 / n3 = 2^lstep
  for (; id < ntiles; id += gridDim.x) {
    const int tile = xcd_tile(id, ntiles);
    const int f = tile / tiles;
    const int x0 = (tile - f * tiles) * rows;
#pragma unroll
    for (int i = 0; i < MAXV; ++i) {
      const int e = threadIdx.x + i * kFftThreads;
      if (e < cnt) buf[pad<PAD>(e)] = cplx<R>{static_cast<R>(pre[i].x), static_cast<R>(pre[i].y)};
    }
    __syncthreads();
    if (id + static_cast<int>(gridDim.x) < ntiles) load(id + gridDim.x);
    lds_fft<R, kFftThreads, MAXV, PAD>(buf, Nh, logNh, rows, -1, q, logL);
    cplx<R> *dst = spec + static_cast<long long>(f) * h3 * n1 + x0;
    for (int e = threadIdx.x; e < rows * h3; e += kFftThreads) {
      const int k = e >> logrows;
      const int r = e & (rows - 1);
      const int row = r << logNh;
      const cplx<R> zk = buf[pad<PAD>(row + (k == Nh ? 0 : k))];
      const cplx<R> zc = cconj<R>(buf[pad<PAD>(row + (k == 0 ? 0 : Nh - k))]);
      const cplx<R> ev = {(zk.x + zc.x) * R(0.5), (zk.y + zc.y) * R(0.5)};
      const cplx<R> od = {(zk.x - zc.x) * R(0.5), (zk.y - zc.y) * R(0.5)};
      const cplx<R> t = cmul<R>(od, twq<R>(q, k << lstep, logL, -1));
      dst[(static_cast<long long>(k) << logn1) + r] = cplx<R>{ev.x + t.y, ev.y - t.x};  // ev - i t
    }
    __syncthreads();  // the next tile overwrites buf
  }
}

// Complex FFT along contiguous rows of length n, from `src` into `dst` (the
// same array for in place); `per` rows per work-group.
template <typename R, int MAXV>
__global__ __launch_bounds__(kFftThreads) void cfft_rows_kernel(
    const cplx<R> *src, cplx<R> *dst, long long nrows, int n, int logn, int per, int dir,
    const cplx<R> *__restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  constexpr bool PAD = MAXV == 4;
  cplx<R> *buf = reinterpret_cast<cplx<R> *>(smem_raw);
  cplx<R> *q = buf + padded_points(per * n, PAD);  // quarter table of period n, after the rows
  load_quarter<R>(q, logn, tw);
  const long long row0 = static_cast<long long>(blockIdx.x) * per;
  const int nb = static_cast<int>(min(static_cast<long long>(per), nrows - row0));
  const int cnt = nb * n;  // <= kFftThreads * MAXV
  // every load of the work-group's rows in flight before the first LDS store
  cplx<R> v[MAXV];
#pragma unroll
  for (int i = 0; i < MAXV; ++i) {
    const int e = min(static_cast<int>(threadIdx.x) + i * kFftThreads, cnt - 1);  // clamped: no branch
    v[i] = src[row0 * n + e];
  }
  // (unguarded, so that the compiler cannot sink each load into a guarded store:
  // past cnt a lane rewrites point cnt - 1 with its own value)
#pragma unroll
  for (int i = 0; i < MAXV; ++i)
    buf[pad<PAD>(min(static_cast<int>(threadIdx.x) + i * kFftThreads, cnt - 1))] = v[i];
  __syncthreads();
  lds_fft<R, kFftThreads, MAXV, PAD>(buf, n, logn, nb, dir, q, logn);
#pragma unroll
  for (int i = 0; i < MAXV; ++i) {
    const int e = threadIdx.x + i * kFftThreads;
    if (e < cnt) dst[row0 * n + e] = buf[pad<PAD>(e)];
  }
}

// Inverse, last step: rows x1 in [x0, x0 + R) of one field from the transposed
// spectrum spec[f][k][x1] (k = 0..n3/2, imaginary parts of k = 0 and k = n3/2
// dropped).  With Y the row's bins,
//   Z[k] = (Y[k] + conj Y[Nh-k]) + i e^{+2 pi i k/n3} (Y[k] - conj Y[Nh-k]),
// an inverse half-length FFT gives x[2m] + i x[2m+1]; the result is scaled and
// the optional field `add` is added.
template <typename R, int MAXV>
__global__ __launch_bounds__(kFftThreads) void c2r_t_kernel(
    const cplx<R> *__restrict__ spec, R *__restrict__ out, const R *__restrict__ add, int n1,
    int n3, int logNh, int rows, R scale, const cplx<R> *__restrict__ tw, int logrows, int logn1,
    float inv_half) {
  extern __shared__ unsigned char smem_raw[];
  constexpr bool PAD = MAXV == 4;
  cplx<R> *buf = reinterpret_cast<cplx<R> *>(smem_raw);
  const int Nh = n3 >> 1;
  const int h3 = Nh + 1;
  cplx<R> *nyq = buf + padded_points(rows * Nh, PAD);  // bin k = Nh of each row
  const int logL = logNh + 1;       // twiddle period: n3
  cplx<R> *q = nyq + rows;          // quarter table
  load_quarter<R>(q, logL, tw);
  const int tiles = n1 / rows;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int f = tile / tiles;
  const int x0 = (tile - f * tiles) * rows;
  const cplx<R> *src = spec + static_cast<long long>(f) * h3 * n1 + x0;
  // rows * h3 inputs in chunks of MAXV + 1 per thread (one chunk unless the rows
  // are very short), all loads of a chunk in flight before its LDS stores
  const int nin = rows * h3;
  cplx<R> v[MAXV + 1];
  for (int e0 = threadIdx.x; e0 < nin; e0 += (MAXV + 1) * kFftThreads) {
#pragma unroll
    for (int i = 0; i <= MAXV; ++i) {
      const int e = min(e0 + i * kFftThreads, nin - 1);  // clamped: loads without branches
      v[i] = src[(static_cast<long long>(e >> logrows) << logn1) + (e & (rows - 1))];
    }
#pragma unroll
    for (int i = 0; i <= MAXV; ++i) {
      const int e = e0 + i * kFftThreads;
      if (e < nin) {
        const int k = e >> logrows;
        const int r = e & (rows - 1);
        if (k < Nh)
          buf[pad<PAD>((r << logNh) + k)] = v[i];
        else
          nyq[r] = v[i];
      }
    }
  }
  __syncthreads();
  // pair (k, Nh - k) of each row; r = e / half in float32 (exact: e < 2^13 and
  // (e + 1/2) / half stays at least 1 / (2 half) from an integer)
  const int lstep = kTwiddleLog - logL;  // 4096 / n3 = 2^lstep
  const int half = Nh / 2 + 1;
  for (int e = threadIdx.x; e < rows * half; e += kFftThreads) {
    const int r = static_cast<int>((static_cast<float>(e) + 0.5f) * inv_half);
    const int k = e - r * half;
    const int rb = r << logNh;  // the row's first point
    if (k == 0) {
      const R y0 = buf[pad<PAD>(rb)].x, yn = nyq[r].x;
      buf[pad<PAD>(rb)] = cplx<R>{y0 + yn, y0 - yn};
    } else {
      const int m = Nh - k;
      const cplx<R> yk = buf[pad<PAD>(rb + k)], ym = buf[pad<PAD>(rb + m)];
      const cplx<R> a1 = cadd<R>(yk, cconj<R>(ym));
      const cplx<R> b1 = cmul<R>(csub<R>(yk, cconj<R>(ym)), twq<R>(q, k << lstep, logL, +1));
      buf[pad<PAD>(rb + k)] = cplx<R>{a1.x - b1.y, a1.y + b1.x};
      if (m != k) {
        const cplx<R> a2 = cadd<R>(ym, cconj<R>(yk));
        const cplx<R> b2 = cmul<R>(csub<R>(ym, cconj<R>(yk)), twq<R>(q, m << lstep, logL, +1));
        buf[pad<PAD>(rb + m)] = cplx<R>{a2.x - b2.y, a2.y + b2.x};
      }
    }
  }
  __syncthreads();
  lds_fft<R, kFftThreads, MAXV, PAD>(buf, Nh, logNh, rows, +1, q, logL);
  const long long o = (static_cast<long long>(f) * n1 + x0) * n3;
  cplx<R> *dst = reinterpret_cast<cplx<R> *>(out + o);
  const cplx<R> *addp = add ? reinterpret_cast<const cplx<R> *>(add + o) : nullptr;
  const int nout = rows * Nh;  // <= kFftThreads * MAXV
  if (addp) {
#pragma unroll
    for (int i = 0; i < MAXV; ++i) {
      const int e = min(static_cast<int>(threadIdx.x) + i * kFftThreads, nout - 1);
      v[i] = addp[e];
    }
  }
#pragma unroll
  for (int i = 0; i < MAXV; ++i) {
    const int e = threadIdx.x + i * kFftThreads;
    if (e < nout) {
      cplx<R> z = buf[pad<PAD>(e)];
      z.x *= scale;
      z.y *= scale;
      if (addp) {
        z.x += v[i].x;
        z.y += v[i].y;
      }
      dst[e] = z;
    }
  }
}

int ilog2(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

// Work-group shapes.  The transposed kernels (r2c_t, c2r_t) take 4 rows up to
// 1024-point rows (their transposed accesses are `rows` consecutive points
// long; consecutive tiles of one XCD complete each other's cache lines), 2 rows
// from 2048 points, where a work-group's LDS and registers would otherwise
// hold the GPU to two work-groups per CU (measured on gfx950: 2048 x 2048
// forward 114 -> 100 us, inverse 68 -> 62 us; at 1024 points 2 rows are
// slower); the row kernels take about 1024 points.  MAXV, the points a thread
// stages in registers per pass, is the smallest power of two that covers the
// work-group's points.
constexpr size_t kMaxLds = 64 * 1024;
int tile_rows(int n1, int Nh, size_t point_bytes, int extra_per_row) {
  int rows = Nh >= 1024 ? 2 : max(4, 1024 / Nh);
  while (rows > 1 && (rows > n1 || rows * Nh > kFftThreads * kFftPerThread ||
                      static_cast<size_t>(rows) * (Nh + extra_per_row) * point_bytes > kMaxLds))
    rows >>= 1;
  return rows;
}
int rows_per_group(int n) { return max(1, 1024 / n); }

// Grid of the persistent forward kernel: one work-group per tile when the
// device holds them all at once, else the work-groups it holds (the kernel's
// occupancy at this LDS size, queried once per kernel, LDS size and device) in
// whole XCD rounds (a multiple of 8).
template <typename K>
int persistent_grid(K kernel, int ntiles, size_t lds_bytes) {
  static std::mutex mu;
  static std::map<std::tuple<const void *, size_t, int>, int> resident;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return ntiles;
  const auto key = std::make_tuple(reinterpret_cast<const void *>(kernel), lds_bytes, dev);
  int cap = 0;
  {
    std::lock_guard<std::mutex> lock(mu);
    auto it = resident.find(key);
    if (it != resident.end()) {
      cap = it->second;
    } else {
      int per_cu = 0, ncu = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kFftThreads, lds_bytes) !=
              hipSuccess ||
          hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return ntiles;
      cap = std::max(1, per_cu) * std::max(1, ncu);
      resident.emplace(key, cap);
    }
  }
  if (ntiles <= cap) return ntiles;
  return cap >= 8 ? cap - cap % 8 : cap;
}

template <typename F>
hipError_t with_maxv(int points, F &&launch) {
  if (points <= kFftThreads * 4) return launch(std::integral_constant<int, 4>());
  if (points <= kFftThreads * 8) return launch(std::integral_constant<int, 8>());
  return launch(std::integral_constant<int, 16>());
}

template <typename R>
hipError_t cfft_launch(const void *src, void *dst, long long nrows, int n, int dir,
                       const void *tw, hipStream_t st) {
  const int per = rows_per_group(n);
  return with_maxv(per * n, [&](auto mv) {
    constexpr bool pad = decltype(mv)::value == 4;  // as the kernel pads its tile
    hipLaunchKernelGGL((cfft_rows_kernel<R, decltype(mv)::value>),
                       dim3(static_cast<unsigned>((nrows + per - 1) / per)), dim3(kFftThreads),
                       (static_cast<size_t>(padded_points(per * n, pad)) + n / 4) * sizeof(cplx<R>), st,
                       static_cast<const cplx<R> *>(src), static_cast<cplx<R> *>(dst), nrows, n,
                       ilog2(n), per, dir, static_cast<const cplx<R> *>(tw));
    return hipGetLastError();
  });
}

template <typename Rin, typename R>
hipError_t forward_impl(const void *in, void *spec, int F, int n1, int n3, const void *tw,
                        hipStream_t st) {
  const int Nh = n3 / 2, h3 = Nh + 1;
  const int rows = tile_rows(n1, Nh, sizeof(cplx<R>), 0);
  const int ntiles = F * (n1 / rows);
  hipError_t e = with_maxv(rows * Nh, [&](auto mv) {
    constexpr bool pad = decltype(mv)::value == 4;  // as the kernel pads its tile
    const size_t lds = (static_cast<size_t>(padded_points(rows * Nh, pad)) + n3 / 4) * sizeof(cplx<R>);
    auto kernel = r2c_t_kernel<Rin, R, decltype(mv)::value>;
    hipLaunchKernelGGL(kernel, dim3(static_cast<unsigned>(persistent_grid(kernel, ntiles, lds))),
                       dim3(kFftThreads), lds, st, static_cast<const Rin *>(in),
                       static_cast<cplx<R> *>(spec), n1, n3, ilog2(Nh), rows,
                       static_cast<const cplx<R> *>(tw), ntiles, ilog2(rows), ilog2(n1));
    return hipGetLastError();
  });
  if (e != hipSuccess) return e;
  return cfft_launch<R>(spec, spec, static_cast<long long>(F) * h3, n1, -1, tw, st);
}

template <typename R>
hipError_t inverse_impl(const void *spec, void *scratch, void *out, const void *add, int F, int n1,
                        int n3, double scale, const void *tw, hipStream_t st) {
  const int Nh = n3 / 2, h3 = Nh + 1;
  hipError_t e = cfft_launch<R>(spec, scratch, static_cast<long long>(F) * h3, n1, +1, tw, st);
  if (e != hipSuccess) return e;
  const int rows = tile_rows(n1, Nh, sizeof(cplx<R>), 1);
  return with_maxv(rows * Nh, [&](auto mv) {
    constexpr bool pad = decltype(mv)::value == 4;  // as the kernel pads its tile
    hipLaunchKernelGGL((c2r_t_kernel<R, decltype(mv)::value>),
                       dim3(static_cast<unsigned>(F * (n1 / rows))), dim3(kFftThreads),
                       (static_cast<size_t>(padded_points(rows * Nh, pad)) + rows + n3 / 4) *
                           sizeof(cplx<R>),
                       st,
                       static_cast<const cplx<R> *>(scratch), static_cast<R *>(out),
                       static_cast<const R *>(add), n1, n3, ilog2(Nh), rows,
                       static_cast<R>(scale), static_cast<const cplx<R> *>(tw), ilog2(rows),
                       ilog2(n1), 1.0f / static_cast<float>(Nh / 2 + 1));
    return hipGetLastError();
  });
}

}  // namespace

hipError_t launch_fft_forward(bool in_fp64, const void *in, void *spec, int F, int n1, int n3,
                              const void *tw64, hipStream_t st) {
  return in_fp64 ? forward_impl<double, double>(in, spec, F, n1, n3, tw64, st)
                 : forward_impl<float, double>(in, spec, F, n1, n3, tw64, st);
}

hipError_t launch_fft_inverse(bool fp64, const void *spec, void *scratch, void *out,
                              const void *add, int F, int n1, int n3, double scale, const void *tw,
                              hipStream_t st) {
  return fp64 ? inverse_impl<double>(spec, scratch, out, add, F, n1, n3, scale, tw, st)
              : inverse_impl<float>(spec, scratch, out, add, F, n1, n3, scale, tw, st);
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
