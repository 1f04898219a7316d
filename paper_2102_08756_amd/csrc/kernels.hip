// Mode-space kernels of the boundary-integral step on gfx950:
//   step_kernel      two kinds of items in one launch per step:
//                    mode items: the push (rotate the new spectrum into the
//                    wavevector frame, update the float64 running state, store
//                    the history ring slot) and, from the same registers, the
//                    traction of the step (pending history sum plus the newest
//                    lags, damping and instantaneous terms of Eq. SBI, Sec. 2.3,
//                    rotation back to (x1, x2, x3));
//                    sweep items: the truncated history convolution (the
//                    nonlocal term of Eq. SBI), one pass over a block's history
//                    serving the next several steps;
//   tabulate_kernel  float64 quadrature of the per-lag kernel weights.
//
// Layouts (one material group; modes sorted by (W desc, q asc), 64 per block):
//   ring    [record][plane][component L,N,T][64 lanes] complex.  Step n of
//           block b lives in record blk_off[b] + (n mod blk_cap[b]) * blk_stride[b]:
//           consecutive blocks of one sweep phase (b mod depth) with equal
//           capacity form a run laid out slot-major (stride = run length), so
//           one history slot of a run is contiguous;
//   table   class-major rows: entry cls_off[class] + j holds (w11, w12, w22, w33)
//           of lag j, j < W of the class.
#include <cmath>
#include <type_traits>

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
  __device__ __forceinline__ R value() const { return s; }
  // add the accumulator of the lane `off` lanes away (butterfly reduction)
  __device__ __forceinline__ void fold_lane(int off) { s += __shfl_xor(s, off); }
};
template <> struct Acc<float, true> {
  float s = 0.f, c = 0.f;
  // Kahan's compensated addition (c holds the part of the sum lost by s)
  __device__ __forceinline__ void fold(float x) {
    const float y = x + c;
    const float t = s + y;
    c = y - (t - s);
    s = t;
  }
  __device__ __forceinline__ float value() const { return s + c; }
  __device__ __forceinline__ void fold_lane(int off) {
    const float s2 = __shfl_xor(s, off);
    const float c2 = __shfl_xor(c, off);
    neumaier(s, c, s2);
    c += c2;
  }
};

// Five complex history sums per plane: C11[U_L], C12[U_N], C22[U_N], C12[U_L], C33[U_T].
constexpr int kSums = 10;  // real accumulators per plane

// part[.] += w * u for the five history sums of one plane.
template <typename R>
__device__ __forceinline__ void fma_lag(R (&part)[kSums], const typename W4<R>::T &w,
                                        const cplx<R> (&u)[3]) {
  part[0] = fma(w.x, u[0].x, part[0]);
  part[1] = fma(w.x, u[0].y, part[1]);
  part[2] = fma(w.y, u[1].x, part[2]);
  part[3] = fma(w.y, u[1].y, part[3]);
  part[4] = fma(w.z, u[1].x, part[4]);
  part[5] = fma(w.z, u[1].y, part[5]);
  part[6] = fma(w.y, u[0].x, part[6]);
  part[7] = fma(w.y, u[0].y, part[7]);
  part[8] = fma(w.w, u[2].x, part[8]);
  part[9] = fma(w.w, u[2].y, part[9]);
}

// History entries whose loads the sweep issues together (measured on gfx950,
// 512x512 x 2 planes, W = 1000): float32 at depth 8, float64 and the
// compensated form fit one more wavefront per SIMD with pairs.
template <typename R, int S, bool COMP> constexpr int sweep_group() {
  constexpr int g = (COMP || sizeof(R) == 8 || S >= 8) ? 2 : 4;
  return S % g == 0 ? g : (S % 2 == 0 ? 2 : 1);  // a divisor of the span
}

// Lag chunks per sweep wavefront (measured on gfx950, 512x512 and 1024x1024 x
// 2 planes, W = 1000 and 2000): four for float32 with one lane per mode (16
// modes x 4 chunks, three wavefronts per SIMD), two otherwise (float64 and the
// compensated form: 32 modes x 2 chunks, 256-byte segments of float32 pairs;
// with two lanes per mode 16 modes x 2 x 2 in every form).  Depth 6 is the
// short-window sweep (mean window under 64 lags): one chunk of 64 modes, as
// chunks of whole spans would mostly pass the windows' ends (2048x2048 x 2,
// per-mode windows of mean 18 lags: 0.85 -> 0.80 ms per step).
template <typename R, int S, int T, bool COMP> constexpr int sweep_lag_groups() {
  if (S == 6 && T == 1) return 1;
  return (COMP || sizeof(R) == 8 || T > 1) ? 2 : 4;
}

// Rows k0 .. k0+S-1 of a mode's kernel.  A class's W rows are followed by a
// zero row, so clamping the lag to W gives zero from the window on.
template <typename R, int S>
__device__ __forceinline__ void load_rows(typename W4<R>::T (&w)[S],
                                          const typename W4<R>::T *__restrict__ rowp, int k0,
                                          int wl) {
#pragma unroll
  for (int k = 0; k < S; ++k) w[k] = rowp[min(k0 + k, wl)];
}

// sums[s] += products of S consecutive history entries (lags i .. i+S-1) with
// rows i+s .. i+s+S-1, the rows held as A = rows i .. i+S-1 and
// B = rows i+S .. i+2S-1.  hp / x point at the ring record / slot of lag i
// and are advanced past lag i+S-1.
template <typename R, int S, int G>
__device__ __forceinline__ void sweep_span(R (&sums)[S][kSums], const typename W4<R>::T (&A)[S],
                                           const typename W4<R>::T (&B)[S],
                                           const cplx<R> *__restrict__ &hp, int &x, int cap,
                                           long long dstep, long long dwrap) {
  static_assert(S % G == 0, "load groups must tile the span");
  typedef R nv2 __attribute__((ext_vector_type(2)));
#pragma unroll
  for (int g0 = 0; g0 < S; g0 += G) {
    cplx<R> u[G][3];
#pragma unroll
    for (int t = 0; t < G; ++t) {
      // the history is read once per sweep: non-temporal loads keep it from
      // displacing the kernel rows in the caches
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const nv2 v = __builtin_nontemporal_load(reinterpret_cast<const nv2 *>(hp + c * kLanes));
        u[t][c] = cplx<R>{v.x, v.y};
      }
      const bool wrap = x == 0;  // next older slot
      hp += wrap ? dwrap - dstep : -dstep;
      x = wrap ? cap - 1 : x - 1;
    }
#pragma unroll
    for (int t = 0; t < G; ++t)
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int k = g0 + t + s;
        fma_lag<R>(sums[s], k < S ? A[k] : B[k - S], u[t]);
      }
  }
}

// The sweep launched with step n serves steps t0 = n+1 .. n+D (depth D = S T).
// Blocks of phase t0 mod D read their history up to step n-1 once, U^{t0-i}
// for i = 2 .. min(cap-1, t0), and form for each of those steps t0+u its sum
// over that history:
//   pending[(t0+u) mod (D+1)] = sum_{i>=2} w_{i+u} (x) U^{t0-i}   (lags i+u inside the window).
// It reads neither U^n nor the pending sum of step n, so it runs in the same
// launch as the push and traction of step n (D+1 pending slots keep step n's
// sum apart from the D being written).
// Each history entry thus serves D steps.  A lane holds the sums of S of
// them (registers bound S); T lanes per mode and lag chunk take the D steps
// in groups u = g S + s, g < T.  They load the same history entries in the
// same instructions, so each entry is fetched from memory once for all D
// steps.  The kernel rows i+gS .. i+gS+2S-2 that a span of S entries needs are
// held in two register arrays used in turn, so each row is loaded once per
// lane and never moved.
//
// Lag chunks are whole spans long, so chunks never overlap and no lane needs a
// mask: chunks reach past the last entry by less than LG spans, and a lag
// i > min(cap-1, t0) either meets zero kernel rows (i + s >= cap >= W) or a
// ring slot not written since the last reset, which holds zero (the slot that
// the concurrent push writes is lag 1 or cap+1, whose rows are unused or zero).
//
// Work item (one wavefront) = (block of the phase, plane, group of Q of the
// block's 64 modes).  Its 64 lanes are Q modes x T step groups x LG lag
// chunks (Q = 64 / (T LG)): lane l takes mode l mod Q of the group, step
// group (l / Q) mod T and chunk l / (Q T) of the lags, so each history load
// fetches LG segments of Q x 8 bytes (float32), one per chunk.  The chunks
// are then summed by a butterfly over lanes l ^ QT, l ^ 2QT, ... (fixed
// order, so the result is bitwise reproducible).
template <typename R, int S, int T, bool COMP>
__device__ __forceinline__ void sweep_item(const SweepArgs &a, long long item) {
  using W = typename W4<R>::T;
  const cplx<R> *__restrict__ ring = static_cast<const cplx<R> *>(a.ring);
  const W *__restrict__ table = static_cast<const W *>(a.table);
  R *__restrict__ pending = static_cast<R *>(a.pending);
  const long long M = a.M, step = a.step;
  const int np = a.np;
  constexpr int LG = sweep_lag_groups<R, S, T, COMP>();
  constexpr int Q = kLanes / (LG * T);  // modes per item
  constexpr int NQ = kLanes / Q;        // items per block and plane
  constexpr int D = S * T;
  // Items of one block get ids congruent mod 8, so they run on one XCD and
  // share the block's kernel rows in its L2.
  const int per_blk = NQ * np;
  const long long kb = (item / (8LL * per_blk)) * 8 + (item & 7);
  if (kb >= a.nphase) return;
  const int r = static_cast<int>((item >> 3) % per_blk);
  const int p = r / NQ;
  const long long t0 = step + 1;
  const long long b = t0 % D + D * kb;
  const int lane = threadIdx.x;
  const int lg = lane / (Q * T);
  const int u0 = (lane / Q) % T * S;        // first of the lane's S steps (t0 + u0 ..)
  const int col = (r % NQ) * Q + lane % Q;  // lane of the mode in its block
  const long long sm = b * kLanes + col;
  const bool valid = sm < M;
  const int cap = a.blk_cap[b];
  // history entries (lags 2 .. min(cap-1, t0) of step t0) that the window can reach
  const int nent = static_cast<int>(max(0LL, min(static_cast<long long>(cap) - 1, t0) - 1));
  const int wl = valid ? a.win[sm] : 0;
  const int cl = valid ? a.cls[sm] : 0;
  const int per = (nent + LG * S - 1) / (LG * S) * S;  // lags per chunk
  const int i0 = 2 + lg * per;

  constexpr int G = sweep_group<R, S, COMP>();
  // plain form: the running sums; compensated form: the products since the
  // last fold into the compensated accumulators (up to 6S lags, three span pairs)
  R sums[S][kSums];
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int k = 0; k < kSums; ++k) sums[s][k] = R(0);
  Acc<R, COMP> acc[S][kSums];
  if (per > 0) {  // then cap > 2, so the block has a mode with W > 0 and class 0 exists
    const long long rec_len = static_cast<long long>(np) * 3 * kLanes;
    const long long dstep = a.blk_stride[b] * rec_len;  // elements between consecutive slots
    const long long dwrap = static_cast<long long>(cap) * dstep;
    // ring slot of lag i0 of step t0 (i0 may pass t0)
    int x = static_cast<int>((((t0 - i0) % cap) + cap) % cap);
    const cplx<R> *hp = ring +
                        (a.blk_off[b] + static_cast<long long>(x) * a.blk_stride[b]) * rec_len +
                        static_cast<long long>(p) * 3 * kLanes + col;
    // a mode without history (W = 0) reads the zero row after class 0's rows
    const W *rowp = wl > 0 ? table + a.cls_off[cl] : table + a.cls_off[0] + a.cls_w0;
    W ra[S], rb[S];
    load_rows<R, S>(ra, rowp, i0 + u0, wl);
    for (int it = 0; it < per; it += 2 * S) {
      const int i = i0 + u0 + it;
      load_rows<R, S>(rb, rowp, i + S, wl);
      sweep_span<R, S, G>(sums, ra, rb, hp, x, cap, dstep, dwrap);
      if (it + S >= per) break;
      load_rows<R, S>(ra, rowp, i + 2 * S, wl);
      sweep_span<R, S, G>(sums, rb, ra, hp, x, cap, dstep, dwrap);
      // compensated form: fold the plain partial sums of the last 6S lags
      // (every third pass of this loop; the branch is uniform over the wavefront)
      if constexpr (COMP) {
        if ((it / (2 * S)) % 3 == 2) {
#pragma unroll
          for (int s = 0; s < S; ++s)
#pragma unroll
            for (int k = 0; k < kSums; ++k) {
              acc[s][k].fold(sums[s][k]);
              sums[s][k] = R(0);
            }
        }
      }
    }
  }
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int k = 0; k < kSums; ++k) acc[s][k].fold(sums[s][k]);
  // sum the lag chunks of each mode; lanes of chunk 0 store
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const long long slot = (t0 + u0 + s) % (D + 1);
#pragma unroll
    for (int k = 0; k < kSums; ++k) {
#pragma unroll
      for (int off = Q * T; off < kLanes; off <<= 1) acc[s][k].fold_lane(off);
      if (lg == 0 && valid)
        pending[((slot * np + p) * kSums + k) * M + sm] = acc[s][k].value();
    }
  }
}

// ------------------------------------------------------- matrix-core sweep

typedef float v4f __attribute__((ext_vector_type(4)));

// A value equal on every lane, moved to a scalar register.
__device__ __forceinline__ long long uniform64(long long v) {
  const unsigned lo = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(v));
  const unsigned hi = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(static_cast<unsigned long long>(v) >> 32));
  return static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo);
}

// Word 3 of a raw buffer resource on gfx9-family chips (data format 32 bits,
// no swizzle): what untyped dword loads through __builtin_amdgcn_make_buffer_rsrc need.
constexpr int kBufferWord3 = 0x00020000;

// Kernel-row blocks a compensated quad sweep sums in plain float32 (the
// matrix-core accumulators) before folding them into its compensated sums:
// 8 blocks of 4 lags.
constexpr int kQuadFold = 8;
// Blocks of 4 lags whose history and kernel rows the quad sweep has in flight
// ahead of its products (measured on gfx950: 2 to 8 within 3%; 2 fits the
// compensated form's register budget best).
constexpr int kQuadAhead = 2;

// f(integral_constant<int, 0>) ... f(integral_constant<int, N - 1>), in order.
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
  if constexpr (N > 0) {
    static_for<N - 1>(f);
    f(std::integral_constant<int, N - 1>());
  }
}

// The sweep on the matrix cores, for float32 history of two planes that share
// their kernel rows (one material group, one window for every mode).  Its
// sums are the same as sweep_item's: the launch of step n serves steps
// t0 = n+1 .. n+D (D = 16 G) from the history up to step n-1,
//   pending[(t0+u) mod (D+1)] = sum_{i>=2} w_{i+u} (x) U^{t0-i},
// but per class of modes the product over lags is a Toeplitz matrix times a
// matrix of history columns:
//   out[u][col] = sum_i w[i + u] U^{t0-i}[col],
// done as 16x16x4 float32 products (one per 4 lags and 16 steps), each the
// sequence of four fused multiply-adds of a lane's FMA chain in lag order.
//
// Classes are padded to multiples of 4 sorted positions, so the four lanes
// 4j .. 4j+3 of a block ("quad" j) share one kernel row.  The 16 columns are
// (plane p, mode mq of the quad, real/imaginary part): col = 8 p + 2 mq + reim.
// Per 4 lags i0 .. i0+3 and 16-step group g the operands are
//   A[s][k] = w_type[i0 + k + s + 16 g]   (lane s + 16 k; rows past the class's
//                                          window clamp to its zero row),
//   B[k][col] = U^{t0-i0-k}[col]          (lane col + 16 k, one float of the ring),
// and the five products per group are (w11, U_L), (w12, U_N), (w22, U_N),
// (w12, U_L), (w33, U_T) -> sums 2 tau + reim, tau = 0..4, as fma_lag orders
// them.  Output lane l, register v of group g: step u = 16 g + 4 (l/16) + v,
// column l mod 16.
//
// Work-group = one quad of a block of this launch's phase; its LG wavefronts
// take consecutive ranges of the 4-lag blocks and are summed in LDS in a fixed
// order (the compensated sums with Neumaier's rule), so results are bitwise
// reproducible.  Work-group ids of one block are congruent mod 8, so the 16
// quads of a block, which share the history's cache lines, run on one XCD.
// Lags past min(cap-1, t0) meet zero rows or never-written (zero) ring slots,
// as in sweep_item.
// One component of the next block's Toeplitz operand of a 16-step group: lane
// (s, k) = s + 16 k takes lane s + 4 of `cur` for s < 12 and lane s - 12 of
// `above` (the group 16 steps later) for s >= 12 (DPP row shifts within rows of
// 16 lanes).
__device__ __forceinline__ float shift_row4(float cur, float above) {
  const int t = __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, 0.f),
                                            __builtin_bit_cast(int, above), 0x11C /* row_shr:12 */,
                                            0xF, 0xF, false);
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(t, __builtin_bit_cast(int, cur),
                                                               0x104 /* row_shl:4 */, 0xF, 0xF,
                                                               false));
}
__device__ __forceinline__ float4 shift_rows4(float4 cur, float4 above) {
  return float4{shift_row4(cur.x, above.x), shift_row4(cur.y, above.y),
                shift_row4(cur.z, above.z), shift_row4(cur.w, above.w)};
}

template <bool COMP, int G>
__device__ __forceinline__ void quad_sweep(const SweepArgs &a, long long wg, int LG, int QW,
                                           float *__restrict__ lds) {
  constexpr int D = 16 * G;
  // Wavefront w of the work-group: quad qi = w / LG of the work-group's QW
  // quads, lag range chunk = w mod LG (uniform: kept in scalar registers, so
  // the loop control below is scalar).
  const int w = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
  const int chunk = w % LG, qi = w / LG;
  const int per_block = 16 / QW;  // work-groups per block
  const long long kb = (wg / (8 * per_block)) * 8 + (wg & 7);
  if (kb >= a.nphase) return;     // uniform over the work-group
  const int j = static_cast<int>((wg >> 3) % per_block) * QW + qi;  // quad of the block
  const long long M = a.M, step = a.step;
  const long long t0 = step + 1;
  const long long b = t0 % D + D * kb;
  const int lane = threadIdx.x & 63;
  const int s_ = lane & 15;                 // A row (step in group) / B column
  const int k_ = lane >> 4;                 // lag within a 4-lag block
  const int p = s_ >> 3, mq = (s_ >> 1) & 3, reim = s_ & 1;
  const long long sq = b * kLanes + 4 * j;  // first sorted position of the quad
  // Past the last mode (M is a multiple of 4) a quad has no work; it still takes
  // part in the work-group's barrier below (uniform over the wavefront).
  const bool active = sq < M;
  const int cap = __builtin_amdgcn_readfirstlane(a.blk_cap[b]);
  // the class's window (its first position is a mode)
  const int wl = active ? __builtin_amdgcn_readfirstlane(a.win[sq]) : 0;
  const int nent = wl > 0 ? static_cast<int>(max(0LL, min(static_cast<long long>(cap) - 1, t0) - 1)) : 0;
  const int nblk = (nent + 3) / 4;
  const int per = (nblk + LG - 1) / LG;
  const int beta0 = min(nblk, chunk * per);
  const int beta1 = min(nblk, beta0 + per);

  v4f C[G][5];
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int t = 0; t < 5; ++t) C[g][t] = v4f{0.f, 0.f, 0.f, 0.f};
  Acc<float, COMP> acc[G][5][4];
  if (beta1 > beta0) {
    // The quad's operands come through buffer loads: a resource per work-group
    // (the block's slot 0 of the ring, the class's first kernel row) and a
    // 32-bit byte offset per lane; a load past the resource's range returns 0.
    // (Buffer loads also keep the compiler from moving a prefetch down to its
    // use, which it does with plain loads.)
    // (every value a resource is built from is read as uniform, so that the
    // resources live in scalar registers)
    const long long cls0 = uniform64(a.cls_off[__builtin_amdgcn_readfirstlane(a.cls[sq])]);
    const float4 *rowp = static_cast<const float4 *>(a.table) + cls0;
    const __amdgpu_buffer_rsrc_t rows_rsrc = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float4 *>(rowp), 0, (wl + 1) * 16, kBufferWord3);
    // History: slot x of the block at x * dstep floats (the host keeps the
    // block's capacity times dstep below 2^30 floats, so byte offsets fit 32 bits).
    const float *run =
        static_cast<const float *>(a.ring) + uniform64(a.blk_off[b]) * (2LL * 3 * kLanes * 2);
    const int dstep = __builtin_amdgcn_readfirstlane(a.blk_stride[b]) * (2 * 3 * kLanes * 2);
    // (byte counts and offsets in unsigned 32-bit arithmetic: they reach 2^32 - 1)
    const unsigned udstep = static_cast<unsigned>(dstep);
    const __amdgpu_buffer_rsrc_t ring_rsrc = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float *>(run), 0,
        static_cast<int>((static_cast<unsigned>(cap - 1) * udstep + 2u * 3u * kLanes * 2u) * 4u),
        kBufferWord3);
    const int col = ((p * 3) * kLanes + 4 * j + mq) * 2 + reim;
    // (the builtins return the loaded bits as integers)
    auto hist = [&](int x, int c) {
      return __builtin_bit_cast(
          float, __builtin_amdgcn_raw_buffer_load_b32(
                     ring_rsrc,
                     static_cast<int>((static_cast<unsigned>(x) * udstep +
                                       static_cast<unsigned>(col + c * kLanes * 2)) * 4u),
                     0, 0));
    };
    auto row = [&](int r) {
      const v4f v = __builtin_bit_cast(
          v4f, __builtin_amdgcn_raw_buffer_load_b128(rows_rsrc, min(r, wl) * 16, 0, 0));
      return float4{v[0], v[1], v[2], v[3]};
    };
    // The history loads run kQuadAhead blocks ahead of the products (they come
    // from memory); xl is the ring slot of this lane's lag in the next block to load.
    // Every load is issued unconditionally, also for blocks past the range (their
    // values are never used), so that the loop below has no branch around a load
    // and each product waits only for the loads of its own block, not for the
    // ones in flight behind them.  Those loads stay in range: the slot index is
    // clamped at 0 (it only goes negative when cap < 4, and then the range has a
    // single block) and the rows clamp to the class's zero row.
    int xl = static_cast<int>((((t0 - (2 + 4 * beta0) - k_) % cap) + cap) % cap);
    float bq[kQuadAhead][3];
#pragma unroll
    for (int q = 0; q < kQuadAhead; ++q) {
#pragma unroll
      for (int c = 0; c < 3; ++c) bq[q][c] = hist(max(xl, 0), c);
      // the next block's slot is 4 lags older
      xl -= 4;
      if (xl < 0) xl += cap;
    }
    // Kernel-row operands: the top 16-step group's rows are loaded (as far ahead
    // as the history, since the rows' leading edge comes from memory); the
    // lower group's operand follows by a row shift of 4 lanes: lane (s, k) of
    // the next block takes lane (s + 4, k) of its own group, or lane (s - 12, k)
    // of the group above for s >= 12.
    const int r0 = k_ + s_;
    float4 fq[kQuadAhead];
#pragma unroll
    for (int q = 0; q < kQuadAhead; ++q) fq[q] = row(2 + 4 * (beta0 + q) + r0 + 16 * (G - 1));
    float4 a0 = G == 2 ? row(2 + 4 * beta0 + r0) : float4{0.f, 0.f, 0.f, 0.f};
    int fold = 0;
    // One 4-lag block from register set Q (a compile-time index).
    auto block = [&](auto qc, int beta) {
      constexpr int q = decltype(qc)::value;
      const float4 top = fq[q];
      float4 rw[G];
      if constexpr (G == 2) {
        rw[0] = a0;
        rw[1] = top;
      } else {
        rw[0] = top;
      }
#pragma unroll
      for (int g = 0; g < G; ++g) {
        C[g][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(rw[g].x, bq[q][0], C[g][0], 0, 0, 0);
        C[g][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(rw[g].y, bq[q][1], C[g][1], 0, 0, 0);
        C[g][2] = __builtin_amdgcn_mfma_f32_16x16x4f32(rw[g].z, bq[q][1], C[g][2], 0, 0, 0);
        C[g][3] = __builtin_amdgcn_mfma_f32_16x16x4f32(rw[g].y, bq[q][0], C[g][3], 0, 0, 0);
        C[g][4] = __builtin_amdgcn_mfma_f32_16x16x4f32(rw[g].w, bq[q][2], C[g][4], 0, 0, 0);
      }
      if constexpr (G == 2) a0 = shift_rows4(a0, top);
      // this register set now takes block beta + kQuadAhead (loaded also past the
      // range, see above)
#pragma unroll
      for (int c = 0; c < 3; ++c) bq[q][c] = hist(max(xl, 0), c);
      fq[q] = row(2 + 4 * (beta + kQuadAhead) + r0 + 16 * (G - 1));
      // keep the scheduler from sinking these loads towards their use
      __builtin_amdgcn_sched_barrier(0);
      xl -= 4;
      if (xl < 0) xl += cap;
      if constexpr (COMP) {
        // fold the plain partial sums of the last kQuadFold blocks (uniform branch)
        if (++fold == kQuadFold) {
          fold = 0;
#pragma unroll
          for (int g = 0; g < G; ++g)
#pragma unroll
            for (int t = 0; t < 5; ++t)
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                acc[g][t][v].fold(C[g][t][v]);
                C[g][t][v] = 0.f;
              }
        }
      }
    };
    // Whole rounds of kQuadAhead blocks with no branch between the loads of one
    // block and the products of the next (so the compiler's waits are exact:
    // the products of a block wait for its own loads only), then the rest.
    int base = beta0;
    for (; base + kQuadAhead <= beta1; base += kQuadAhead)
      static_for<kQuadAhead>([&](auto qc) { block(qc, base + decltype(qc)::value); });
    static_for<kQuadAhead - 1>([&](auto qc) {
      if (base + decltype(qc)::value < beta1) block(qc, base + decltype(qc)::value);
    });
  }
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int t = 0; t < 5; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[g][t][v].fold(C[g][t][v]);
  // lag ranges of the other wavefronts, added in chunk order by wavefront 0
  if (LG > 1) {
    constexpr int NV = G * 5 * 4;
    constexpr int PER = COMP ? 2 : 1;
    lds += static_cast<long long>(qi) * (LG - 1) * NV * PER * kLanes;  // this quad's partial sums
    if (chunk > 0) {
      float *dst = lds + static_cast<long long>(chunk - 1) * NV * PER * kLanes + lane;
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int t = 0; t < 5; ++t)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int idx = (g * 5 + t) * 4 + v;
            dst[(idx * PER) * kLanes] = acc[g][t][v].s;
            if constexpr (COMP) dst[(idx * PER + 1) * kLanes] = acc[g][t][v].c;
          }
    }
    __syncthreads();
    if (chunk == 0) {
      for (int w = 1; w < LG; ++w) {
        const float *src = lds + static_cast<long long>(w - 1) * NV * PER * kLanes + lane;
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
          for (int t = 0; t < 5; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int idx = (g * 5 + t) * 4 + v;
              if constexpr (COMP) {
                neumaier(acc[g][t][v].s, acc[g][t][v].c, src[(idx * PER) * kLanes]);
                acc[g][t][v].c += src[(idx * PER + 1) * kLanes];
              } else {
                acc[g][t][v].s += src[(idx * PER) * kLanes];
              }
            }
      }
    }
  }
  if (chunk != 0 || !active) return;
  float *__restrict__ pending = static_cast<float *>(a.pending);
  const long long col_off = (static_cast<long long>(p) * kSums + reim) * M + sq + mq;
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const long long slot = (t0 + 16 * g + 4 * k_ + v) % (D + 1);
      float *dst = pending + slot * 2 * kSums * M + col_off;
#pragma unroll
      for (int t = 0; t < 5; ++t) dst[2 * t * M] = acc[g][t][v].value();
    }
}

// Mode item of step n for one (mode, plane): the push, then the traction of
// the same step from the same registers.
//   push:    rotate the new spectrum into the wavevector frame, update the
//            float64 running state, store the ring slot of step n;
//   traction: the pending history sum of step n plus the lags from the
//            block's last sweep on (compensated for the compensated form),
//            damping and instantaneous terms, rotation back to (x1, x2, x3),
//            scatter into the natural half-spectrum layout.
// The lag-0 history value and the velocity of the damping term are the ones
// just computed (rounded to the working precision as the ring stores them).
template <typename R, bool COMP>
__device__ __forceinline__ void mode_step(const ModeArgs &a, int p, long long s) {
  using W = typename W4<R>::T;
  const double2 *__restrict__ spec = static_cast<const double2 *>(a.spec);
  const double2 *__restrict__ spec_v = static_cast<const double2 *>(a.spec_v);
  cplx<R> *__restrict__ ring = static_cast<cplx<R> *>(a.ring);
  double2 *__restrict__ state = a.state;
  const long long M = a.M, nh = a.nh, step = a.step;
  const int np = a.np;
  const long long natural = a.nat[s];
  if (natural < 0) return;  // a padding position of the matrix-core layout: no mode
  const double q = a.geom[4 * s + 0];
  const double kh1 = a.geom[4 * s + 1];
  const double kh3 = a.geom[4 * s + 2];
  const long long b = s >> 6;
  const int lane = static_cast<int>(s & 63);
  const int cap = a.blk_cap[b];
  const long long base = a.blk_off[b];
  const long long stride = a.blk_stride[b];
  const long long rec_len = static_cast<long long>(np) * 3 * kLanes;
  const int x0 = cap > 0 ? static_cast<int>(step % cap) : 0;
  const PlaneParams &pp = p == 0 ? a.p0 : a.p1;
  const int pg = pp.index;

  // ---- push
  cplx<R> u0[3], v0[3];
  {
    double2 x[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) x[c] = spec[(pg * 3 + c) * nh + natural];
    // (1, 2, 3) -> (L, N, T)
    const double2 xr[3] = {{kh1 * x[0].x + kh3 * x[2].x, kh1 * x[0].y + kh3 * x[2].y},
                           x[1],
                           {-kh3 * x[0].x + kh1 * x[2].x, -kh3 * x[0].y + kh1 * x[2].y}};
    double2 vr[3];
    if (a.vel_rule == VEL_INPUT) {
      double2 y[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) y[c] = spec_v[(pg * 3 + c) * nh + natural];
      vr[0] = double2{kh1 * y[0].x + kh3 * y[2].x, kh1 * y[0].y + kh3 * y[2].y};
      vr[1] = y[1];
      vr[2] = double2{-kh3 * y[0].x + kh1 * y[2].x, -kh3 * y[0].y + kh1 * y[2].y};
    }
    cplx<R> *rp = ring + (base + static_cast<long long>(x0) * stride) * rec_len +
                  static_cast<long long>(p) * 3 * kLanes + lane;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const long long si = (static_cast<long long>(p) * 3 + c) * M + s;
      const double2 prev = state[si];
      double2 now;
      if (a.state_rule == STATE_ACCUM)
        now = double2{prev.x + xr[c].x, prev.y + xr[c].y};
      else
        now = xr[c];
      state[si] = now;
      double2 v;
      if (a.vel_rule == VEL_DIFF)
        v = double2{(now.x - prev.x) * a.inv_dt, (now.y - prev.y) * a.inv_dt};
      else if (a.vel_rule == VEL_SCALE)
        v = double2{xr[c].x * a.inv_dt, xr[c].y * a.inv_dt};
      else if (a.vel_rule == VEL_INPUT)
        v = vr[c];
      else if (a.vel_rule == VEL_ZERO)
        v = double2{0.0, 0.0};
      else
        v = xr[c];
      v0[c] = cplx<R>{static_cast<R>(v.x), static_cast<R>(v.y)};
      u0[c] = cplx<R>{static_cast<R>(now.x), static_cast<R>(now.y)};
      if (cap > 0) rp[c * kLanes] = u0[c];
    }
  }

  // ---- history sums of step n
  const int wl = a.win[s];
  const int S = a.depth;
  const int phi = static_cast<int>(b % S);
  // The sweep launched with step m-1 covers steps m .. m+S-1 (m = phi mod S,
  // m >= 1) over the history up to step m-2.  Lags not in the pending sum:
  // those from step m-1 on, or all of them before the block's first sweep.
  const bool swept = step >= (phi == 0 ? S : phi);
  const int fresh =
      min(wl, swept ? static_cast<int>((step - phi) % S) + 2 : static_cast<int>(step) + 1);
  R cs[kSums];
  {
    Acc<R, COMP> acc[kSums];
    if (swept) {
      const R *__restrict__ pend = static_cast<const R *>(a.pending) +
                                   ((step % (S + 1)) * np + p) * kSums * M + s;
#pragma unroll
      for (int k = 0; k < kSums; ++k) acc[k].s = pend[k * M];
    }
    if (fresh > 0) {
      // the newest lags: plain products (the compensated form folds their sum,
      // at most depth + 1 lags, into the pending sum once)
      const W *__restrict__ rowp = static_cast<const W *>(a.table) + a.cls_off[a.cls[s]];
      R part[kSums];
#pragma unroll
      for (int k = 0; k < kSums; ++k) part[k] = COMP ? R(0) : acc[k].s;
      fma_lag<R>(part, rowp[0], u0);
      const cplx<R> *rp = ring + base * rec_len + static_cast<long long>(p) * 3 * kLanes + lane;
      // The older lags in batches of FB, every load of a batch in flight before
      // its products: the lag index is clamped (fresh <= W <= cap, so the ring
      // slot stays in the block's ring), the loads need no branch, and lags
      // past `fresh` take zero weights, which leave the sums unchanged.
      constexpr int FB = 4;  // measured on gfx950: as fast as 8 with fewer registers
      for (int j0 = 1; j0 < fresh; j0 += FB) {
        cplx<R> u[FB][3];
        W w[FB];
#pragma unroll
        for (int i = 0; i < FB; ++i) {
          const int j = min(j0 + i, fresh - 1);
          int x = x0 - j;
          if (x < 0) x += cap;
          const cplx<R> *qp = rp + static_cast<long long>(x) * stride * rec_len;
          u[i][0] = qp[0];
          u[i][1] = qp[kLanes];
          u[i][2] = qp[2 * kLanes];
          w[i] = rowp[j];
        }
#pragma unroll
        for (int i = 0; i < FB; ++i) {
          const bool on = j0 + i < fresh;
          const W wi = {on ? w[i].x : R(0), on ? w[i].y : R(0), on ? w[i].z : R(0),
                        on ? w[i].w : R(0)};
          fma_lag<R>(part, wi, u[i]);
        }
      }
#pragma unroll
      for (int k = 0; k < kSums; ++k) {
        if constexpr (COMP)
          acc[k].fold(part[k]);
        else
          acc[k].s = part[k];
      }
    }
#pragma unroll
    for (int k = 0; k < kSums; ++k) cs[k] = acc[k].value();
  }

  // ---- traction of step n
  const R sg = static_cast<R>(pp.side);
  const R muq = static_cast<R>(pp.mu * q);
  const R damp = static_cast<R>(pp.mu / pp.cs);
  const R inst = static_cast<R>((2.0 - pp.eta) * pp.mu * q);
  const R eta = static_cast<R>(pp.eta);
  const R r1 = static_cast<R>(kh1), r3 = static_cast<R>(kh3);
  cplx<R> u[3] = {{R(0), R(0)}, {R(0), R(0)}, {R(0), R(0)}};
  if (cap > 0 && wl > 0) {
#pragma unroll
    for (int c = 0; c < 3; ++c) u[c] = u0[c];
  }
  // conv + instantaneous (rotated frame):
  //   A_L = -sg mu q C11 + i (2-eta) mu q U_N - i mu q C12[U_N]
  //   A_N = -sg mu q C22 - i (2-eta) mu q U_L + i mu q C12[U_L]
  //   A_T = -sg mu q C33
  cplx<R> t[3];
  t[0] = cplx<R>{-sg * muq * cs[0] - inst * u[1].y + muq * cs[3],
                 -sg * muq * cs[1] + inst * u[1].x - muq * cs[2]};
  t[1] = cplx<R>{-sg * muq * cs[4] + inst * u[0].y - muq * cs[7],
                 -sg * muq * cs[5] - inst * u[0].x + muq * cs[6]};
  t[2] = cplx<R>{-sg * muq * cs[8], -sg * muq * cs[9]};
  // damping: -sg (mu/c_s) diag(1, eta, 1) V
  const cplx<R> d[3] = {{-sg * damp * v0[0].x, -sg * damp * v0[0].y},
                        {-sg * damp * eta * v0[1].x, -sg * damp * eta * v0[1].y},
                        {-sg * damp * v0[2].x, -sg * damp * v0[2].y}};
  if (a.lam) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const long long si = (static_cast<long long>(p) * 3 + c) * M + s;
      double2 l = a.lam[si];
      l.x += static_cast<double>(t[c].x);
      l.y += static_cast<double>(t[c].y);
      a.lam[si] = l;
      t[c] = cplx<R>{static_cast<R>(l.x), static_cast<R>(l.y)};
    }
  }
  cplx<R> *__restrict__ out_a = static_cast<cplx<R> *>(a.out_a);
  cplx<R> *__restrict__ out_b = static_cast<cplx<R> *>(a.out_b);
  if (!out_b) {
#pragma unroll
    for (int c = 0; c < 3; ++c) t[c] = cplx<R>{t[c].x + d[c].x, t[c].y + d[c].y};
  }
  // (L, N, T) -> (1, 2, 3)
  out_a[(pg * 3 + 0) * nh + natural] = cplx<R>{r1 * t[0].x - r3 * t[2].x, r1 * t[0].y - r3 * t[2].y};
  out_a[(pg * 3 + 1) * nh + natural] = t[1];
  out_a[(pg * 3 + 2) * nh + natural] = cplx<R>{r3 * t[0].x + r1 * t[2].x, r3 * t[0].y + r1 * t[2].y};
  if (out_b) {
    out_b[(pg * 3 + 0) * nh + natural] =
        cplx<R>{r1 * d[0].x - r3 * d[2].x, r1 * d[0].y - r3 * d[2].y};
    out_b[(pg * 3 + 1) * nh + natural] = d[1];
    out_b[(pg * 3 + 2) * nh + natural] =
        cplx<R>{r3 * d[0].x + r1 * d[2].x, r3 * d[0].y + r1 * d[2].y};
  }
}

// Mode items in XCD-contiguous order.  Work-group ids go round-robin over the 8
// XCDs, so id m of a launch's mode part (which starts at a multiple of 8) runs on
// XCD m mod 8; it takes item (m mod 8) * per + m / 8 of the n items, so each XCD
// works through a contiguous eighth of the sorted blocks (nearby q), whose
// natural-order spectrum gathers and traction scatters then share cache lines
// in that XCD's L2.  The mode part has 8 * per ids; the ones past n return.
__device__ __forceinline__ long long xcd_chunk(long long m, long long n) {
  return (m & 7) * ((n + 7) / 8) + (m >> 3);
}
inline long long xcd_chunk_ids(long long n) { return (n + 7) / 8 * 8; }

// One launch per step of mode-space work: the sweep items of the blocks whose
// turn it is, then one mode item per (64-mode block, plane).  The two kinds
// share no data (see sweep_item), so the latency-bound push gathers and
// traction scatters run beside the streaming sweep.
template <typename R, int S, int T, bool COMP>
__device__ __forceinline__ void step_items(const SweepArgs &sa, const ModeArgs &ma,
                                           long long sweep_items, long long nblocks) {
  const long long item = blockIdx.x;
  if (item < sweep_items) {
    sweep_item<R, S, T, COMP>(sa, item);
    return;
  }
  const long long k = xcd_chunk(item - sweep_items, nblocks * ma.np);
  if (k >= nblocks * ma.np) return;
  const int p = static_cast<int>(k / nblocks);
  const long long s = (k - p * nblocks) * kLanes + threadIdx.x;
  if (s < ma.M) mode_step<R, COMP>(ma, p, s);
}

template <typename R, int S, int T, bool COMP>
__global__ __launch_bounds__(kLanes) void step_kernel(SweepArgs sa, ModeArgs ma,
                                                      long long sweep_items, long long nblocks) {
  step_items<R, S, T, COMP>(sa, ma, sweep_items, nblocks);
}

// The float32 sweep at 6 steps per lane and two lanes per mode, held to four
// wavefronts per SIMD (128 registers; the compiler alone takes 131, three).
template <typename R, int S, int T, bool COMP>
__global__ __launch_bounds__(kLanes) __attribute__((amdgpu_waves_per_eu(4))) void step_kernel_w4(
    SweepArgs sa, ModeArgs ma, long long sweep_items, long long nblocks) {
  step_items<R, S, T, COMP>(sa, ma, sweep_items, nblocks);
}

// The compensated sweep at up to 6 steps per lane, held to two wavefronts per
// SIMD: left to itself the compiler takes the whole register file (one
// wavefront) for a couple of registers that it then keeps in scratch instead.
template <typename R, int S, int T, bool COMP>
__global__ __launch_bounds__(kLanes) __attribute__((amdgpu_waves_per_eu(2))) void step_kernel_w2(
    SweepArgs sa, ModeArgs ma, long long sweep_items, long long nblocks) {
  step_items<R, S, T, COMP>(sa, ma, sweep_items, nblocks);
}

// The launch of the matrix-core form: work-groups of LG wavefronts, first the
// quad sweeps of this launch's phase, then the mode items (LG (block, plane)
// items per work-group, one per wavefront).  LDS (dynamic) holds the partial
// sums of wavefronts 1 .. LG-1 of a quad.
template <bool COMP, int G, int WAVES>
__global__ __launch_bounds__(4 * kLanes) __attribute__((amdgpu_waves_per_eu(WAVES))) void
step_kernel_mfma(SweepArgs sa, ModeArgs ma, long long sweep_wgs, long long nblocks, int LG, int QW) {
  extern __shared__ float quad_lds[];
  const long long wg = blockIdx.x;
  if (wg < sweep_wgs) {
    quad_sweep<COMP, G>(sa, wg, LG, QW, quad_lds);
    return;
  }
  const long long mode_wgs = (nblocks * ma.np + LG * QW - 1) / (LG * QW);
  const long long mw = xcd_chunk(wg - sweep_wgs, mode_wgs);
  if (mw >= mode_wgs) return;
  const long long k = mw * (LG * QW) + (threadIdx.x >> 6);
  if (k >= nblocks * ma.np) return;
  const int p = static_cast<int>(k / nblocks);
  const long long s = (k - p * nblocks) * kLanes + (threadIdx.x & 63);
  if (s < ma.M) mode_step<float, COMP>(ma, p, s);
}

// -------------------------------------------------------------- tabulate

// Piece A (0 < y < 1): y = sin(t).  Piece B (1 < y < eta): y^2 = 1 + (eta^2-1) sin^2(t).
// Both map t in [0, pi/2] and remove the square-root end points of the
// branch-cut densities D_ab (see the oracle-independent derivation in the
// library notes): the substituted integrands are analytic.
struct Node {
  double y, g11, g12, g22, g33, ph_hi, ph_lo, c_step, s_step;
};

// Lags a thread of tabulate_kernel sums, kTabThreads apart.
constexpr int kTabThreads = 256;
constexpr int kTabLags = 8;

// x - 2 pi k for the double-double x = hi + lo, reduced in two parts
// (Cody-Waite): accurate to ~1e-16 absolute however many periods x spans.
__device__ __forceinline__ double reduce_two_pi(double hi, double lo) {
  const double two_pi_hi = 6.283185307179586;      // nearest double to 2 pi
  const double two_pi_lo = 2.4492935982947064e-16;  // 2 pi - two_pi_hi
  const double inv_two_pi = 0.15915494309189535;
  const double k = rint(hi * inv_two_pi);
  const double r = fma(-k, two_pi_hi, hi);  // exact
  return fma(-k, two_pi_lo, r) + lo;
}

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
  // the phase step between the lags of one thread, kTabThreads y dT (exact scaling)
  sincos(reduce_two_pi(kTabThreads * n.ph_hi, kTabThreads * n.ph_lo), &n.s_step, &n.c_step);
  return n;
}

// w_ab,j = sum_nodes g_ab cos or sin((j + 1/2) y dT).  A thread takes lags
// j, j + kTabThreads, ..., j + (kTabLags-1) kTabThreads.  For the first the
// phase is formed as a double-double and reduced by 2 pi (reduce_two_pi) and
// its sine and cosine evaluated; each next one is that pair rotated by the
// node's phase step (at most kTabLags-1 rotations, a few ulps).
template <typename R>
__global__ __launch_bounds__(kTabThreads) void tabulate_kernel(
    typename W4<R>::T *__restrict__ table, const long long *__restrict__ cls_off,
    const double *__restrict__ cls_q, const int *__restrict__ cls_w, double cs, double dt,
    double eta, double rate, const double *__restrict__ gl_x, const double *__restrict__ gl_w) {
  __shared__ Node nodes[kTabThreads];
  const int c = blockIdx.x;
  const int W = cls_w[c];
  const double q = cls_q[c];
  const double dT = q * cs * dt;
  const double tmax = dT * W * rate;
  const int npan = max(1, static_cast<int>(ceil(tmax / 40.0)));
  const int nnodes = 2 * npan * kGaussN;
  constexpr int span = kTabThreads * kTabLags;
  for (int jb = 0; jb <= W; jb += span) {  // j = W: the zero row
    const int j0 = jb + threadIdx.x;
    // lags of this thread inside the window
    const int nl = j0 < W ? min(kTabLags, (W - 1 - j0) / kTabThreads + 1) : 0;
    const double m = j0 + 0.5;
    double w[kTabLags][4];
#pragma unroll
    for (int t = 0; t < kTabLags; ++t) w[t][0] = w[t][1] = w[t][2] = w[t][3] = 0.0;
    for (int nb = 0; nb < nnodes; nb += kTabThreads) {
      __syncthreads();
      if (nb + threadIdx.x < nnodes)
        nodes[threadIdx.x] = make_node(nb + threadIdx.x, npan, eta, dT, gl_x, gl_w);
      __syncthreads();
      const int cnt = min(kTabThreads, nnodes - nb);
      if (nl > 0) {
        for (int i = 0; i < cnt; ++i) {
          const Node &nd = nodes[i];
          const double p_hi = m * nd.ph_hi;
          const double p_lo = fma(m, nd.ph_lo, fma(m, nd.ph_hi, -p_hi));
          double sn, cn;
          sincos(reduce_two_pi(p_hi, p_lo), &sn, &cn);
#pragma unroll
          for (int t = 0; t < kTabLags; ++t) {
            if (t >= nl) break;
            w[t][0] = fma(nd.g11, cn, w[t][0]);
            w[t][1] = fma(nd.g12, sn, w[t][1]);
            w[t][2] = fma(nd.g22, cn, w[t][2]);
            w[t][3] = fma(nd.g33, cn, w[t][3]);
            const double c2 = fma(cn, nd.c_step, -sn * nd.s_step);
            sn = fma(sn, nd.c_step, cn * nd.s_step);
            cn = c2;
          }
        }
      }
    }
#pragma unroll
    for (int t = 0; t < kTabLags; ++t) {
      const int j = j0 + t * kTabThreads;
      if (t < nl) {
        typename W4<R>::T o;
        o.x = static_cast<R>(w[t][0]);
        o.y = static_cast<R>(w[t][1]);
        o.z = static_cast<R>(w[t][2]);
        o.w = static_cast<R>(w[t][3]);
        table[cls_off[c] + j] = o;
      }
      if (j == W) table[cls_off[c] + W] = typename W4<R>::T{R(0), R(0), R(0), R(0)};
    }
  }
}

template <typename R, int S, int T, bool COMP>
hipError_t step_launch_s(const sbim_handle *h, const Group &g, const SweepArgs &sa0,
                         const ModeArgs &ma, hipEvent_t ev0, hipEvent_t ev1) {
  constexpr int D = S * T;
  SweepArgs sa = sa0;
  const int phase = static_cast<int>((sa.step + 1) % D);
  sa.nphase = g.nblocks > phase ? (g.nblocks - phase + D - 1) / D : 0;
  const long long sweep_items =
      (sa.nphase + 7) / 8 * 8 * (sweep_lag_groups<R, S, T, COMP>() * T) * g.np;
  const long long items = sweep_items + xcd_chunk_ids(g.nblocks * g.np);
  if (ev0) {
    const hipError_t e = hipEventRecord(ev0, h->stream);
    if (e != hipSuccess) return e;
  }
  if constexpr (!COMP && sizeof(R) == 4 && S == 6 && T == 2)
    hipLaunchKernelGGL((step_kernel_w4<R, S, T, COMP>), dim3(static_cast<unsigned>(items)),
                       dim3(kLanes), 0, h->stream, sa, ma, sweep_items, g.nblocks);
  else if constexpr (COMP && S <= 6)
    hipLaunchKernelGGL((step_kernel_w2<R, S, T, COMP>), dim3(static_cast<unsigned>(items)),
                       dim3(kLanes), 0, h->stream, sa, ma, sweep_items, g.nblocks);
  else
    hipLaunchKernelGGL((step_kernel<R, S, T, COMP>), dim3(static_cast<unsigned>(items)),
                       dim3(kLanes), 0, h->stream, sa, ma, sweep_items, g.nblocks);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && ev1) e = hipEventRecord(ev1, h->stream);
  return e;
}

template <bool COMP, int G>
hipError_t step_launch_q(const sbim_handle *h, const Group &g, const SweepArgs &sa0,
                         const ModeArgs &ma, hipEvent_t ev0, hipEvent_t ev1) {
  constexpr int D = 16 * G;
  SweepArgs sa = sa0;
  const int phase = static_cast<int>((sa.step + 1) % D);
  sa.nphase = g.nblocks > phase ? (g.nblocks - phase + D - 1) / D : 0;
  const int LG = h->lag_chunks, QW = h->sweep_quads;
  const long long sweep_wgs = (sa.nphase + 7) / 8 * 8 * (16 / QW);
  const long long mode_wgs = (g.nblocks * g.np + LG * QW - 1) / (LG * QW);
  const size_t lds = static_cast<size_t>(QW) * (LG - 1) * G * 5 * 4 * (COMP ? 2 : 1) * kLanes *
                     sizeof(float);
  if (ev0) {
    const hipError_t e = hipEventRecord(ev0, h->stream);
    if (e != hipSuccess) return e;
  }
  // Register budget: three wavefronts per SIMD (168 registers; the compensated
  // two-group form takes 165).  At two wavefronts per SIMD the 2080 sweep
  // wavefronts of a 512^2 phase (1040 quads, two lag ranges each) do not all
  // fit at once, and the rest take a second round (measured on gfx950 with one
  // quad per work-group: 4-8% slower).
  constexpr int WAVES = 3;
  hipLaunchKernelGGL((step_kernel_mfma<COMP, G, WAVES>),
                     dim3(static_cast<unsigned>(sweep_wgs + xcd_chunk_ids(mode_wgs))),
                     dim3(LG * QW * kLanes), lds, h->stream, sa, ma, sweep_wgs, g.nblocks, LG, QW);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && ev1) e = hipEventRecord(ev1, h->stream);
  return e;
}

template <typename R, bool COMP>
hipError_t step_launch_r(const sbim_handle *h, const Group &g, const SweepArgs &sa,
                         const ModeArgs &ma, hipEvent_t ev0, hipEvent_t ev1) {
  switch (h->depth) {
    case 1: return step_launch_s<R, 1, 1, COMP>(h, g, sa, ma, ev0, ev1);
    case 2: return step_launch_s<R, 2, 1, COMP>(h, g, sa, ma, ev0, ev1);
    case 4: return step_launch_s<R, 4, 1, COMP>(h, g, sa, ma, ev0, ev1);
    case 6: return step_launch_s<R, 6, 1, COMP>(h, g, sa, ma, ev0, ev1);
    case 8: return step_launch_s<R, 8, 1, COMP>(h, g, sa, ma, ev0, ev1);
    case 12: return step_launch_s<R, 6, 2, COMP>(h, g, sa, ma, ev0, ev1);
    case 16: return step_launch_s<R, 8, 2, COMP>(h, g, sa, ma, ev0, ev1);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_step(const sbim_handle *h, const Group &g, const StepLaunch &w,
                       hipEvent_t ev0, hipEvent_t ev1) {
  ModeArgs ma;
  ma.spec = w.spec;
  ma.spec_v = w.spec_v;
  ma.ring = w.ring;
  ma.state = reinterpret_cast<double2 *>(w.state);
  ma.pending = w.pending;
  ma.table = g.table;
  ma.cls_off = g.cls_off;
  ma.cls = g.cls;
  ma.win = g.win;
  ma.nat = g.nat;
  ma.geom = g.geom;
  ma.blk_off = g.blk_off;
  ma.blk_cap = g.blk_cap;
  ma.blk_stride = g.blk_stride;
  ma.lam = reinterpret_cast<double2 *>(w.lam);
  ma.out_a = w.out_a;
  ma.out_b = w.out_b;
  ma.M = g.M;
  ma.nh = w.nh;
  ma.step = w.step;
  ma.np = g.np;
  ma.depth = h->depth;
  ma.inv_dt = 1.0 / w.dt;
  ma.vel_rule = w.vel_rule;
  ma.state_rule = w.state_rule;
  ma.p0 = g.pl[0];
  ma.p1 = g.np > 1 ? g.pl[1] : g.pl[0];
  SweepArgs sa;
  sa.ring = w.ring;
  sa.table = g.table;
  sa.pending = w.pending;
  sa.cls = g.cls;
  sa.win = g.win;
  sa.blk_off = g.blk_off;
  sa.blk_cap = g.blk_cap;
  sa.blk_stride = g.blk_stride;
  sa.cls_off = g.cls_off;
  sa.cls_w0 = g.wmax;
  sa.M = g.M;
  sa.step = w.step;
  sa.np = g.np;
  sa.nphase = 0;
  if (h->mfma) {
    if (g.np != 2 || h->fp64 || (h->depth != 16 && h->depth != 32) || h->lag_chunks < 1 ||
        h->lag_chunks > 4)
      return hipErrorInvalidValue;
    if (h->comp)
      return h->depth == 32 ? step_launch_q<true, 2>(h, g, sa, ma, ev0, ev1)
                            : step_launch_q<true, 1>(h, g, sa, ma, ev0, ev1);
    return h->depth == 32 ? step_launch_q<false, 2>(h, g, sa, ma, ev0, ev1)
                          : step_launch_q<false, 1>(h, g, sa, ma, ev0, ev1);
  }
  if (h->fp64) return step_launch_r<double, false>(h, g, sa, ma, ev0, ev1);
  if (h->comp) return step_launch_r<float, true>(h, g, sa, ma, ev0, ev1);
  return step_launch_r<float, false>(h, g, sa, ma, ev0, ev1);
}

hipError_t launch_tabulate(bool fp64, const Group &g, double dt, const double *gl_x,
                           const double *gl_w, hipStream_t st) {
  if (g.nclasses == 0) return hipSuccess;
  const double rate = fmax(1.0, (g.eta * g.eta - 1.0) / 2.0);
  if (fp64) {
    hipLaunchKernelGGL(tabulate_kernel<double>, dim3(static_cast<unsigned>(g.nclasses)), dim3(kTabThreads),
                       0, st, static_cast<double4 *>(g.table), g.cls_off, g.cls_q, g.cls_w, g.cs, dt,
                       g.eta, rate, gl_x, gl_w);
  } else {
    hipLaunchKernelGGL(tabulate_kernel<float>, dim3(static_cast<unsigned>(g.nclasses)), dim3(kTabThreads),
                       0, st, static_cast<float4 *>(g.table), g.cls_off, g.cls_q, g.cls_w, g.cs, dt,
                       g.eta, rate, gl_x, gl_w);
  }
  return hipGetLastError();
}

}  // namespace sbim
