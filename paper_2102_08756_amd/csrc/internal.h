// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "sbim.h"

namespace sbim {

constexpr int kLanes = 64;            // modes per wavefront / per ring block
constexpr int kTwiddleLog = 12;       // twiddle table covers lengths up to 4096
constexpr int kTwiddleN = 1 << kTwiddleLog;
constexpr int kFftThreads = 256;
constexpr int kFftPerThread = 16;     // transform points per thread in the LDS FFT kernels
constexpr int kGaussN = 32;           // Gauss-Legendre points per quadrature panel
constexpr int kMaxSweep = 8;          // deepest sweep: steps served by one pass over a history

// How the push forms the velocity of the damping term.
enum VelRule : int {
  VEL_DIFF = 0,   // (x_rot - previous state) / dt
  VEL_SCALE = 1,  // x_rot / dt
  VEL_INPUT = 2,  // rotate(spectrum of the supplied velocity)
  VEL_COPY = 3,   // x_rot
  VEL_ZERO = 4    // no damping term (the fault solve adds it)
};
enum StateRule : int { STATE_REPLACE = 0, STATE_ACCUM = 1 };

struct PlaneParams {
  double mu, cs, eta;
  int side;
  int index;        // global plane index (field slot)
};

// Device arrays and sizes of one material group (planes with equal c_s, c_p).
struct Group {
  int np = 0;                     // planes in the group (1 or 2)
  PlaneParams pl[SBIM_MAX_PLANES];
  double cs = 0, cp = 0, eta = 0;
  long long M = 0;                // modes (half spectrum)
  long long nblocks = 0;          // ceil(M / 64)
  long long nclasses = 0;         // kernel rows
  int wmax = 0;                   // largest W(q)
  long long ring_records = 0;     // sum of block capacities
  long long table_rows = 0;       // sum over classes of W + 1
  // device
  int *nat = nullptr;             // [M] sorted position -> spectrum bin i3 * n1 + i1
  int *cls = nullptr;             // [M] sorted position -> class
  int *win = nullptr;             // [M] W(q) per sorted position
  double *geom = nullptr;         // [M][4] q, kh1, kh3, 0 per sorted position
  long long *blk_off = nullptr;   // [nblocks] first ring record of the block
  int *blk_cap = nullptr;         // [nblocks] ring capacity of the block (its largest W)
  int *blk_stride = nullptr;      // [nblocks] records between consecutive slots of the block
  long long *cls_off = nullptr;   // [nclasses] first table entry of each class
  double *cls_q = nullptr;        // [nclasses]
  int *cls_w = nullptr;           // [nclasses]
  void *table = nullptr;          // [table_rows] x 4 reals (w11, w12, w22, w33)
  void *ring = nullptr;           // [ring_records][np][3][64] complex
  double *state = nullptr;        // [np][3][M] complex double (rotated frame, sorted)
  void *pending = nullptr;        // [depth+1][np][10][M] real_t: history sums of coming steps
  // adjoint (allocated on first use)
  void *ring_adj = nullptr;
  void *pending_adj = nullptr;
  double *state_adj = nullptr;    // previous g spectrum (float64)
  double *lam_adj = nullptr;      // reverse running sum (float64)
  // host copies for diagnostics / work accounting
  std::vector<int> h_nat, h_cls, h_win;
  std::vector<long long> h_cls_off;
  std::vector<int> h_cls_w, h_blk_cap;
};

}  // namespace sbim

struct sbim_handle {
  sbim_config cfg;
  hipStream_t stream = nullptr;
  int device = 0;
  bool fp64 = true;
  bool comp = false;
  size_t rsize = 8;               // sizeof(real_t)
  int n1 = 0, n3 = 0, h3 = 0;     // h3 = n3/2 + 1
  long long nh = 0;               // n1 * h3
  int ngroups = 0;
  sbim::Group g[SBIM_MAX_PLANES];
  long long step = 0;             // pushes done
  long long bstep = 0;            // backward calls done
  int depth = 1;                  // sweep depth: steps served by one pass over a block's history
  bool mfma = false;              // history sweep on the matrix cores (quads of one class)
  int lag_chunks = 1;             // matrix-core sweep: wavefronts per quad, each a lag range
  int sweep_quads = 1;            // matrix-core sweep: quads per work-group (1, 2 or 4)
  void *twiddle = nullptr;        // [4096] complex real_t, exp(-2 pi i m / 4096)
  void *twiddle64 = nullptr;      // the same in float64 (== twiddle for SBIM_FP64)
  void *spec = nullptr;           // [P][3][h3][n1] complex float64: spectrum of the pushed field
  void *spec_v = nullptr;         // same for the velocity; second traction output of backward
  void *out_spec = nullptr;       // [P][3][h3][n1] complex: traction spectrum of the last push
  void *out_adj = nullptr;        // the same for the last sbim_backward (allocated on first use)
  long long *count_scratch = nullptr;  // device address of the static partial counts (checks.hip)
  int profile_every = 0;          // bracket every n-th step launch with events (0: off)
  long long profile_seen = 0;     // step launches since sbim_profile_conv
  std::vector<hipEvent_t> ev_start, ev_stop;  // reusable pool
  size_t ev_used = 0;                          // pairs recorded since sbim_profile_conv
  std::string err;
};

namespace sbim {

// fft.hip: fields [F][n1][n3] real <-> spectrum [F][n3/2+1][n1] complex.
// The forward transform always computes in float64 (its output feeds the
// float64 running state); in_fp64 selects the type of the input field.
hipError_t launch_fft_forward(bool in_fp64, const void *in, void *spec, int F, int n1, int n3,
                              const void *tw64, hipStream_t st);
// out = scale * inverse(spec) + add_or_null; spec is left intact, `scratch`
// (the size of spec) receives the intermediate transform.
hipError_t launch_fft_inverse(bool fp64, const void *spec, void *scratch, void *out,
                              const void *add_or_null, int F, int n1, int n3, double scale,
                              const void *tw, hipStream_t st);
hipError_t upload_twiddles(bool fp64, void *dst, hipStream_t st);

// kernels.hip
//
// The history sums are split over time.  Block b of 64 modes has phase
// b mod depth.  The launch of step n sweeps the blocks of phase (n+1) mod
// depth: each reads its history up to step n-1 once and stores, for each of
// the steps n+1 .. n+depth, the part of that step's sum over that history
// ("pending" sums, depth+1 slots).  The same launch pushes step n for every
// mode and completes its traction: the pending sum of step n plus the lags
// from the block's last sweep on (at most depth+1 of them), damping and
// instantaneous terms.
struct StepLaunch {
  const void *spec;       // [P][3][nh] complex float64 (spectrum layout)
  const void *spec_v;     // velocity spectrum (same type) or null
  void *ring;
  double *state;
  void *pending;
  double *lam;            // non-null: accumulate (conv + instantaneous) into this float64 state
  void *out_a;            // [P][3][nh] complex: output spectrum
  void *out_b;            // non-null: damping part written here instead of added to out_a
  long long nh;
  long long step;         // index of this push
  double dt;
  int vel_rule, state_rule;
};
// One launch, bracketed by ev0/ev1 when they are non-null.
hipError_t launch_step(const sbim_handle *h, const Group &g, const StepLaunch &w,
                       hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// Kernel arguments (device pointers) of the two item kinds of that launch.
struct ModeArgs {
  const void *spec, *spec_v;
  void *ring;
  double2 *state;
  const void *pending, *table;
  const long long *cls_off;
  const int *cls, *win, *nat;
  const double *geom;
  const long long *blk_off;
  const int *blk_cap, *blk_stride;
  double2 *lam;
  void *out_a, *out_b;
  long long M, nh, step;
  int np, depth;
  double inv_dt;
  int vel_rule, state_rule;
  PlaneParams p0, p1;
};
struct SweepArgs {
  const void *ring, *table;
  void *pending;
  const int *cls, *win;
  const long long *blk_off;
  const int *blk_cap, *blk_stride;
  const long long *cls_off;
  int cls_w0;             // rows of class 0 (its zero row follows them)
  long long M, step;
  int np;
  long long nphase;       // blocks of this launch's sweep phase
};

// fault.hip: interface solve of a frictional fault between the two sides.
// Fields are [component][cell] with cell = i1 * n3 + i3; u, v hold the upper
// side in components 0..2 and the lower side in 3..5.
struct FaultArgs {
  const void *functional;     // [P][3][cells] working precision: tractions without damping
  const double *tau0, *mu_s, *mu_k, *d_c;
  double *u, *v;              // [2][3][cells]
  double *slip, *rate;        // [2][cells]: components (x1, x3)
  double *tau;                // [3][cells]
  double *tau_out, *rate_out; // optional copies for the caller
  void *push;                 // [P][3][cells] working precision: input of the next push
  long long cells;
  double zp[3], zm[3];        // eta_ii mu / c_s of the upper and lower side
  double dt;
  int increment;              // the next push takes the increment dt v instead of u
};
hipError_t launch_fault_step(bool fp64, bool mirror, const FaultArgs &a, hipStream_t st);
hipError_t launch_fault_check(const double *tau0, const double *mu_s, const double *mu_k,
                              const double *d_c, long long cells, long long *bad, hipStream_t st);
// strip.hip: finite-element strip of the hybrid scheme.  Node fields are
// float64 [3][n2+1][n1][n3] over the storage node layers; cell fields
// [rows][n1][n3].  One-sided (the fault a symmetry plane): layer 0 is the
// fault, layer n2 is S+.  Two-sided: layers 0..fault_lo are the block below the
// fault (0 = S-, fault_lo = the lower copy of the split fault nodes), layers
// fault_hi = fault_lo + 1 .. n2 the block above it (n2 = S+).
struct StripArgs {
  const double *u;            // [3][nodes] u_{t+1}, read by the stencil
  double *u_next;             // [3][nodes] u_{t+2}, written (the other displacement buffer)
  double *vh;                 // [3][nodes] in: v_{t+1/2}; out: v_{t+3/2}
  double *v;                  // [3][nodes] out: v_{t+1}
  const double *stencil;      // [n2+1][27][3][3]: stiffness block of each neighbour offset
                              // (o1, o2, o3), index (o1+1) + 3 (o2+1) + 9 (o3+1)
  const double *mass;         // [n2+1] lumped mass of a node of each layer
  const void *tau_sbi;        // [P][3][cells] working precision: tractions at S+ (and S-)
  void *push_u, *push_v;      // [P][3][cells] working precision: S+ (and S-) displacement
                              // (or increment) and predicted velocity of the next step
  double *r_fault;            // two-sided: [2][3][cells] forces on the upper, lower fault copy
  const double *tau0, *mu_s, *mu_k, *d_c;
  double *tau, *rate, *slip, *sliding;   // fault outputs [3], [2], [2], [1] x cells
  double *tau_out, *rate_out;            // optional caller copies
  long long nodes, cells;
  int n1, n3, n2;
  int fault_lo;               // two-sided: storage layer of the lower fault copy; -1 one-sided
  double dt, area;
  int increment;
};
hipError_t launch_strip_correct(bool fp64, const StripArgs &a, hipStream_t st);
hipError_t launch_strip_fault2(const StripArgs &a, hipStream_t st);
hipError_t launch_strip_repredict(bool fp64, double *u_pred, const double *u_prev, double *vh,
                                  const double *v, void *push_u, void *push_v, long long nodes,
                                  long long cells, bool two_sided, bool increment, double dt,
                                  double dt_old, hipStream_t st);
hipError_t launch_tabulate(bool fp64, const Group &g, double dt, const double *gl_x,
                           const double *gl_w, hipStream_t st);

}  // namespace sbim
