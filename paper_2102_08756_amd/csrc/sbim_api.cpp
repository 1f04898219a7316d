// C ABI of the boundary-integral library: configuration checks, the mode
// ordering and kernel-row classes, device memory, and the per-call launch
// sequences.  No arithmetic of the method runs here; it all runs in the HIP
// kernels of fft.hip and kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "api_internal.h"
#include "checks.h"

using sbim::Group;

namespace sbim_api {

thread_local std::string g_init_error;

int fail(sbim_handle *h, int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (h)
    h->err = buf;
  else
    g_init_error = buf;
  return code;
}

int hip_fail(sbim_handle *h, hipError_t e, const char *what) {
  return fail(h, SBIM_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool pow2_in(int n, int lo, int hi) { return n >= lo && n <= hi && (n & (n - 1)) == 0; }

bool finite_pos(double x) { return std::isfinite(x) && x > 0; }

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_n in long double.
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
  x.resize(n);
  w.resize(n);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < n; ++i) {
    long double z = cosl(pi * (i + 0.75L) / (n + 0.5L));
    long double dp = 0;
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1);
      const long double dz = p1 / dp;
      z -= dz;
      if (fabsl(dz) < 1e-19L) break;
    }
    long double p0 = 1, p1 = z;
    for (int k = 2; k <= n; ++k) {
      const long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1);
    x[i] = static_cast<double>(z);
    w[i] = static_cast<double>(2 / ((1 - z * z) * dp * dp));
  }
}

struct ModeKey {
  int w;
  double q;
  int nat;
};

hipError_t dev_alloc_bytes(void **p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) return hipSuccess;
  return hipMalloc(p, bytes);
}

void free_group(Group &g) {
  void *ptrs[] = {g.nat,   g.cls,   g.win,   g.geom,      g.blk_off,   g.blk_cap, g.blk_stride, g.cls_off,
                  g.cls_q, g.cls_w, g.table, g.ring,      g.state,     g.pending,
                  g.ring_adj, g.state_adj, g.lam_adj, g.pending_adj};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  g = Group();
}

void free_handle(sbim_handle *h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  for (int i = 0; i < h->ngroups; ++i) free_group(h->g[i]);
  if (h->twiddle64 && h->twiddle64 != h->twiddle) (void)hipFree(h->twiddle64);
  void *ptrs[] = {h->twiddle, h->spec, h->spec_v, h->out_spec, h->out_adj};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  for (auto e : h->ev_start) (void)hipEventDestroy(e);
  for (auto e : h->ev_stop) (void)hipEventDestroy(e);
  delete h;
}

long long ring_bytes(const sbim_handle *h, const Group &g) {
  return g.ring_records * g.np * 3LL * sbim::kLanes * 2 * static_cast<long long>(h->rsize);
}
long long table_bytes(const sbim_handle *h, const Group &g) {
  return g.table_rows * 4LL * static_cast<long long>(h->rsize);
}
long long state_bytes_g(const Group &g) { return g.np * 3LL * g.M * 16; }
long long pending_bytes(const sbim_handle *h, const Group &g) {
  return (h->depth + 1LL) * g.np * 10LL * g.M * static_cast<long long>(h->rsize);
}
long long out_spec_bytes(const sbim_handle *h) {
  return static_cast<long long>(h->cfg.nplanes) * 3 * h->nh * 2 * static_cast<long long>(h->rsize);
}

int validate(const sbim_config *c) {
  if (!c) return fail(nullptr, SBIM_E_INVALID, "config is NULL");
  if (!pow2_in(c->n1, 4, 4096) || !pow2_in(c->n3, 4, 4096))
    return fail(nullptr, SBIM_E_INVALID, "n1=%d, n3=%d: each must be a power of two in [4, 4096]",
                c->n1, c->n3);
  if (!finite_pos(c->dx1) || !finite_pos(c->dx3) || !finite_pos(c->dt))
    return fail(nullptr, SBIM_E_INVALID, "dx1, dx3 and dt must be finite and > 0");
  if (c->nplanes < 1 || c->nplanes > SBIM_MAX_PLANES)
    return fail(nullptr, SBIM_E_INVALID, "nplanes=%d: must be 1 or 2", c->nplanes);
  for (int p = 0; p < c->nplanes; ++p) {
    const sbim_plane &pl = c->plane[p];
    if (pl.side != 1 && pl.side != -1)
      return fail(nullptr, SBIM_E_INVALID, "plane %d: side must be +1 or -1", p);
    if (!finite_pos(pl.mu) || !finite_pos(pl.cs) || !std::isfinite(pl.cp))
      return fail(nullptr, SBIM_E_INVALID, "plane %d: mu, cs must be finite and > 0", p);
    if (!(pl.cp > pl.cs * std::sqrt(4.0 / 3.0)))
      return fail(nullptr, SBIM_E_INVALID,
                  "plane %d: cp=%g must exceed cs*sqrt(4/3)=%g (positive bulk modulus)", p, pl.cp,
                  pl.cs * std::sqrt(4.0 / 3.0));
  }
  if (c->window_cap < 1 || c->window_cap > (1 << 20))
    return fail(nullptr, SBIM_E_INVALID, "window_cap=%d: must be in [1, 2^20]", c->window_cap);
  if (c->window_mode != SBIM_W_FIXED && c->window_mode != SBIM_W_PER_MODE &&
      c->window_mode != SBIM_W_STATIC)
    return fail(nullptr, SBIM_E_INVALID, "window_mode=%d unknown", c->window_mode);
  if (c->window_mode == SBIM_W_PER_MODE && !finite_pos(c->eta_w))
    return fail(nullptr, SBIM_E_INVALID, "eta_w must be finite and > 0");
  if (c->precision != SBIM_FP64 && c->precision != SBIM_FP32 && c->precision != SBIM_FP32_COMP)
    return fail(nullptr, SBIM_E_INVALID, "precision=%d unknown", c->precision);
  if (c->input_kind != SBIM_ABSOLUTE && c->input_kind != SBIM_INCREMENT)
    return fail(nullptr, SBIM_E_INVALID, "input_kind=%d unknown", c->input_kind);
  return SBIM_OK;
}

// Mean history window over the half-spectrum's modes of a plane with shear
// wave speed cs (the per-mode window rule of plan_group).
double mean_window(const sbim_config &c, double cs) {
  if (c.window_mode == SBIM_W_STATIC) return 1.0;
  if (c.window_mode == SBIM_W_FIXED) return c.window_cap;
  const int n1 = c.n1, h3 = c.n3 / 2 + 1;
  const double two_pi = 2.0 * M_PI;
  double sum = 0;
  for (int i1 = 0; i1 < n1; ++i1) {
    const int m1 = i1 < n1 / 2 ? i1 : i1 - n1;
    const double k1 = (two_pi * m1) / (n1 * c.dx1);
    for (int i3 = 0; i3 < h3; ++i3) {
      const double k3 = (two_pi * i3) / (c.n3 * c.dx3);
      const double q = std::sqrt(k1 * k1 + k3 * k3);
      if (q > 0)
        sum += std::min(static_cast<double>(c.window_cap),
                        std::ceil((two_pi * c.eta_w) / (q * cs * c.dt)));
    }
  }
  return sum / (static_cast<double>(n1) * h3);
}

// Mode geometry, windows, ordering and classes of one material group (host).
// With `quads` (the matrix-core sweep) every class starts at a multiple of 4
// sorted positions and is padded to a multiple of 4 with positions that hold
// no mode (bin -1, window 0, the class's row set), so each aligned group of
// four lanes shares one kernel row.
void plan_group(const sbim_config &c, int depth, bool quads, Group &g, std::vector<double> &geom,
                std::vector<long long> &blk_off, std::vector<int> &blk_cap,
                std::vector<int> &blk_stride, std::vector<double> &cls_q) {
  const int n1 = c.n1, h3 = c.n3 / 2 + 1;
  const long long M = static_cast<long long>(n1) * h3;
  const double two_pi = 2.0 * M_PI;
  std::vector<ModeKey> keys(M);
  std::vector<double> qv(M), k1v(M), k3v(M);
  for (int i1 = 0; i1 < n1; ++i1) {
    const int m1 = i1 < n1 / 2 ? i1 : i1 - n1;
    const double k1 = (two_pi * m1) / (n1 * c.dx1);
    for (int i3 = 0; i3 < h3; ++i3) {
      const double k3 = (two_pi * i3) / (c.n3 * c.dx3);
      const double q = std::sqrt(k1 * k1 + k3 * k3);
      int w = 0;
      if (q > 0) {
        if (c.window_mode == SBIM_W_STATIC) {
          w = 1;
        } else if (c.window_mode == SBIM_W_FIXED) {
          w = c.window_cap;
        } else {
          const double x = (two_pi * c.eta_w) / (q * g.cs * c.dt);
          w = static_cast<int>(std::min(static_cast<double>(c.window_cap), std::ceil(x)));
        }
      }
      const long long f = static_cast<long long>(i3) * n1 + i1;  // spectrum bin
      keys[f] = ModeKey{w, q, static_cast<int>(f)};
      qv[f] = q;
      k1v[f] = k1;
      k3v[f] = k3;
    }
  }
  // Blocks hold modes of equal window.  With one window for all modes, modes
  // of equal q sit together so that a block's lanes share kernel rows.  With
  // per-mode windows (short histories, where the push and traction gathers
  // dominate) modes of equal window stay in spectrum order, so the gathers of
  // the spectrum and the scatters of the traction spectrum are contiguous runs.
  const bool by_q = c.window_mode != SBIM_W_PER_MODE;
  std::sort(keys.begin(), keys.end(), [by_q](const ModeKey &a, const ModeKey &b) {
    if (a.w != b.w) return a.w > b.w;
    if (by_q && a.q != b.q) return a.q < b.q;
    return a.nat < b.nat;
  });
  if (quads) {
    // pad each run of equal (W, q) (a class, sorted together) to a multiple of 4;
    // a padding position carries nat = -1
    std::vector<ModeKey> padded;
    padded.reserve(M + M / 2);
    for (long long s0 = 0; s0 < M;) {
      long long s1 = s0;
      while (s1 < M && keys[s1].w == keys[s0].w && keys[s1].q == keys[s0].q) ++s1;
      for (long long s = s0; s < s1; ++s) padded.push_back(keys[s]);
      for (long long r = (s1 - s0) % 4; r != 0 && r < 4; ++r)
        padded.push_back(ModeKey{keys[s0].w, keys[s0].q, -1});
      s0 = s1;
    }
    keys.swap(padded);
  }
  const long long Ms = static_cast<long long>(keys.size());  // sorted positions
  g.M = Ms;
  g.nblocks = (Ms + sbim::kLanes - 1) / sbim::kLanes;
  g.h_nat.resize(Ms);
  g.h_cls.resize(Ms);
  g.h_win.resize(Ms);
  geom.assign(4 * Ms, 0.0);
  cls_q.clear();
  g.h_cls_w.clear();
  // a class per distinct (W, q): kernel rows are shared whatever the order
  std::map<std::pair<int, double>, int> class_of;
  for (long long s = 0; s < Ms; ++s) {
    const ModeKey &k = keys[s];
    if (k.nat < 0) {  // padding: the class of the position before it, no window, no bin
      g.h_nat[s] = -1;
      g.h_cls[s] = g.h_cls[s - 1];
      g.h_win[s] = 0;
      continue;
    }
    int cls = 0;
    if (k.w > 0) {
      bool known = false;
      if (by_q) {                    // sorted by (W, q): equal keys are neighbours
        known = s > 0 && k.w == keys[s - 1].w && k.q == keys[s - 1].q;
        if (known) cls = g.h_cls[s - 1];
      } else {
        auto it = class_of.find({k.w, k.q});
        known = it != class_of.end();
        if (known) cls = it->second;
      }
      if (!known) {
        cls = static_cast<int>(cls_q.size());
        if (!by_q) class_of.emplace(std::make_pair(k.w, k.q), cls);
        cls_q.push_back(k.q);
        g.h_cls_w.push_back(k.w);
      }
    }
    g.h_nat[s] = k.nat;
    g.h_cls[s] = cls;
    g.h_win[s] = k.w;
    const double q = qv[k.nat];
    geom[4 * s + 0] = q;
    geom[4 * s + 1] = q > 0 ? k1v[k.nat] / q : 1.0;
    geom[4 * s + 2] = q > 0 ? k3v[k.nat] / q : 0.0;
  }
  g.nclasses = static_cast<long long>(cls_q.size());
  g.wmax = Ms > 0 ? keys[0].w : 0;
  blk_off.resize(g.nblocks);
  blk_cap.resize(g.nblocks);
  blk_stride.resize(g.nblocks);
  for (long long b = 0; b < g.nblocks; ++b) {  // the largest window of the block's modes
    int cap = 0;
    for (long long s = b * sbim::kLanes; s < std::min(Ms, (b + 1) * sbim::kLanes); ++s)
      cap = std::max(cap, g.h_win[s]);
    blk_cap[b] = cap;
  }
  g.h_blk_cap = blk_cap;
  // Blocks of one sweep phase (b mod depth) are stored together; within a
  // phase, runs of consecutive blocks with equal capacity are stored slot-major.
  long long rec = 0;
  for (int ph = 0; ph < depth; ++ph) {
    for (long long b0 = ph; b0 < g.nblocks;) {
      long long b1 = b0, len = 0;
      while (b1 < g.nblocks && blk_cap[b1] == blk_cap[b0]) {
        b1 += depth;
        ++len;
      }
      for (long long b = b0, i = 0; b < b1; b += depth, ++i) {
        blk_off[b] = rec + i;
        blk_stride[b] = static_cast<int>(len);
      }
      rec += static_cast<long long>(blk_cap[b0]) * len;
      b0 = b1;
    }
  }
  g.ring_records = rec;
  // class-major table: the W_c rows of class c start at entry cls_off[c] and
  // are followed by one zero row
  g.h_cls_off.assign(g.nclasses, 0);
  long long off = 0;
  for (long long c = 0; c < g.nclasses; ++c) {
    g.h_cls_off[c] = off;
    off += g.h_cls_w[c] + 1;
  }
  g.table_rows = off;
}

hipError_t upload(void *dst, const void *src, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
}

int check_ptr(sbim_handle *h, const void *p, const char *name) {
  if (!p) return fail(h, SBIM_E_INVALID, "%s is NULL", name);
  return SBIM_OK;
}

// Forward real 2-D FFT of a [P][3][n1][n3] field into `spec`.
hipError_t fft_forward(sbim_handle *h, const void *field, void *spec) {
  return sbim::launch_fft_forward(h->fp64, field, spec, h->cfg.nplanes * 3, h->n1, h->n3,
                                  h->twiddle64, h->stream);
}

// Inverse of a traction spectrum (destroyed) into a [P][3][n1][n3] field.
hipError_t fft_inverse(sbim_handle *h, const void *spec, void *scratch, void *field,
                       const void *add) {
  return sbim::launch_fft_inverse(h->fp64, spec, scratch, field, add, h->cfg.nplanes * 3, h->n1,
                                  h->n3,
                                  1.0 / (static_cast<double>(h->n1) * h->n3), h->twiddle,
                                  h->stream);
}

// Adjoint buffers of every group, allocated and cleared on first use.  A group
// is complete once its state_adj is set; a failed allocation or clear frees
// that group's partial buffers again, so a later call starts from scratch.
int ensure_adjoint(sbim_handle *h) {
  for (int i = 0; i < h->ngroups; ++i) {
    Group &g = h->g[i];
    if (g.state_adj) continue;
    const size_t rb = static_cast<size_t>(ring_bytes(h, g));
    const size_t sb = static_cast<size_t>(state_bytes_g(g));
    const size_t pb = static_cast<size_t>(pending_bytes(h, g));
    size_t free_b = 0, total_b = 0;
    const size_t need = rb + 2 * sb + pb + (h->out_adj ? 0 : static_cast<size_t>(out_spec_bytes(h)));
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && need > free_b)
      return fail(h, SBIM_E_OOM, "adjoint buffers need %zu bytes, %zu free", need, free_b);
    void *ring = nullptr, *pending = nullptr;
    double *state = nullptr, *lam = nullptr;
    auto release = [&]() {
      void *ptrs[] = {ring, pending, state, lam};
      for (void *q : ptrs)
        if (q) (void)hipFree(q);
    };
    hipError_t e;
    if ((e = dev_alloc_bytes(&ring, rb)) != hipSuccess ||
        (e = dev_alloc_bytes(&pending, pb)) != hipSuccess ||
        (e = dev_alloc(&state, sb / 8)) != hipSuccess ||
        (e = dev_alloc(&lam, sb / 8)) != hipSuccess) {
      release();
      return fail(h, SBIM_E_OOM, "adjoint allocation failed: %s", hipGetErrorString(e));
    }
    if (!h->out_adj && (e = dev_alloc_bytes(&h->out_adj, out_spec_bytes(h))) != hipSuccess) {
      release();
      return fail(h, SBIM_E_OOM, "adjoint allocation failed: %s", hipGetErrorString(e));
    }
    e = rb ? hipMemsetAsync(ring, 0, rb, h->stream) : hipSuccess;
    if (e == hipSuccess) e = hipMemsetAsync(state, 0, sb, h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(lam, 0, sb, h->stream);
    if (e != hipSuccess) {
      (void)hipStreamSynchronize(h->stream);
      release();
      return hip_fail(h, e, "clearing adjoint state");
    }
    g.ring_adj = ring;
    g.pending_adj = pending;
    g.lam_adj = lam;
    g.state_adj = state;
  }
  return SBIM_OK;
}

// The launch of step `w.step` for one group (push, traction spectrum and the
// sweep for the coming steps); while sbim_profile_conv is on, every n-th such
// launch is bracketed by a pair of the handle's reusable events.
int step_group(sbim_handle *h, Group &g, const sbim::StepLaunch &w, bool timed) {
  hipError_t e;
  if (timed && h->profile_every > 0 && h->profile_seen++ % h->profile_every == 0) {
    if (h->ev_used == h->ev_start.size()) {  // grow the reusable event pool
      hipEvent_t e0, e1;
      if ((e = hipEventCreate(&e0)) != hipSuccess) return hip_fail(h, e, "hipEventCreate");
      if ((e = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(h, e, "hipEventCreate");
      }
      h->ev_start.push_back(e0);
      h->ev_stop.push_back(e1);
    }
    e = sbim::launch_step(h, g, w, h->ev_start[h->ev_used], h->ev_stop[h->ev_used]);
    ++h->ev_used;
  } else {
    e = sbim::launch_step(h, g, w);
  }
  if (e != hipSuccess) return hip_fail(h, e, "step kernel");
  return SBIM_OK;
}

// One forward step: transform u (and v for VEL_INPUT), then the step launch of
// every material group with the given rule for the damping term's velocity.
int push_fields(sbim_handle *h, const void *u, const void *v, int vel_rule) {
  hipError_t e = fft_forward(h, u, h->spec);
  if (e != hipSuccess) return hip_fail(h, e, "forward FFT of u");
  if (vel_rule == sbim::VEL_INPUT) {
    e = fft_forward(h, v, h->spec_v);
    if (e != hipSuccess) return hip_fail(h, e, "forward FFT of v");
  }
  const bool incr = h->cfg.input_kind == SBIM_INCREMENT;
  for (int i = 0; i < h->ngroups; ++i) {
    Group &g = h->g[i];
    sbim::StepLaunch w;
    w.spec = h->spec;
    w.spec_v = vel_rule == sbim::VEL_INPUT ? h->spec_v : nullptr;
    w.ring = g.ring;
    w.state = g.state;
    w.pending = g.pending;
    w.lam = nullptr;
    w.out_a = h->out_spec;
    w.out_b = nullptr;
    w.nh = h->nh;
    w.step = h->step;
    w.dt = h->cfg.dt;
    w.state_rule = incr ? sbim::STATE_ACCUM : sbim::STATE_REPLACE;
    w.vel_rule = vel_rule;
    int rc = step_group(h, g, w, true);
    if (rc) return rc;
  }
  h->step += 1;
  return SBIM_OK;
}

}  // namespace sbim_api

using namespace sbim_api;

extern "C" {

int sbim_init(const sbim_config *cfg, sbim_handle **out) {
  if (!out) return fail(nullptr, SBIM_E_INVALID, "out is NULL");
  *out = nullptr;
  int rc = validate(cfg);
  if (rc != SBIM_OK) return rc;
  sbim_handle *h = new (std::nothrow) sbim_handle();
  if (!h) return fail(nullptr, SBIM_E_OOM, "host allocation failed");
  h->cfg = *cfg;
  h->stream = static_cast<hipStream_t>(cfg->stream);
  h->fp64 = cfg->precision == SBIM_FP64;
  h->comp = cfg->precision == SBIM_FP32_COMP;
  h->rsize = h->fp64 ? 8 : 4;
  h->n1 = cfg->n1;
  h->n3 = cfg->n3;
  h->h3 = cfg->n3 / 2 + 1;
  h->nh = static_cast<long long>(h->n1) * h->h3;
  hipError_t e = hipGetDevice(&h->device);
  if (e != hipSuccess) {
    delete h;
    return fail(nullptr, SBIM_E_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
  }
  // the device address of the allocation-free count's static scratch (once per device)
  e = sbim::count_scratch_address(h->device, &h->count_scratch);
  if (e != hipSuccess) {
    delete h;
    return fail(nullptr, SBIM_E_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s",
                h->device, hipGetErrorString(e));
  }

  // material groups: planes with equal (c_s, c_p) share kernel tables and one pass
  for (int p = 0; p < cfg->nplanes; ++p) {
    const sbim_plane &pl = cfg->plane[p];
    int gi = -1;
    for (int i = 0; i < h->ngroups; ++i)
      if (h->g[i].cs == pl.cs && h->g[i].cp == pl.cp) gi = i;
    if (gi < 0) {
      gi = h->ngroups++;
      h->g[gi].cs = pl.cs;
      h->g[gi].cp = pl.cp;
      h->g[gi].eta = pl.cp / pl.cs;
    }
    Group &g = h->g[gi];
    g.pl[g.np++] = sbim::PlaneParams{pl.mu, pl.cs, pl.cp / pl.cs, pl.side, p};
  }

  struct HostPlan {
    std::vector<double> geom, cls_q;
    std::vector<long long> blk_off;
    std::vector<int> blk_cap, blk_stride;
  };
  // Sweep depth: steps served by one pass over a block's history.  Deeper
  // sweeps divide the history traffic, but the newest lags of each step (up
  // to depth + 1 of them) are summed by the mode items.  A lane holds the 10
  // sums of up to 8 steps (float32) or 6 (float64 and the compensated form,
  // whose sums take two registers each); depths 12 and 16 give each mode two
  // lanes, one per half of the steps.  Measured on gfx950 (two planes,
  // 512^2 at W = 1000, 1024^2 at W = 2000, 2048^2 with per-mode windows of
  // mean 18 lags): with long windows float64 and the compensated form run
  // fastest at 12; float32 at 8 for W = 1000 (by 5%) and at 12 for W = 2000
  // (by 7%); with mean windows under 64 lags every form runs fastest at 6.
  double wbar = 0;
  for (int p = 0; p < cfg->nplanes; ++p)
    wbar = std::max(wbar, mean_window(*cfg, cfg->plane[p].cs));
  h->depth = wbar < 64 ? 6 : (h->comp || h->fp64 || wbar >= 1500 ? 12 : 8);
  // Matrix-core sweep: float32 history, one window for every mode, both planes
  // in one material group (their kernel rows shared), windows long enough for
  // the deep sweep to pay.  Its depth is 16 or 32 (one or two 16-step groups of
  // the 16x16x4 products); measured on gfx950 (two planes 512^2 at W = 1000,
  // 1024^2 at W = 2000): 32 for both float32 forms.
  const bool mfma_able = !h->fp64 && cfg->window_mode == SBIM_W_FIXED && h->ngroups == 1 &&
                         h->g[0].np == 2;
  h->mfma = mfma_able && wbar >= 64;
  if (const char *env = std::getenv("SBIM_SWEEP_KIND")) {  // tuning override
    if (std::strcmp(env, "valu") == 0) h->mfma = false;
    if (std::strcmp(env, "mfma") == 0) h->mfma = mfma_able;
  }
  if (h->mfma) h->depth = 32;
  if (const char *env = std::getenv("SBIM_SWEEP_DEPTH")) {  // tuning override
    const int v = std::atoi(env);
    if (h->mfma) {
      if (v == 16 || v == 32) h->depth = v;
    } else if (v == 1 || v == 2 || v == 4 || v == 6 || v == 8 || v == 12 || v == 16) {
      h->depth = v;
    }
  }
  std::vector<HostPlan> plan(h->ngroups);
  size_t need = 0;
  for (int i = 0; i < h->ngroups; ++i) {
    Group &g = h->g[i];
    plan_group(*cfg, h->depth, h->mfma, g, plan[i].geom, plan[i].blk_off, plan[i].blk_cap,
               plan[i].blk_stride, plan[i].cls_q);
    need += ring_bytes(h, g) + table_bytes(h, g) + state_bytes_g(g);
    need += pending_bytes(h, g);
    need += g.M * (4 * 3 + 32) + g.nblocks * 16 + g.nclasses * 20;
  }
  if (h->mfma) {
    // The quad sweep addresses a block's history with 32-bit byte offsets from
    // its slot 0: every block's capacity times its slot stride must stay below
    // 2^30 floats, else the vector-unit sweep plans the group instead.
    const Group &g0 = h->g[0];
    bool fits = true;
    for (long long b = 0; b < g0.nblocks; ++b)
      if (static_cast<long long>(plan[0].blk_cap[b]) * plan[0].blk_stride[b] * 2 * 3 * sbim::kLanes * 2 >=
          (1LL << 30))
        fits = false;
    if (!fits) {
      h->mfma = false;
      h->depth = wbar < 64 ? 6 : (h->comp || wbar >= 1500 ? 12 : 8);
      need = 0;
      Group &g = h->g[0];
      const double cs = g.cs, cp = g.cp, eta = g.eta;
      const int np = g.np;
      sbim::PlaneParams pl[SBIM_MAX_PLANES] = {g.pl[0], g.pl[1]};
      g = Group();
      g.cs = cs, g.cp = cp, g.eta = eta, g.np = np;
      for (int k = 0; k < np; ++k) g.pl[k] = pl[k];
      plan[0] = HostPlan();
      plan_group(*cfg, h->depth, false, g, plan[0].geom, plan[0].blk_off, plan[0].blk_cap,
                 plan[0].blk_stride, plan[0].cls_q);
      need += ring_bytes(h, g) + table_bytes(h, g) + state_bytes_g(g) + pending_bytes(h, g);
      need += g.M * (4 * 3 + 32) + g.nblocks * 16 + g.nclasses * 20;
    }
  }
  if (h->mfma) {
    // Wavefronts per quad (lag ranges, each at least 16 blocks of 4 lags),
    // measured on gfx950 (two planes 512^2 at W = 1000, 1024^2 at W = 2000):
    // two for the compensated form (its registers allow three wavefronts per
    // SIMD), four for plain float32.
    const Group &g = h->g[0];
    const int nblk = (std::max(0, g.wmax - 2) + 3) / 4;
    const int want = h->comp ? 2 : 4;
    h->lag_chunks = 1;
    while (h->lag_chunks < want && nblk >= 16 * 2 * h->lag_chunks) h->lag_chunks *= 2;
    if (const char *env = std::getenv("SBIM_SWEEP_CHUNKS")) {  // tuning override
      const int v = std::atoi(env);
      if (v == 1 || v == 2 || v == 4) h->lag_chunks = v;
    }
    // Quads per work-group: neighbouring quads of a block share the cache lines
    // of their history (a line holds 4 quads' pieces), and in one work-group they
    // stream them together.  Measured on gfx950: two for the compensated form
    // (1024^2 at W = 2000: 5% faster; 512^2 at W = 1000: 1% faster since the
    // mode items run XCD-contiguous, 1% slower before), one for plain float32 with
    // its four lag ranges (two quads of two ranges: 6% slower at 512^2).
    h->sweep_quads = (h->comp && h->lag_chunks <= 2) ? 2 : 1;
    if (const char *env = std::getenv("SBIM_SWEEP_QUADS")) {  // tuning override
      const int v = std::atoi(env);
      if ((v == 1 || v == 2 || v == 4) && v * h->lag_chunks <= 4) h->sweep_quads = v;
    }
  }
  // input spectra are float64 in every form; the traction spectrum is real_t
  const size_t spec_bytes = static_cast<size_t>(cfg->nplanes) * 3 * h->nh * 2 * sizeof(double);
  const size_t out_bytes = static_cast<size_t>(cfg->nplanes) * 3 * h->nh * 2 * h->rsize;
  need += 2 * spec_bytes + out_bytes + sbim::kTwiddleN * 2 * (h->rsize + sizeof(double));
  size_t free_b = 0, total_b = 0;
  e = hipMemGetInfo(&free_b, &total_b);
  if (e != hipSuccess) {
    free_handle(h);
    return fail(nullptr, SBIM_E_DEVICE, "hipMemGetInfo: %s", hipGetErrorString(e));
  }
  if (need > free_b) {
    free_handle(h);
    return fail(nullptr, SBIM_E_OOM, "needs %zu bytes of device memory, %zu free", need, free_b);
  }


  std::vector<double> glx, glw;
  gauss_legendre(sbim::kGaussN, glx, glw);
  double *d_glx = nullptr, *d_glw = nullptr;

#define TRY(expr)                                         \
  do {                                                    \
    e = (expr);                                           \
    if (e != hipSuccess) {                                \
      const int code = (e == hipErrorOutOfMemory) ? SBIM_E_OOM : SBIM_E_DEVICE; \
      if (d_glx) (void)hipFree(d_glx);                    \
      if (d_glw) (void)hipFree(d_glw);                    \
      free_handle(h);                                     \
      return fail(nullptr, code, "%s: %s", #expr, hipGetErrorString(e)); \
    }                                                     \
  } while (0)

  TRY(dev_alloc_bytes(&h->twiddle, sbim::kTwiddleN * 2 * h->rsize));
  if (h->fp64) {
    h->twiddle64 = h->twiddle;
  } else {
    TRY(dev_alloc_bytes(&h->twiddle64, sbim::kTwiddleN * 2 * sizeof(double)));
    TRY(sbim::upload_twiddles(true, h->twiddle64, h->stream));
  }
  TRY(dev_alloc_bytes(&h->spec, spec_bytes));
  TRY(dev_alloc_bytes(&h->spec_v, spec_bytes));
  TRY(dev_alloc_bytes(&h->out_spec, out_bytes));
  TRY(sbim::upload_twiddles(h->fp64, h->twiddle, h->stream));
  TRY(dev_alloc(&d_glx, glx.size()));
  TRY(dev_alloc(&d_glw, glw.size()));
  TRY(upload(d_glx, glx.data(), glx.size() * sizeof(double), h->stream));
  TRY(upload(d_glw, glw.data(), glw.size() * sizeof(double), h->stream));
  for (int i = 0; i < h->ngroups; ++i) {
    Group &g = h->g[i];
    HostPlan &hp = plan[i];
    TRY(dev_alloc(&g.nat, g.M));
    TRY(dev_alloc(&g.cls, g.M));
    TRY(dev_alloc(&g.win, g.M));
    TRY(dev_alloc(&g.geom, 4 * g.M));
    TRY(dev_alloc(&g.blk_off, g.nblocks));
    TRY(dev_alloc(&g.blk_cap, g.nblocks));
    TRY(dev_alloc(&g.blk_stride, g.nblocks));
    TRY(dev_alloc(&g.cls_off, g.nclasses));
    TRY(dev_alloc(&g.cls_q, g.nclasses));
    TRY(dev_alloc(&g.cls_w, g.nclasses));
    TRY(dev_alloc_bytes(&g.table, table_bytes(h, g)));
    TRY(dev_alloc_bytes(&g.ring, ring_bytes(h, g)));
    TRY(dev_alloc(&g.state, state_bytes_g(g) / 8));
    TRY(dev_alloc_bytes(&g.pending, pending_bytes(h, g)));
    TRY(upload(g.nat, g.h_nat.data(), g.M * sizeof(int), h->stream));
    TRY(upload(g.cls, g.h_cls.data(), g.M * sizeof(int), h->stream));
    TRY(upload(g.win, g.h_win.data(), g.M * sizeof(int), h->stream));
    TRY(upload(g.geom, hp.geom.data(), hp.geom.size() * sizeof(double), h->stream));
    TRY(upload(g.blk_off, hp.blk_off.data(), hp.blk_off.size() * sizeof(long long), h->stream));
    TRY(upload(g.blk_cap, hp.blk_cap.data(), hp.blk_cap.size() * sizeof(int), h->stream));
    TRY(upload(g.blk_stride, hp.blk_stride.data(), hp.blk_stride.size() * sizeof(int), h->stream));
    TRY(upload(g.cls_off, g.h_cls_off.data(), g.h_cls_off.size() * sizeof(long long), h->stream));
    TRY(upload(g.cls_q, hp.cls_q.data(), hp.cls_q.size() * sizeof(double), h->stream));
    TRY(upload(g.cls_w, g.h_cls_w.data(), g.h_cls_w.size() * sizeof(int), h->stream));
    if (ring_bytes(h, g)) TRY(hipMemsetAsync(g.ring, 0, ring_bytes(h, g), h->stream));
    TRY(hipMemsetAsync(g.state, 0, state_bytes_g(g), h->stream));
    TRY(hipMemsetAsync(g.pending, 0, pending_bytes(h, g), h->stream));
    if (cfg->window_mode == SBIM_W_STATIC) {
      // one row per class: the static integrals G_ab(infinity) of the kernels,
      // i.e. the static surface stiffness K_ab(0) less the instantaneous L-N
      // coupling, (w11, w12, w22, w33); then the zero row
      const double e2 = g.eta * g.eta;
      const double row[4] = {2.0 * e2 / (e2 + 1.0), -2.0 / (e2 + 1.0) - (g.eta - 2.0),
                             2.0 * e2 / (e2 + 1.0), 1.0};
      std::vector<double> t64(static_cast<size_t>(g.table_rows) * 4, 0.0);
      for (long long c = 0; c < g.nclasses; ++c)
        for (int k = 0; k < 4; ++k) t64[static_cast<size_t>(g.h_cls_off[c]) * 4 + k] = row[k];
      if (h->fp64) {
        TRY(upload(g.table, t64.data(), t64.size() * sizeof(double), h->stream));
        TRY(hipStreamSynchronize(h->stream));
      } else {
        std::vector<float> t32(t64.begin(), t64.end());
        TRY(upload(g.table, t32.data(), t32.size() * sizeof(float), h->stream));
        TRY(hipStreamSynchronize(h->stream));
      }
    } else {
      TRY(sbim::launch_tabulate(h->fp64, g, cfg->dt, d_glx, d_glw, h->stream));
    }
    // the host vectors must outlive the asynchronous copies
    TRY(hipStreamSynchronize(h->stream));
  }
  TRY(hipStreamSynchronize(h->stream));
#undef TRY
  (void)hipFree(d_glx);
  (void)hipFree(d_glw);
  *out = h;
  return SBIM_OK;
}

int sbim_push_displacement(sbim_handle *h, const void *u, const void *v) {
  if (!h) return fail(nullptr, SBIM_E_INVALID, "handle is NULL");
  int rc = check_ptr(h, u, "u");
  if (rc) return rc;
  const bool incr = h->cfg.input_kind == SBIM_INCREMENT;
  return push_fields(h, u, v, v ? sbim::VEL_INPUT : (incr ? sbim::VEL_SCALE : sbim::VEL_DIFF));
}

int sbim_tractions(sbim_handle *h, const void *tau_inf, void *tau) {
  if (!h) return fail(nullptr, SBIM_E_INVALID, "handle is NULL");
  int rc = check_ptr(h, tau, "tau");
  if (rc) return rc;
  if (h->step == 0) return fail(h, SBIM_E_STATE, "sbim_tractions before any push");
  // the traction spectrum of the last step was completed by its push; the
  // forward spectrum buffer serves as scratch until the next push
  hipError_t e = fft_inverse(h, h->out_spec, h->spec, tau, tau_inf);
  if (e != hipSuccess) return hip_fail(h, e, "inverse FFT");
  return SBIM_OK;
}

int sbim_backward(sbim_handle *h, const void *g_tau, void *du, void *dv) {
  if (!h) return fail(nullptr, SBIM_E_INVALID, "handle is NULL");
  int rc = check_ptr(h, g_tau, "dL_dtau");
  if (rc) return rc;
  rc = check_ptr(h, du, "dL_du");
  if (rc) return rc;
  rc = ensure_adjoint(h);
  if (rc) return rc;
  hipError_t e = fft_forward(h, g_tau, h->spec);
  if (e != hipSuccess) return hip_fail(h, e, "forward FFT of dL/dtau");
  const bool incr = h->cfg.input_kind == SBIM_INCREMENT;
  for (int i = 0; i < h->ngroups; ++i) {
    Group &g = h->g[i];
    sbim::StepLaunch w;
    w.spec = h->spec;
    w.spec_v = nullptr;
    w.ring = g.ring_adj;
    w.state = g.state_adj;
    w.pending = g.pending_adj;
    w.lam = incr ? g.lam_adj : nullptr;
    w.out_a = h->out_adj;
    w.out_b = dv ? h->spec_v : nullptr;
    w.nh = h->nh;
    w.step = h->bstep;
    w.dt = h->cfg.dt;
    w.state_rule = sbim::STATE_REPLACE;
    // transpose of the velocity rule of the forward push
    w.vel_rule = dv ? sbim::VEL_COPY : (incr ? sbim::VEL_SCALE : sbim::VEL_DIFF);
    rc = step_group(h, g, w, false);
    if (rc) return rc;
  }
  e = fft_inverse(h, h->out_adj, h->spec, du, nullptr);
  if (e != hipSuccess) return hip_fail(h, e, "inverse FFT of dL/du");
  if (dv) {
    e = fft_inverse(h, h->spec_v, h->spec, dv, nullptr);
    if (e != hipSuccess) return hip_fail(h, e, "inverse FFT of dL/dv");
  }
  h->bstep += 1;
  return SBIM_OK;
}

int sbim_backward_reset(sbim_handle *h) {
  if (!h) return fail(nullptr, SBIM_E_INVALID, "handle is NULL");
  for (int i = 0; i < h->ngroups; ++i) {
    Group &g = h->g[i];
    if (!g.state_adj) continue;
    const size_t rb = static_cast<size_t>(ring_bytes(h, g));
    hipError_t e = hipSuccess;
    if (rb) e = hipMemsetAsync(g.ring_adj, 0, rb, h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(g.state_adj, 0, state_bytes_g(g), h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(g.lam_adj, 0, state_bytes_g(g), h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "clearing adjoint state");
  }
  h->bstep = 0;
  return SBIM_OK;
}

int sbim_reset(sbim_handle *h) {
  if (!h) return fail(nullptr, SBIM_E_INVALID, "handle is NULL");
  for (int i = 0; i < h->ngroups; ++i) {
    Group &g = h->g[i];
    hipError_t e = hipSuccess;
    if (ring_bytes(h, g)) e = hipMemsetAsync(g.ring, 0, ring_bytes(h, g), h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(g.state, 0, state_bytes_g(g), h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "clearing state");
  }
  h->step = 0;
  return sbim_backward_reset(h);
}

int sbim_destroy(sbim_handle *h) {
  free_handle(h);
  return SBIM_OK;
}

const char *sbim_last_error(const sbim_handle *h) {
  return h ? h->err.c_str() : g_init_error.c_str();
}

int sbim_set_stream(sbim_handle *h, void *stream) {
  if (!h) return fail(nullptr, SBIM_E_INVALID, "handle is NULL");
  hipStream_t next = static_cast<hipStream_t>(stream);
  if (next != h->stream) {
    // work queued on the new stream starts after everything queued so far
    hipEvent_t ev;
    hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(h, e, "sbim_set_stream: hipEventCreate");
    e = hipEventRecord(ev, h->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(next, ev, 0);
    (void)hipEventDestroy(ev);
    if (e != hipSuccess) return hip_fail(h, e, "sbim_set_stream: ordering after the old stream");
  }
  h->stream = next;
  h->cfg.stream = stream;
  return SBIM_OK;
}

int sbim_set_dt(sbim_handle *h, double dt) {
  if (!h) return fail(nullptr, SBIM_E_INVALID, "handle is NULL");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(h, SBIM_E_INVALID, "dt must be finite and > 0");
  if (h->cfg.window_mode != SBIM_W_STATIC)
    return fail(h, SBIM_E_STATE, "the time step of a dynamic handle is fixed at sbim_init");
  h->cfg.dt = dt;
  return SBIM_OK;
}

}  // extern "C"
