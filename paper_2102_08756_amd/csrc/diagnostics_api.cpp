// C ABI, diagnostics beside the step: non-finite counts, the traction
// spectrum, handle information, snapshots (full and running state), work
// accounting of a step, per-mode kernel rows and step-launch timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "api_internal.h"
#include "checks.h"

using sbim::Group;
using namespace sbim_api;

extern "C" {

int sbim_count_nonfinite(sbim_handle *h, const void *field, long long *count) {
  if (!h) return fail(nullptr, SBIM_E_INVALID, "handle is NULL");
  if (!field || !count) return fail(h, SBIM_E_INVALID, "field or count is NULL");
  const long long n = static_cast<long long>(h->cfg.nplanes) * 3 * h->n1 * h->n3;
  long long *partial = nullptr;
  hipError_t e = hipMalloc(&partial, sizeof(long long) * sbim::kCheckBlocks);
  if (e != hipSuccess) return fail(h, SBIM_E_OOM, "count buffer: %s", hipGetErrorString(e));
  std::vector<long long> part(sbim::kCheckBlocks, 0);
  e = sbim::launch_count_nonfinite(h->fp64, field, n, partial, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(part.data(), partial, sizeof(long long) * part.size(),
                       hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  (void)hipFree(partial);
  if (e != hipSuccess) return hip_fail(h, e, "non-finite count");
  long long c = 0;
  for (long long v : part) c += v;
  *count = c;
  return SBIM_OK;
}

int sbim_count_nonfinite_noalloc(sbim_handle *h, const void *field, long long *count_dev) {
  if (!h) return fail(nullptr, SBIM_E_INVALID, "handle is NULL");
  if (!field || !count_dev) return fail(h, SBIM_E_INVALID, "field or count_dev is NULL");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(h, e, "hipGetDevice");
  if (dev != h->device)
    return fail(h, SBIM_E_STATE, "current device %d is not the handle's device %d", dev, h->device);
  const long long n = static_cast<long long>(h->cfg.nplanes) * 3 * h->n1 * h->n3;
  e = sbim::launch_count_nonfinite_static(h->fp64, field, n, h->count_scratch, count_dev,
                                          h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "non-finite count (static scratch)");
  return SBIM_OK;
}

int sbim_traction_spectrum(sbim_handle *h, void *dst) {
  if (!h) return fail(nullptr, SBIM_E_INVALID, "handle is NULL");
  int rc = check_ptr(h, dst, "dst");
  if (rc) return rc;
  if (h->step == 0) return fail(h, SBIM_E_STATE, "sbim_traction_spectrum before any push");
  const hipError_t e =
      hipMemcpyAsync(dst, h->out_spec, out_spec_bytes(h), hipMemcpyDeviceToDevice, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "sbim_traction_spectrum");
  return SBIM_OK;
}

int sbim_get_info(const sbim_handle *h, sbim_info *out) {
  if (!h || !out) return fail(nullptr, SBIM_E_INVALID, "handle or out is NULL");
  std::memset(out, 0, sizeof *out);
  out->modes_per_plane = h->nh;
  for (int i = 0; i < h->ngroups; ++i) {
    const Group &g = h->g[i];
    out->kernel_classes += g.nclasses;
    out->ring_bytes += ring_bytes(h, g);
    out->table_bytes += table_bytes(h, g);
    out->state_bytes += state_bytes_g(g);
  }
  out->step = h->step;
  out->backward_step = h->bstep;
  out->material_groups = h->ngroups;
  out->sweep_depth = h->depth;
  out->sweep_matrix_cores = h->mfma ? 1 : 0;
  out->sweep_lag_chunks = h->mfma ? h->lag_chunks : 0;
  out->sweep_quads = h->mfma ? h->sweep_quads : 0;
  return SBIM_OK;
}

long long sbim_state_bytes(const sbim_handle *h) {
  if (!h) return -1;
  long long b = 256 + out_spec_bytes(h);  // header (step counter), last traction spectrum
  for (int i = 0; i < h->ngroups; ++i) {
    const Group &g = h->g[i];
    b += ring_bytes(h, g) + state_bytes_g(g) + pending_bytes(h, g);
  }
  return b;
}

int sbim_save_state(sbim_handle *h, void *dst) {
  if (!h) return fail(nullptr, SBIM_E_INVALID, "handle is NULL");
  int rc = check_ptr(h, dst, "dst");
  if (rc) return rc;
  char *d = static_cast<char *>(dst);
  hipError_t e = hipMemcpyAsync(d, &h->step, sizeof(long long), hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);  // &h->step may change after return
  d += 256;
  if (e == hipSuccess)
    e = hipMemcpyAsync(d, h->out_spec, out_spec_bytes(h), hipMemcpyDeviceToDevice, h->stream);
  d += out_spec_bytes(h);
  for (int i = 0; i < h->ngroups && e == hipSuccess; ++i) {
    Group &g = h->g[i];
    const size_t rb = ring_bytes(h, g), sb = state_bytes_g(g);
    if (rb) e = hipMemcpyAsync(d, g.ring, rb, hipMemcpyDeviceToDevice, h->stream);
    d += rb;
    if (e == hipSuccess) e = hipMemcpyAsync(d, g.state, sb, hipMemcpyDeviceToDevice, h->stream);
    d += sb;
    const size_t pb = pending_bytes(h, g);
    if (e == hipSuccess) e = hipMemcpyAsync(d, g.pending, pb, hipMemcpyDeviceToDevice, h->stream);
    d += pb;
  }
  if (e != hipSuccess) return hip_fail(h, e, "sbim_save_state");
  return SBIM_OK;
}

int sbim_load_state(sbim_handle *h, const void *src) {
  if (!h) return fail(nullptr, SBIM_E_INVALID, "handle is NULL");
  int rc = check_ptr(h, src, "src");
  if (rc) return rc;
  const char *s = static_cast<const char *>(src);
  long long step = 0;
  hipError_t e = hipMemcpyAsync(&step, s, sizeof(long long), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "sbim_load_state header");
  if (step < 0) return fail(h, SBIM_E_INVALID, "snapshot header is corrupt");
  s += 256;
  e = hipMemcpyAsync(h->out_spec, s, out_spec_bytes(h), hipMemcpyDeviceToDevice, h->stream);
  s += out_spec_bytes(h);
  for (int i = 0; i < h->ngroups && e == hipSuccess; ++i) {
    Group &g = h->g[i];
    const size_t rb = ring_bytes(h, g), sb = state_bytes_g(g);
    if (rb) e = hipMemcpyAsync(g.ring, s, rb, hipMemcpyDeviceToDevice, h->stream);
    s += rb;
    if (e == hipSuccess) e = hipMemcpyAsync(g.state, s, sb, hipMemcpyDeviceToDevice, h->stream);
    s += sb;
    const size_t pb = pending_bytes(h, g);
    if (e == hipSuccess) e = hipMemcpyAsync(g.pending, s, pb, hipMemcpyDeviceToDevice, h->stream);
    s += pb;
  }
  if (e != hipSuccess) return hip_fail(h, e, "sbim_load_state");
  h->step = step;
  return SBIM_OK;
}

long long sbim_running_state_bytes(const sbim_handle *h) {
  if (!h) return -1;
  long long b = 256;  // header (step counter)
  for (int i = 0; i < h->ngroups; ++i) b += state_bytes_g(h->g[i]);
  return b;
}

int sbim_save_running_state(sbim_handle *h, void *dst) {
  if (!h) return fail(nullptr, SBIM_E_INVALID, "handle is NULL");
  int rc = check_ptr(h, dst, "dst");
  if (rc) return rc;
  char *d = static_cast<char *>(dst);
  hipError_t e = hipMemcpyAsync(d, &h->step, sizeof(long long), hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);  // &h->step may change after return
  d += 256;
  for (int i = 0; i < h->ngroups && e == hipSuccess; ++i) {
    const Group &g = h->g[i];
    e = hipMemcpyAsync(d, g.state, state_bytes_g(g), hipMemcpyDeviceToDevice, h->stream);
    d += state_bytes_g(g);
  }
  if (e != hipSuccess) return hip_fail(h, e, "sbim_save_running_state");
  return SBIM_OK;
}

int sbim_load_running_state(sbim_handle *h, const void *src) {
  if (!h) return fail(nullptr, SBIM_E_INVALID, "handle is NULL");
  int rc = check_ptr(h, src, "src");
  if (rc) return rc;
  const char *s = static_cast<const char *>(src);
  long long step = 0;
  hipError_t e = hipMemcpyAsync(&step, s, sizeof(long long), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "sbim_load_running_state header");
  if (step < 0) return fail(h, SBIM_E_INVALID, "running-state snapshot header is corrupt");
  s += 256;
  for (int i = 0; i < h->ngroups && e == hipSuccess; ++i) {
    Group &g = h->g[i];
    e = hipMemcpyAsync(g.state, s, state_bytes_g(g), hipMemcpyDeviceToDevice, h->stream);
    s += state_bytes_g(g);
    // the history before the snapshot is gone: start from an empty ring and no pending sums
    const size_t rb = static_cast<size_t>(ring_bytes(h, g));
    if (e == hipSuccess && rb) e = hipMemsetAsync(g.ring, 0, rb, h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(g.pending, 0, pending_bytes(h, g), h->stream);
  }
  if (e != hipSuccess) return hip_fail(h, e, "sbim_load_running_state");
  h->step = step;
  return SBIM_OK;
}

int sbim_step_work(const sbim_handle *h, long long n, double *mode_lags, double *conv_bytes) {
  if (!h || !mode_lags || !conv_bytes || n < 0)
    return fail(nullptr, SBIM_E_INVALID, "bad arguments to sbim_step_work");
  const double r = static_cast<double>(h->rsize);
  const int S = h->depth;
  double lags = 0, bytes = 0;
  for (int i = 0; i < h->ngroups; ++i) {
    const Group &g = h->g[i];
    double mode_lag_g = 0;
    for (long long s = 0; s < g.M; ++s)
      mode_lag_g += static_cast<double>(std::min<long long>(g.h_win[s], n + 1));
    lags += mode_lag_g * g.np;
    // the sweep launched with step n (for steps n+1 .. n+S): blocks of phase
    // (n+1) mod S read the history up to step n-1 that each of their modes
    // needs (lags 2 .. W-1 of step n+1), the kernel rows of each distinct class
    // of the block (lags 2 .. min(cap-1, n+1) + S - 1), the per-mode
    // class/window indices and block descriptors, and write S pending sums per
    // mode and plane
    for (long long b = (n + 1) % S; b < g.nblocks; b += S) {
      const long long last = std::min<long long>(g.h_blk_cap[b] - 1, n + 1);
      int last_cls = -1;
      for (long long s = b * sbim::kLanes; s < std::min(g.M, (b + 1) * sbim::kLanes); ++s) {
        if (g.h_nat[s] < 0) continue;  // padding position of the matrix-core layout
        const int w = g.h_win[s];
        bytes += std::max(0LL, std::min<long long>(w - 1, n + 1) - 1) * g.np * 3.0 * 2.0 * r;
        bytes += 8.0 + S * g.np * 10.0 * r;
        if (w > 2 && g.h_cls[s] != last_cls) {
          last_cls = g.h_cls[s];
          bytes += std::max(0LL, std::min<long long>(w - 1, last + S - 1) - 1) * 4.0 * r;
        }
      }
      bytes += 16.0;
    }
    // the mode items of step n (same launch), per mode and plane: the three
    // float64 spectrum values, the float64 state read and written, the ring
    // slot written, the pending sum read, the newest lags (history from the
    // ring beyond lag 0, kernel rows), the traction written; per mode its bin,
    // q and direction, window, class and row offset; per block its descriptors
    for (long long s = 0; s < g.M; ++s) {
      if (g.h_nat[s] < 0) continue;
      const long long b = s / sbim::kLanes;
      const int phi = static_cast<int>(b % S);
      const bool swept = n >= (phi == 0 ? S : phi);
      const long long fresh = std::min<long long>(g.h_win[s], swept ? (n - phi) % S + 2 : n + 1);
      double per_plane = 3.0 * 16.0 + 3.0 * 32.0 + 3.0 * 2.0 * r + 3.0 * 2.0 * r;
      if (swept) per_plane += 10.0 * r;
      per_plane += std::max(0LL, fresh - 1) * 3.0 * 2.0 * r + fresh * 4.0 * r;
      bytes += per_plane * g.np + 4.0 + 24.0 + 4.0 + 4.0 + (fresh > 0 ? 8.0 : 0.0);
    }
    bytes += g.nblocks * 16.0;
  }
  *mode_lags = lags;
  *conv_bytes = bytes;
  return SBIM_OK;
}

int sbim_mode_kernel(sbim_handle *h, int p, int i1, int i3, double *host_out, int max_lags) {
  if (!h) return fail(nullptr, SBIM_E_INVALID, "handle is NULL");
  if (p < 0 || p >= h->cfg.nplanes || i1 < 0 || i1 >= h->n1 || i3 < 0 || i3 >= h->h3 ||
      max_lags < 0 || (max_lags > 0 && !host_out))
    return fail(h, SBIM_E_INVALID, "bad arguments to sbim_mode_kernel");
  const Group *gp = nullptr;
  for (int i = 0; i < h->ngroups; ++i)
    for (int k = 0; k < h->g[i].np; ++k)
      if (h->g[i].pl[k].index == p) gp = &h->g[i];
  const Group &g = *gp;
  const int f = i3 * h->n1 + i1;
  long long s = -1;
  for (long long t = 0; t < g.M; ++t)
    if (g.h_nat[t] == f) s = t;
  const int w = g.h_win[s];
  if (w == 0) return 0;
  const int c = g.h_cls[s];
  hipError_t e = hipStreamSynchronize(h->stream);
  const int nl = std::min(w, max_lags);
  std::vector<char> tmp(4 * h->rsize);
  for (int j = 0; j < nl && e == hipSuccess; ++j) {
    const char *src = static_cast<const char *>(g.table) + (g.h_cls_off[c] + j) * 4 * h->rsize;
    e = hipMemcpy(tmp.data(), src, 4 * h->rsize, hipMemcpyDeviceToHost);
    for (int k = 0; k < 4; ++k) {
      double v;
      if (h->fp64)
        std::memcpy(&v, tmp.data() + 8 * k, 8);
      else {
        float fv;
        std::memcpy(&fv, tmp.data() + 4 * k, 4);
        v = fv;
      }
      host_out[static_cast<long long>(k) * max_lags + j] = v;
    }
  }
  if (e != hipSuccess) return hip_fail(h, e, "sbim_mode_kernel copy");
  return w;
}

int sbim_profile_conv(sbim_handle *h, int every) {
  if (!h) return fail(nullptr, SBIM_E_INVALID, "handle is NULL");
  if (every < 0) return fail(h, SBIM_E_INVALID, "sbim_profile_conv: every must be >= 0");
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "sbim_profile_conv sync");
  h->ev_used = 0;
  h->profile_every = every;
  h->profile_seen = 0;
  return SBIM_OK;
}

int sbim_conv_timing(sbim_handle *h, double *total_ms, long long *launches) {
  if (!h || !total_ms || !launches) return fail(nullptr, SBIM_E_INVALID, "bad arguments");
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "sbim_conv_timing sync");
  double tot = 0;
  for (size_t i = 0; i < h->ev_used; ++i) {
    float ms = 0;
    e = hipEventElapsedTime(&ms, h->ev_start[i], h->ev_stop[i]);
    if (e != hipSuccess) return hip_fail(h, e, "hipEventElapsedTime");
    tot += ms;
  }
  *total_ms = tot;
  *launches = static_cast<long long>(h->ev_used);
  return SBIM_OK;
}

}  // extern "C"
