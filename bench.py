"""Benchmark of the boundary-integral (SBIM) traction update on one MI355X.

Workload (default): two boundary planes of 512 x 512, three displacement
components, mu = 1, c_s = 1, c_p = sqrt(3), dx = 1, dt = 0.2, history window
1000 steps, a 2000-step job; inputs are the seeded |k|^-2 increment fields
(bank of 64 per plane and component) plus a Gaussian ramp pulse of width 20
cells on u1.  A "step" is one push of the displacement plus one traction
evaluation (forward FFT, history update, convolution, inverse FFT).

The timed region is the steady state of the job: the steps run from an empty
history, the first ones untimed until the window is full and only the last
``--steps`` of the job are left (every timed step then sums its whole
1000-lag window), and those are timed with the inputs resident in HBM.
Reported: mode-history-steps per second (sum over the timed steps, planes and
modes of min(W, n+1)) for the compensated float32 form (headline), plain
float32 and float64; the float32-vs-float64 relative L2 error over the whole
2000-step job; the HBM roofline fraction of the dominant kernel (the launch
that pushes a step, completes its traction spectrum and runs the history
sweep) over the same timed steps; and the float64 CPU oracle on a bounded
sample.  Further legs time the stand-alone dynamic rupture of the paper's
TPV3 setup (1024 x 1024 cells of 50 m, 2000 steps) through the fault entry
points, the hybrid strip and the quasi-dynamic limit on it, and the adjoint
on the 256^2 job.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SBIM mode·history-steps/s + % HBM peak; FP32 vs FP64 at 1e-5 rel L2"
UNIT = "mode·history-steps/s"
HBM_PEAK_GBS = 8000.0
MFMA_F32_PEAK_TFLOPS = 157.3     # dense float32 matrix-core peak of the MI355X
# the step launch of every 7th timed step carries events (7 is prime to every sweep depth,
# so the timed launches meet each phase of the sweep)
TIMING_EVERY = 7
PROFILES = os.path.join(ROOT, "profiles")


def kernel_source_hash():
    """Hash of the step kernel's sources and of the host code that picks its launch shape,
    with comments and blank lines stripped (a comment edit does not invalidate recorded
    counters; any code change does)."""
    import re
    h = hashlib.sha256()
    for f in ("kernels.hip", "internal.h", "sbim_api.cpp"):
        with open(os.path.join(ROOT, "paper_2102_08756_amd", "csrc", f)) as fh:
            for line in fh:
                code = re.sub(r"//.*", "", line).rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def read_traffic(workload, precision, regime="steady"):
    """Per-dispatch HBM bytes of the step launch (push, traction, history sweep) in the
    given regime from the committed rocprofv3 counter summary, scaled by the copy-kernel
    calibration; None if absent or taken on other kernel sources."""
    path = os.path.join(PROFILES, "step_kernel_traffic.txt")
    if not os.path.exists(path):
        return None
    want = f"{workload} {precision} {regime} "
    src = None
    val = None
    for line in open(path):
        if line.startswith("kernel_source_hash"):
            src = line.split("=", 1)[1].strip()
        if line.startswith(want):
            val = float(line.split()[3])
    if src != kernel_source_hash() or val is None:
        return None
    return val


def host_cpu():
    """Cores this process may run on, the machine's logical CPU count and the CPU model."""
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    model = None
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    if model is None:
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
    return {"nproc": usable, "logical_cpus": os.cpu_count(), "model": model}


class Inputs:
    """Per-step increments resident in HBM: each distinct field of the workload
    (bank entries and the pulse-ramp steps) uploaded once.  A workload with a
    uniform slip ramp adds its uniform part with one device add per step."""

    def __init__(self, wl, dtype, device):
        import torch
        import workloads
        fields, self.index, self.uniform = workloads.step_sources(wl)
        self.fields = [torch.tensor(f, dtype=dtype, device=device) for f in fields]
        self.has_uniform = bool(wl.slip_ramp)
        self.scratch = torch.empty_like(self.fields[0]) if self.has_uniform else None
        self.dtype, self.device = dtype, device

    def __call__(self, n):
        f = self.fields[self.index(n)]
        if not self.has_uniform:
            return f
        import torch
        u = torch.tensor(self.uniform(n), dtype=self.dtype, device=self.device)
        torch.add(f, u[:, :, None, None], out=self.scratch)
        return self.scratch


def run_job(sb, inputs, steps, tau):
    for n in steps:
        sb.push(inputs(n))
        sb.tractions(out=tau)


def steady_window(wl, timed):
    """First timed step of the steady state: the last ``timed`` steps of the job, but never
    before every mode's window is full (step W_cap - 1 on); a request for more steps than the
    job has at a full window runs past its end (each step then costs the same)."""
    return max(wl.steps - timed, wl.window_cap - 1, 0)


def default_timed_steps(wl):
    return max(1, wl.steps - wl.window_cap)


def bracketed_steps(n0, steps, every):
    """The timed steps whose step launch sbim_profile_conv(h, every) brackets with events:
    the first after the call and every ``every``-th after it."""
    return range(n0, n0 + steps, every)


def measure_form(wl, precision, steps, warmup, device, inputs_cache):
    """Time ``steps`` steps of the job at a full history window: ``warmup`` steps and a
    reset, the job's first steps untimed (the window fills), then the timed ones."""
    import torch
    from paper_2102_08756_amd import SBIM, Config
    cfg = Config.from_dict(wl.config_dict(), precision=precision)
    t0 = time.time()
    sb = SBIM(cfg, device=device)
    t_init = time.time() - t0
    key = cfg.dtype
    if key not in inputs_cache:
        inputs_cache[key] = Inputs(wl, cfg.dtype, device)
    inputs = inputs_cache[key]
    tau = sb.new_field()
    n0 = steady_window(wl, steps)
    # The step launch of every TIMING_EVERY-th timed step is bracketed by HIP events (each
    # pair of event records costs a few microseconds of the step it brackets); with more
    # than one material group per handle the launches of a step alternate, so every launch
    # is timed then.
    every = TIMING_EVERY if sb.info()["material_groups"] == 1 else 1
    # warmup, then the job from an empty history; the launches are bracketed by events
    # from here on, so the event pool has grown before the timed steps
    sb.profile_conv(True, every)
    run_job(sb, inputs, range(warmup), tau)
    sb.reset()
    run_job(sb, inputs, range(n0), tau)
    sb.profile_conv(True, every)       # synchronises and restarts the launch timing
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run_job(sb, inputs, range(n0, n0 + steps), tau)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    conv_ms, launches = sb.conv_timing()
    sb.profile_conv(False)
    lags = 0.0
    conv_lags = conv_bytes = 0.0   # mode-lags and algorithmic bytes of the bracketed launches
    bracketed = set(bracketed_steps(n0, steps, every))
    for n in range(n0, n0 + steps):
        a, b = sb.step_work(n)
        lags += a
        if n in bracketed:
            conv_lags += a
            conv_bytes += b
    info = sb.info()
    sb.close()
    del sb
    torch.cuda.empty_cache()
    gbs = conv_bytes / (conv_ms * 1e-3) / 1e9
    traffic = read_traffic(wl.name, precision)
    r = 8 if precision == "fp64" else 4
    P = len(wl.planes)
    shared = 1 if P == 1 or any(p != wl.planes[0] for p in wl.planes[1:]) else P
    # bytes a direct (per-step) convolution streams for the same work: the whole window of
    # history (3 complex per plane, mode and lag) and the kernel rows (4 reals per mode and
    # lag, read once for the planes that share them)
    direct_bytes = conv_lags * (6 * r + 4 * r / shared)
    return {
        "value": lags / elapsed,
        "ms_per_step": 1e3 * elapsed / steps,
        "elapsed_s": elapsed,
        "init_s": t_init,
        "mode_lags": lags,
        "first_timed_step": n0,
        "roofline": {
            "kernel": (f"step_kernel{'_mfma' if info['sweep_matrix_cores'] else ''} (push, traction "
                       f"and history sweep, depth {info['sweep_depth']}"
                       f"{', matrix cores' if info['sweep_matrix_cores'] else ''})"),
            "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS,
            "traffic": traffic,
            "regime": (f"steady state: steps {n0}..{n0 + steps - 1} of the job, every mode's "
                       f"window full; achieved over the step launches of every {every}-th of "
                       f"these steps (HIP events), traffic over all of their launches"),
            "algorithmic_bytes_per_launch": conv_bytes / launches if launches else None,
            "traffic_over_algorithmic": (traffic * launches / conv_bytes
                                         if traffic and launches else None),
            "avg_launch_ms": conv_ms / launches if launches else None,
            "launches": launches,
            "matrix_cores": {
                "achieved": 20.0 * conv_lags / (conv_ms * 1e-3) / 1e12,
                "peak": MFMA_F32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": 20.0 * conv_lags / (conv_ms * 1e-3) / 1e12 / MFMA_F32_PEAK_TFLOPS,
                "note": ("the history products, 20 flop (10 FMAs) per plane, mode and lag, in the "
                         "step launch time: on the matrix cores (16x16x4 float32) when "
                         "sweep_matrix_cores is 1, the newest lags of each step on the vector units"),
            } if info["sweep_matrix_cores"] else None,
            "direct_convolution_equivalent": {
                "GBs": direct_bytes / (conv_ms * 1e-3) / 1e9,
                "x_hbm_peak": direct_bytes / (conv_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                "note": (f"the history and kernel-row bytes a per-step convolution would stream "
                         f"for the same work in the same launch time; the sweep reads each "
                         f"history entry once per {info['sweep_depth']} steps, so it is not a "
                         f"fraction of the HBM peak"),
            },
        },
        "info": info,
    }


def accuracy(wl, steps, device, inputs_cache, forms=("fp32_comp", "fp32"), block=500):
    """Relative L2 of float32 forms against float64 on the same inputs: whole job, worst
    single step, and per block of ``block`` steps (to show how the error grows with time)."""
    import torch
    from paper_2102_08756_amd import SBIM, Config
    ref = SBIM(Config.from_dict(wl.config_dict(), precision="fp64"), device=device)
    others = {f: SBIM(Config.from_dict(wl.config_dict(), precision=f), device=device) for f in forms}
    in64 = inputs_cache[torch.float64]
    in32 = inputs_cache[torch.float32]
    zero = lambda: torch.zeros((), dtype=torch.float64, device=device)  # noqa: E731
    num = {f: zero() for f in forms}
    bnum = {f: zero() for f in forms}
    worst = {f: zero() for f in forms}
    den, bden = zero(), zero()
    blocks = {f: [] for f in forms}
    t64 = ref.new_field()
    t32 = {f: others[f].new_field() for f in forms}
    for n in range(steps):
        ref.push(in64(n))
        ref.tractions(out=t64)
        d = (t64 * t64).sum()
        den += d
        bden += d
        for f in forms:
            others[f].push(in32(n))
            others[f].tractions(out=t32[f])
            e = ((t32[f].double() - t64) ** 2).sum()
            num[f] += e
            bnum[f] += e
            worst[f] = torch.maximum(worst[f], torch.sqrt(e / d))
        if (n + 1) % block == 0 or n + 1 == steps:
            for f in forms:
                blocks[f].append(float(torch.sqrt(bnum[f] / bden)))
                bnum[f].zero_()
            bden.zero_()
            print(f"[bench] accuracy: step {n + 1}/{steps}: "
                  + ", ".join(f"{f} {blocks[f][-1]:.3e}" for f in forms), file=sys.stderr, flush=True)
    out = {"block_steps": block}
    for f in forms:
        out[f"{f}_vs_fp64_rel_l2"] = float(torch.sqrt(num[f] / den))
        out[f"{f}_vs_fp64_worst_step_rel_l2"] = float(worst[f])
        out[f"{f}_vs_fp64_rel_l2_per_block"] = blocks[f]
    ref.close()
    for s in others.values():
        s.close()
    return out


def measure_rupture(fw, precision, device, warmup=20, window_mode=None):
    """Stand-alone rupture on the fault between two half-spaces (the paper's TPV3 setup
    at its resolution; the lower half-space is the mirror image of the upper one): the
    whole run timed from rest, one library step (push without damping, inverse FFT,
    interface solve) per time step."""
    import torch
    from paper_2102_08756_amd import SBIM, Config, Fault
    cd = fw.config_dict()
    if window_mode:
        cd["window_mode"] = window_mode
    cfg = Config.from_dict(cd, precision=precision, input_kind="increment")
    t0 = time.time()
    sb = SBIM(cfg, device=device)
    prm = [torch.tensor(a, dtype=torch.float64, device=device).contiguous() for a in fw.params()]
    flt = Fault(sb, *prm)
    t_init = time.time() - t0
    sb.profile_conv(True)
    for _ in range(warmup):
        flt.step()
    flt.reset()
    sb.profile_conv(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(fw.steps):
        flt.step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    conv_ms, launches = sb.conv_timing()
    sb.profile_conv(False)
    lags = conv_bytes = 0.0
    for n in range(fw.steps):
        a, b = sb.step_work(n)
        lags += a
        conv_bytes += b
    slip = flt.read("slip").cpu().numpy()
    amp = np.hypot(slip[0], slip[1])
    info = sb.info()
    flt.close()
    sb.close()
    del sb, flt, prm
    torch.cuda.empty_cache()
    _, region = fw.masks()
    gbs = conv_bytes / (conv_ms * 1e-3) / 1e9
    return {
        "ms_per_step": 1e3 * elapsed / fw.steps, "mode_lags_per_s": lags / elapsed,
        "step_kernel_GBs": gbs, "step_kernel_frac": gbs / HBM_PEAK_GBS,
        "sweep_depth": info["sweep_depth"], "init_s": t_init, "ring_bytes": info["ring_bytes"],
        "region_slipped_frac": float((amp[region] > 0).mean()),
        "outside_slipped_cells": int((amp[~region] > 0).sum()),
        "max_slip_m": float(np.abs(slip).max()), "_slip": slip,
    }


def measure_hybrid(fw, precision, device, layers=2, warmup=20):
    """The hybrid scheme on the same setup: a strip of ``layers`` element layers of the
    bulk material between the fault and S+ (two layers = the paper's strip width 4 dx
    for the symmetric half), the whole run timed from rest.  A workload with its own
    lower half-space gets the two-sided strip: ``layers`` element layers of the lower
    material between the fault and S- as well."""
    import torch
    import workloads
    from paper_2102_08756_amd import SBIM, Config, Strip
    t = workloads.TPV3
    cfg = Config.from_dict(fw.config_dict(), precision=precision, input_kind="increment")
    t0 = time.time()
    sb = SBIM(cfg, device=device)
    prm = [torch.tensor(a, dtype=torch.float64, device=device).contiguous() for a in fw.params()]
    below = None
    if fw.lower is not None:
        lo = fw.lower
        below = [(lo["mu"] / lo["cs"] ** 2, lo["cp"], lo["cs"])] * layers
    st = Strip(sb, [(t["rho"], t["cp"], t["cs"])] * layers, *prm, layers_below=below)
    t_init = time.time() - t0
    for _ in range(warmup):
        st.step()
    st.reset()
    sb.profile_conv(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(fw.steps):
        st.step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    conv_ms, launches = sb.conv_timing()
    sb.profile_conv(False)
    slip = st.read("slip").cpu().numpy()
    st.close()
    sb.close()
    del sb, st, prm
    torch.cuda.empty_cache()
    nodes = (layers + 1) * (1 if below is None else 2) * fw.n1 * fw.n3
    return {"layers": layers, "two_sided": below is not None, "ms_per_step": 1e3 * elapsed / fw.steps,
            "node_steps_per_s": nodes * fw.steps / elapsed,
            "step_kernel_ms_per_step": conv_ms / launches if launches else None,
            "init_s": t_init, "_slip": slip}


def rupture_leg(fw, forms, device, bimaterial=False):
    out = {"workload": fw.name, "n1": fw.n1, "n3": fw.n3, "dx_m": fw.dx, "dt_s": fw.dt,
           "time_steps": fw.steps, "window_cap": fw.window_cap or fw.steps,
           "lower_half_space": "mirror image" if fw.lower is None else "own material", "forms": {}}
    slips = {}
    for p in forms:
        r = measure_rupture(fw, p, device)
        slips[p] = r.pop("_slip")
        out["forms"][p] = r
        print(f"[bench] rupture {fw.name} {p}: {r['ms_per_step']:.3f} ms/step, "
              f"{r['mode_lags_per_s']:.3e} mode-lags/s, step kernel {r['step_kernel_GBs']:.0f} GB/s; "
              f"region slipped {100 * r['region_slipped_frac']:.1f}%, max slip {r['max_slip_m']:.3f} m",
              file=sys.stderr, flush=True)
    if "fp64" in slips:
        for p in slips:
            if p != "fp64":
                out[f"{p}_vs_fp64_final_slip_rel_l2"] = float(
                    np.linalg.norm(slips[p] - slips["fp64"]) / np.linalg.norm(slips["fp64"]))
    # hybrid: finite-element strip on the fault, closed by the boundary relation at S+
    p = forms[0]
    hy = measure_hybrid(fw, p, device)
    hs = hy.pop("_slip")
    hy["precision"] = p
    hy["final_slip_rel_l2_vs_boundary_integral"] = float(
        np.linalg.norm(hs - slips[p]) / np.linalg.norm(slips[p]))
    out["hybrid"] = hy
    # quasi-dynamic limit of the same rupture (static kernel plus radiation damping)
    qd = measure_rupture(fw, p, device, window_mode="static")
    qd.pop("_slip")
    out["quasi_dynamic"] = {k: qd[k] for k in ("ms_per_step", "init_s", "ring_bytes",
                                               "region_slipped_frac", "max_slip_m")}
    out["quasi_dynamic"]["precision"] = p
    print(f"[bench] quasi-dynamic {fw.name} {p}: {qd['ms_per_step']:.3f} ms/step, "
          f"max slip {qd['max_slip_m']:.3f} m", file=sys.stderr, flush=True)
    print(f"[bench] hybrid {fw.name} {p}: {hy['ms_per_step']:.3f} ms/step "
          f"({hy['layers']} element layers), final slip vs boundary integral "
          f"{hy['final_slip_rel_l2_vs_boundary_integral']:.2e}", file=sys.stderr, flush=True)
    if bimaterial and fw.lower is None:
        # the same rupture between two materials (the lower one slower): the stand-alone
        # two-plane rupture and the two-sided strip, two element layers on each side
        import dataclasses
        import workloads
        bf = dataclasses.replace(fw, name=f"{fw.name}_bimaterial", lower=workloads.SLOWER)
        br = measure_rupture(bf, p, device)
        br.pop("_slip")
        bh = measure_hybrid(bf, p, device)
        bhs = bh.pop("_slip")
        out["bimaterial"] = {
            "workload": bf.name, "lower_half_space": "0.64 mu, 0.8 c_s, 0.8 c_p of the upper",
            "precision": p, "boundary_integral": {k: br[k] for k in (
                "ms_per_step", "init_s", "region_slipped_frac", "max_slip_m")},
            "hybrid_two_sided": dict(bh, max_slip_m=float(np.abs(bhs).max()))}
        print(f"[bench] bimaterial {bf.name} {p}: boundary integral {br['ms_per_step']:.3f} ms/step, "
              f"two-sided hybrid {bh['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    return out


def adjoint_leg(device, forms, every=50, receivers=64, seed=4000):
    """Differentiation on the 256^2 single-plane job (W = 300, 500 steps): the gradient of
    a receiver misfit L = sum_n sum_r sum_i tau_i^n(x_r)^2 (64 receiver cells) with respect
    to the whole displacement history, through SBIMRun (the forward keeps every traction;
    the backward runs the library's transpose in reverse time) and through
    checkpointed_loss (snapshots every ``every`` steps, tractions recomputed per segment in
    the backward).  Each pass is timed whole, from a synchronised device, after one
    untimed pass of each kind; the two gradients are compared."""
    import torch
    import workloads
    from paper_2102_08756_amd import SBIM, Config, SBIMRun, checkpointed_loss
    wl = workloads.WORKLOADS[4]
    out = {"workload": wl.name, "n1": wl.n1, "n3": wl.n3, "window_cap": wl.window_cap,
           "time_steps": wl.steps, "receivers": receivers, "checkpoint_every": every,
           "forms": {}}
    rec = torch.randperm(wl.n1 * wl.n3, generator=torch.Generator().manual_seed(seed))[:receivers]
    for f in forms:
        sb = SBIM(Config.from_dict(wl.config_dict(), precision=f), device=device)
        gen = torch.Generator(device=device).manual_seed(seed + 1)
        u = torch.randn((wl.steps,) + sb.shape, generator=gen, dtype=sb.dtype, device=device)
        r = rec.to(device)
        P = sb.shape[0]

        def full():
            x = u.clone().requires_grad_(True)
            t0 = time.perf_counter()
            tau = SBIMRun.apply(sb, x)
            L = (tau.reshape(wl.steps, P, 3, -1)[..., r] ** 2).sum()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            L.backward()
            torch.cuda.synchronize()
            return x.grad, t1 - t0, time.perf_counter() - t1

        def ckpt():
            x = u.clone().requires_grad_(True)
            t0 = time.perf_counter()
            L = checkpointed_loss(sb, x, lambda tau, n: (tau.reshape(P, 3, -1)[..., r] ** 2).sum(),
                                  every=every)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            L.backward()
            torch.cuda.synchronize()
            return x.grad, t1 - t0, time.perf_counter() - t1

        full()
        ckpt()
        torch.cuda.synchronize()
        g1, f1, b1 = full()
        g2, f2, b2 = ckpt()
        N = wl.steps
        out["forms"][f] = {
            "forward_ms_per_step": 1e3 * f1 / N, "backward_ms_per_step": 1e3 * b1 / N,
            "checkpointed_forward_ms_per_step": 1e3 * f2 / N,
            "checkpointed_backward_ms_per_step": 1e3 * b2 / N,
            "gradient_rel_l2_full_vs_checkpointed": float(
                (g1 - g2).double().norm() / g1.double().norm()),
        }
        o = out["forms"][f]
        print(f"[bench] adjoint {wl.name} {f}: forward {o['forward_ms_per_step']:.3f} ms/step, "
              f"backward {o['backward_ms_per_step']:.3f} ms/step; checkpointed "
              f"{o['checkpointed_forward_ms_per_step']:.3f} + {o['checkpointed_backward_ms_per_step']:.3f}"
              f" ms/step; gradients agree to {o['gradient_rel_l2_full_vs_checkpointed']:.1e}",
              file=sys.stderr, flush=True)
        del u, g1, g2
        sb.close()
        torch.cuda.empty_cache()
    return out


def scaling_sweep(device, sizes=(128, 256, 512, 1024, 2048), window=200, layers=(2, 6)):
    """Cost of one step against the grid size n x n at a fixed history window: the
    boundary relation with the fault's interface solve, and the hybrid scheme with
    two and six element layers (their difference / 4 is the cost of one node layer of
    the strip).  Steady state: the window is full when the timed steps start."""
    import torch
    import workloads
    from paper_2102_08756_amd import SBIM, Config, Fault, Strip
    t = workloads.TPV3
    rows = []
    for n in sizes:
        fw = workloads.FaultWorkload(f"scaling{n}", n, n, 50.0 * 1024 / n, 2 * window,
                                     window_cap=window)
        prm = [torch.tensor(a, dtype=torch.float64, device=device).contiguous() for a in fw.params()]
        row = {"n": n, "modes": n * (n // 2 + 1), "window": window}

        def timed(make):
            sb = SBIM(Config.from_dict(fw.config_dict(), precision="fp32_comp",
                                       input_kind="increment"), device=device)
            obj = make(sb)
            for _ in range(window):
                obj.step()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(window):
                obj.step()
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0) / window
            obj.close()
            sb.close()
            return ms
        row["boundary_ms"] = timed(lambda sb: Fault(sb, *prm))
        for L in layers:
            row[f"hybrid{L}_ms"] = timed(lambda sb: Strip(sb, [(t["rho"], t["cp"], t["cs"])] * L, *prm))
        row["fe_node_layer_ms"] = (row[f"hybrid{layers[1]}_ms"] - row[f"hybrid{layers[0]}_ms"]) / (
            layers[1] - layers[0])
        row["boundary_us_per_kmode"] = 1e3 * row["boundary_ms"] / (row["modes"] / 1e3)
        rows.append(row)
        print(f"[bench] scaling n={n}: boundary {row['boundary_ms']:.3f} ms/step, "
              f"hybrid {layers[0]} layers {row[f'hybrid{layers[0]}_ms']:.3f} ms, "
              f"{layers[1]} layers {row[f'hybrid{layers[1]}_ms']:.3f} ms, "
              f"one node layer {row['fe_node_layer_ms']:.4f} ms", file=sys.stderr, flush=True)
        del prm
        torch.cuda.empty_cache()
    return rows


def cpu_baseline(wl, sample_modes=64, seed=0):
    """float64 oracle on one steady-state step: full naive DFTs, convolution on sampled
    modes; timed with the host's BLAS threads and again limited to one thread (the
    kernel weights, an init cost, are built once and not timed)."""
    import oracle
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        threadpool_limits = None
        cores = os.cpu_count()
    cfg = oracle.Config.from_dict(wl.config_dict())
    rng = np.random.default_rng(seed)
    P = len(cfg.planes)
    h = cfg.n3 // 2 + 1
    W = cfg.window_cap
    fields = rng.standard_normal((P, 3, cfg.n1, cfg.n3))
    ops = []
    for p in range(P):
        i1 = rng.integers(0, cfg.n1, sample_modes)
        i3 = rng.integers(0, h, sample_modes)
        op = oracle.sbim.PlaneOperator(cfg, p, (i1, i3))
        U = rng.standard_normal((W, 3, sample_modes)) + 1j * rng.standard_normal((W, 3, sample_modes))
        V = rng.standard_normal((3, sample_modes)) + 1j * rng.standard_normal((3, sample_modes))
        ops.append((op, U, V))
    M = cfg.n1 * h
    lags = P * M * W

    def one_step():
        from oracle import dft
        t0 = time.perf_counter()
        spec = dft.forward_half(fields)
        t_dft = time.perf_counter() - t0
        t_conv = 0.0
        for op, U, V in ops:
            t0 = time.perf_counter()
            op.apply_last(U, V)
            t_conv += time.perf_counter() - t0
        t0 = time.perf_counter()
        dft.inverse_half(spec, cfg.n3)
        t_dft += time.perf_counter() - t0
        return t_dft, t_conv, t_dft + t_conv * (P * M) / (P * sample_modes)

    t_dft, t_conv, step_s = one_step()
    out = {
        "value": lags / step_s, "unit": UNIT, "cores": cores, "kind": "oracle",
        "host": host_cpu(),
        "sample": (f"one steady-state step (W={W}) of {wl.name}: naive DFT forward+inverse of all "
                   f"{P}x3 fields timed in full ({t_dft:.2f} s); direct convolution timed on "
                   f"{sample_modes} random modes per plane ({t_conv:.3f} s) and scaled to all "
                   f"{P}x{M} modes; kernel weights excluded (init). value_1core: the same step "
                   f"with every thread pool limited to one thread (the convolution, which "
                   f"dominates, is a single-threaded einsum either way)"),
        "step_s_extrapolated": step_s,
    }
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            _, _, step_1 = one_step()
        out["value_1core"] = lags / step_1
        out["step_s_extrapolated_1core"] = step_1
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps at the end of the job, every mode's window full "
                         "(default: all steps of the job after the window has filled)")
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", type=int, default=2)
    ap.add_argument("--forms", default="fp32_comp,fp32,fp64")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--rupture-forms", default="fp32_comp,fp64",
                    help="forms of the rupture leg on the fault workload (empty: skip it)")
    ap.add_argument("--rupture", default="tpv3_1024", help="fault workload of the rupture leg")
    ap.add_argument("--bimaterial", action="store_true",
                    help="also time the rupture between two materials (stand-alone and two-sided strip)")
    ap.add_argument("--adjoint-forms", default="fp64,fp32_comp",
                    help="forms of the adjoint leg on the 256^2 job (empty: skip it)")
    ap.add_argument("--scaling", action="store_true",
                    help="only the step-cost sweep over grid sizes (boundary relation vs strip layers)")
    ap.add_argument("--calibrate-copy", type=float, default=0.0,
                    help="only run a torch device copy of this many GiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU per process: the boundary relation and its fault and strip run on one device; --gpus must be 1"}))
        sys.exit(2)
    import torch
    import workloads
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    device = "cuda:0"
    if args.scaling:
        print(json.dumps({"scaling": scaling_sweep(device)}))
        return
    if args.calibrate_copy:
        n = int(args.calibrate_copy * 2 ** 30 / 4)
        a = torch.ones(n, dtype=torch.float32, device=device)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": 4 * n, "dispatches": 5}))
        return
    wl = workloads.WORKLOADS[args.workload]
    steps = args.steps or default_timed_steps(wl)
    forms = [f for f in args.forms.split(",") if f]
    rforms = [f for f in args.rupture_forms.split(",") if f]
    if not forms:                       # the rupture and adjoint legs alone (profiling runs)
        aforms = [f for f in args.adjoint_forms.split(",") if f]
        print(json.dumps({
            "rupture": rupture_leg(workloads.FAULTS[args.rupture], rforms, device,
                                   args.bimaterial) if rforms else None,
            "adjoint": adjoint_leg(device, aforms) if aforms else None}))
        return
    cache = {}
    res = {}
    for f in forms:
        res[f] = measure_form(wl, f, steps, args.warmup, device, cache)
        print(f"[bench] {f}: {res[f]['value']:.4e} {UNIT}, {res[f]['ms_per_step']:.3f} ms/step, "
              f"step kernel {res[f]['roofline']['achieved']:.0f} GB/s "
              f"({100 * res[f]['roofline']['frac']:.1f}% of HBM peak)",
              file=sys.stderr, flush=True)
    acc = None
    if not args.no_accuracy and "fp64" in forms and len(forms) > 1:
        for dt in (torch.float32, torch.float64):
            if dt not in cache:
                cache[dt] = Inputs(wl, dt, device)
        acc = accuracy(wl, wl.steps, device, cache, [f for f in forms if f != "fp64"])
        print(f"[bench] accuracy: {acc}", file=sys.stderr, flush=True)
    rup = (rupture_leg(workloads.FAULTS[args.rupture], rforms, device, args.bimaterial)
           if rforms else None)
    aforms = [f for f in args.adjoint_forms.split(",") if f]
    adj = adjoint_leg(device, aforms) if aforms else None
    cpu = None if args.no_cpu else cpu_baseline(wl)
    head = forms[0]
    r = res[head]
    line = {
        "metric": METRIC, "value": r["value"], "unit": UNIT, "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if head == "fp64" else "f32", "data": "synthetic",
        "config": {"workload": wl.name, "n1": wl.n1, "n3": wl.n3, "planes": len(wl.planes),
                   "window_cap": wl.window_cap, "window_mode": wl.window_mode,
                   "time_steps": wl.steps, "timed_steps": steps,
                   "first_timed_step": r["first_timed_step"],
                   "mode_lags_per_step": r["mode_lags"] / steps,
                   "precision": head, "input_kind": wl.input_kind},
        "roofline": {k: v for k, v in r["roofline"].items()},
        "cpu_baseline": cpu,
        "forms": {f: {"value": res[f]["value"], "ms_per_step": res[f]["ms_per_step"],
                      "mode_lags_per_step": res[f]["mode_lags"] / steps,
                      "step_kernel_GBs": res[f]["roofline"]["achieved"],
                      "step_kernel_frac": res[f]["roofline"]["frac"],
                      "sweep_depth": res[f]["info"]["sweep_depth"],
                      "sweep_matrix_cores": res[f]["info"]["sweep_matrix_cores"],
                      "sweep_lag_chunks": res[f]["info"]["sweep_lag_chunks"],
                      "sweep_quads": res[f]["info"]["sweep_quads"],
                      "init_s": res[f]["init_s"],
                      "ring_bytes": res[f]["info"]["ring_bytes"],
                      "table_bytes": res[f]["info"]["table_bytes"],
                      "kernel_classes": res[f]["info"]["kernel_classes"]} for f in forms},
        "accuracy": acc,
        "rupture": rup,
        "adjoint": adj,
        "kernel_source_hash": kernel_source_hash(),
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
