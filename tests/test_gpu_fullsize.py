"""Full-size GPU parity on sampled Fourier bins, in the launch configuration bench.py times.

The float64 oracle cannot evaluate whole 512^2..2048^2 fields over thousands of
steps, so it computes the traction spectrum at a few bins from the inputs
(``oracle.mode_response``; input spectra by ``oracle.dft.forward_half_fft``)
and the GPU output's spectrum at the same bins is measured with an explicit
DFT.  Bin errors are normalised by the L2 norm of the traction field of that
plane, component and step: by Parseval their RMS over uniformly drawn bins
estimates the field's relative L2 error, which carries the bars: 1e-12 for the
float64 path and 1e-5 for the float32 forms (whose inputs are the float32
rounding of the same fields).  The largest single-bin error is bounded at ten
times the bar: a bin that holds much of the field's energy (the uniform slip
at k = 0) carries its own rounding, relative to itself, scaled up by
sqrt(n1 n3) in this normalisation, and the highest-|k| bins collect the white
rounding noise of the inputs with the largest traction multiplier.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_2102_08756_amd import SBIM, Config

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def pick_bins(n1, n3, count, seed):
    rng = np.random.default_rng(seed)
    i1 = rng.integers(0, n1, count)
    i3 = rng.integers(1, n3 // 2, count)          # interior columns: no Hermitian folding
    i1 = np.concatenate([[0], i1, [n1 // 2]])       # DC and the Nyquist row
    i3 = np.concatenate([[0], i3, [1]])
    return i1, i3


def oracle_bins(wl, bins, steps):
    fields, index, uniform = workloads.step_sources(wl)
    i1, i3 = bins
    X = np.stack([oracle.dft.forward_half_fft(f)[..., i1, i3] for f in fields])   # [nf, P, 3, B]
    X = X[[index(n) for n in range(steps)]]
    dc = (i1 == 0) & (i3 == 0)
    X[:, :, :, dc] += (np.stack([uniform(n) for n in range(steps)]) * (wl.n1 * wl.n3))[..., None]
    cfg = oracle.Config.from_dict(wl.config_dict())
    assert cfg.input_kind == "increment"
    U = np.cumsum(X, axis=0)
    V = X / cfg.dt
    out = np.empty_like(U)
    cache = {}
    for p in range(len(cfg.planes)):
        out[:, p] = oracle.mode_response(cfg, p, bins, U[:, p], V[:, p], cache)
    return out


def gpu_bins(wl, precision, bins, steps):
    cfg = Config.from_dict(wl.config_dict(), precision=precision)
    sb = SBIM(cfg, device=DEV)
    import bench
    inputs = bench.Inputs(wl, cfg.dtype, DEV)
    n1, n3 = wl.n1, wl.n3
    i1, i3 = bins
    x1 = torch.arange(n1, dtype=torch.float64, device=DEV)
    x3 = torch.arange(n3, dtype=torch.float64, device=DEV)
    b1 = torch.tensor(i1, dtype=torch.float64, device=DEV)
    b3 = torch.tensor(i3, dtype=torch.float64, device=DEV)
    E3 = torch.exp(-2j * math.pi * torch.remainder(torch.outer(x3, b3), n3) / n3)      # [n3, B]
    E1 = torch.exp(-2j * math.pi * torch.remainder(torch.outer(b1, x1), n1) / n1)      # [B, n1]
    P = len(wl.planes)
    got = torch.empty((steps, P * 3, len(i1)), dtype=torch.complex128, device=DEV)
    norm = torch.empty((steps, P * 3), dtype=torch.float64, device=DEV)
    tau = sb.new_field()
    for n in range(steps):
        sb.push(inputs(n))
        sb.tractions(out=tau)
        t = tau.double().reshape(P * 3, n1, n3)
        tmp = t.to(torch.complex128) @ E3                                  # [F, n1, B]
        got[n] = (tmp * E1.T[None]).sum(1)
        norm[n] = torch.sqrt((t * t).sum((1, 2)))
    sb.close()
    return got.cpu().numpy().reshape(steps, P, 3, -1), norm.cpu().numpy().reshape(steps, P, 3)


CASES = {
    "two_planes512_w1000": (2, {}, None, ["fp64", "fp32_comp"]),
    "plane256_w300": (4, {}, None, ["fp64", "fp32"]),
    "two_planes2048_permode400": (3, {"bank": 8}, 450, ["fp32_comp"]),
    "two_planes1024_w2000": (5, {"slip_ramp": 10.0}, 2100, ["fp32_comp"]),
    # the largest grid the library accepts (4096-point transforms along both axes)
    "two_planes4096_permode8": (3, {"n1": 4096, "n3": 4096, "window_cap": 8, "bank": 2}, 12,
                                ["fp64", "fp32_comp"]),
}


@pytest.mark.parametrize("name", list(CASES))
def test_fullsize_sampled_bins(name):
    ident, over, steps, forms = CASES[name]
    wl = workloads.WORKLOADS[ident]
    if over:
        wl = wl.scaled(**over)
    if steps is None:
        steps = wl.steps
    if wl.slip_ramp:
        wl = wl.scaled(steps=steps)   # ramp reaches its final velocity at the last simulated step
    bins = pick_bins(wl.n1, wl.n3, 16, ident)
    print(f"[{name}] {wl.n1}x{wl.n3} x{len(wl.planes)}, W={wl.window_cap} {wl.window_mode}, "
          f"{steps} steps, forms {forms}", flush=True)
    ref = oracle_bins(wl, bins, steps)
    for form in forms:
        got, norm = gpu_bins(wl, form, bins, steps)
        err = np.abs(got - ref) / np.maximum(norm[..., None], 1e-300)
        rms, mx = float(np.sqrt(np.mean(err ** 2))), float(err.max())
        worst = np.unravel_index(np.argmax(err), err.shape)
        print(f"[{name}] {form}: bin error / field norm: rms {rms:.3e}, max {mx:.3e} at step "
              f"{worst[0]}, plane {worst[1]}, component {worst[2]}, bin "
              f"({bins[0][worst[3]]}, {bins[1][worst[3]]})", flush=True)
        if form == "fp64":
            assert rms < 1e-12 and mx < 1e-11
        else:
            assert rms < 1e-5 and mx < 1e-4
