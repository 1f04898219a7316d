"""Differentiable SBIM on the 256x256, W=300, 500-step single-plane workload.

Loss L = sum_n sum_{r in R} sum_i tau_i^n(x_r)^2 over 64 receiver cells R drawn
without replacement (seed 4000).  Checks, all through the C ABI:
  * autograd gradient (sbim_backward over n = N-1..0) against central finite
    differences on the float64 path along 32 Gaussian directions (seeds
    4100+i, eps = 1e-6): L is quadratic, so central differences are exact up
    to round-off; bar 1e-4 relative;
  * the same gradient against the oracle's transpose on sampled Fourier bins
    (full size; bar 1e-12 of the gradient field's norm, estimated relative L2);
  * segment checkpointing (snapshots every 50 steps, recomputation of each
    segment in the backward) gives the same gradient;
  * the float32 adjoint against the float64 one (bar 1e-4 relative L2).
"""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_2102_08756_amd import SBIM, Config, SBIMRun, checkpointed_loss

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def setup():
    wl = workloads.WORKLOADS[4]
    du = workloads.Increments(wl).history(wl.steps)            # [500, 1, 3, 256, 256]
    rng = np.random.default_rng(4000)
    cells = rng.choice(wl.n1 * wl.n3, 64, replace=False)
    r1, r3 = cells // wl.n3, cells % wl.n3
    return wl, du, (r1, r3)


def loss_of(tau_hist, rec):
    r1, r3 = rec
    return (tau_hist[..., r1, r3] ** 2).sum()


def grad_autograd(wl, du, rec, precision):
    sb = SBIM(Config.from_dict(wl.config_dict(), precision=precision), device=DEV)
    dt = sb.dtype
    u = torch.tensor(du, dtype=dt, device=DEV, requires_grad=True)
    tau = SBIMRun.apply(sb, u)
    L = loss_of(tau, (torch.tensor(rec[0], device=DEV), torch.tensor(rec[1], device=DEV)))
    L.backward()
    g = u.grad.double()
    sb.close()
    return float(L.detach()), g


def test_gradient_finite_differences_fp64(setup):
    wl, du, rec = setup
    L0, g = grad_autograd(wl, du, rec, "fp64")
    print(f"[adjoint] L = {L0:.6e}", flush=True)
    sb = SBIM(Config.from_dict(wl.config_dict(), precision="fp64"), device=DEV)
    u = torch.tensor(du, dtype=torch.float64, device=DEV)
    r1 = torch.tensor(rec[0], device=DEV)
    r3 = torch.tensor(rec[1], device=DEV)
    eps = 1e-6

    def L_at(x):
        with torch.no_grad():
            return float(loss_of(SBIMRun.apply(sb, x), (r1, r3)))

    worst = 0.0
    for i in range(32):
        gen = torch.Generator(device=DEV).manual_seed(4100 + i)
        V = torch.randn(u.shape, generator=gen, dtype=torch.float64, device=DEV)
        fd = (L_at(u + eps * V) - L_at(u - eps * V)) / (2 * eps)
        an = float((g * V).sum())
        rel = abs(fd - an) / max(abs(an), 1e-300)
        worst = max(worst, rel)
        assert rel < 1e-4, (i, fd, an)
    print(f"[adjoint] 32 central differences: worst relative deviation {worst:.3e}", flush=True)
    sb.close()


def test_gradient_matches_oracle_transpose_on_bins(setup):
    wl, du, rec = setup
    _, g = grad_autograd(wl, du, rec, "fp64")
    sb = SBIM(Config.from_dict(wl.config_dict(), precision="fp64"), device=DEV)
    u = torch.tensor(du, dtype=torch.float64, device=DEV)
    with torch.no_grad():
        tau = SBIMRun.apply(sb, u).cpu().numpy()
    sb.close()
    # dL/dtau: 2 tau at the receivers (the oracle takes it as given, as the library does)
    gt = np.zeros_like(tau)
    r1, r3 = rec
    gt[..., r1, r3] = 2 * tau[..., r1, r3]
    rng = np.random.default_rng(44)
    i1 = np.concatenate([[0], rng.integers(0, wl.n1, 14), [wl.n1 // 2]])
    i3 = np.concatenate([[0], rng.integers(1, wl.n3 // 2, 14), [1]])
    G = oracle.dft.forward_half_fft(gt)[..., i1, i3]                    # [N, 1, 3, B]
    ref, _ = oracle.adjoint_response(wl.config_dict(), 0, (i1, i3), G[:, 0])
    gn = g.cpu().numpy()
    got = oracle.dft.forward_half_fft(gn)[..., i1, i3][:, 0]
    norm = np.sqrt((gn[:, 0] ** 2).sum(axis=(-1, -2)))[..., None]
    err = np.abs(got - ref) / np.maximum(norm, 1e-300)
    rms = float(np.sqrt(np.mean(err ** 2)))
    print(f"[adjoint] gradient vs oracle transpose: rms {rms:.3e}, max {err.max():.3e}", flush=True)
    assert rms < 1e-12 and err.max() < 1e-11


def test_checkpointed_loss_matches_and_fp32_adjoint(setup):
    wl, du, rec = setup
    L64, g64 = grad_autograd(wl, du, rec, "fp64")
    sb = SBIM(Config.from_dict(wl.config_dict(), precision="fp64"), device=DEV)
    u = torch.tensor(du, dtype=torch.float64, device=DEV, requires_grad=True)
    r1 = torch.tensor(rec[0], device=DEV)
    r3 = torch.tensor(rec[1], device=DEV)
    L = checkpointed_loss(sb, u, lambda t, n: (t[..., r1, r3] ** 2).sum(), every=50)
    L.backward()
    sb.close()
    assert abs(float(L) - L64) < 1e-12 * L64
    rel = float((u.grad - g64).norm() / g64.norm())
    print(f"[adjoint] checkpointed (every 50) vs plain gradient: rel-L2 {rel:.3e}", flush=True)
    assert rel < 1e-12
    L32, g32 = grad_autograd(wl, du, rec, "fp32")
    rel32 = float((g32 - g64).norm() / g64.norm())
    print(f"[adjoint] float32 vs float64 gradient: rel-L2 {rel32:.3e}; loss {abs(L32 - L64) / L64:.3e}",
          flush=True)
    assert rel32 < 1e-4


@pytest.mark.parametrize("precision,kind", [("fp64", "increment"), ("fp32_comp", "increment"),
                                            ("fp32", "absolute")])
def test_running_state_snapshot_and_replay(precision, kind, monkeypatch):
    """A light snapshot (float64 running state and step counter) of step n0, then the pushes
    of steps n0 .. a-1 again (a - n0 = W_cap + sweep_depth + 2): from step a on the tractions
    equal the original run's bit for bit.  Two planes of one material at W = 40 take the
    matrix-core sweep in the float32 forms (forced), the float64 form the vector sweep."""
    monkeypatch.setenv("SBIM_SWEEP_KIND", "mfma")
    cfg = dict(n1=32, n3=32, window_cap=40, planes=[dict(side=1), dict(side=-1)], input_kind=kind)
    sb = SBIM(Config.from_dict(cfg, precision=precision), device=DEV)
    R = sb.replay_steps()
    assert sb.running_state_bytes() * 20 < sb.state_bytes()
    rng = np.random.default_rng(21)
    steps = 2 * R + 30
    u = torch.tensor(rng.standard_normal((steps, 2, 3, 32, 32)), dtype=sb.dtype, device=DEV)
    n0 = 17
    a = n0 + R
    ref = []
    for n in range(steps):
        if n == n0:
            snap = sb.save_running_state()
        sb.push(u[n])
        ref.append(sb.tractions().clone())
    sb.load_running_state(snap)
    assert sb.info()["step"] == n0
    for n in range(n0, a):
        sb.push(u[n])
    for n in range(a, steps):
        sb.push(u[n])
        assert torch.equal(sb.tractions(), ref[n]), n
    sb.close()


def test_checkpointed_loss_memory_and_replay_cost(setup):
    """The checkpoints of checkpointed_loss hold the running state only: on the 256^2,
    W = 300 job they total a few MB against the whole traction history that SBIMRun
    keeps (0.79 GB in float64)."""
    wl, du, rec = setup
    sb = SBIM(Config.from_dict(wl.config_dict(), precision="fp64"), device=DEV)
    N = du.shape[0]
    snaps = len({max(0, s * 50 - sb.replay_steps()) for s in range((N + 49) // 50)})
    ckpt = snaps * sb.running_state_bytes()
    full = N * 3 * wl.n1 * wl.n3 * 8
    print(f"[adjoint] checkpoints {snaps} x {sb.running_state_bytes()} B = {ckpt / 1e6:.1f} MB "
          f"against {full / 1e6:.0f} MB of tractions", flush=True)
    assert ckpt * 50 < full
    sb.close()
