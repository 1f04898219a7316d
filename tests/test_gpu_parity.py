"""GPU parity of the HIP path against the float64 CPU oracle, through the C ABI.

Tolerances (relative L2 over all planes, components, cells and steps):
float64 path 1e-12, float32 paths 1e-5, both against the float64 oracle.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_2102_08756_amd import SBIM, Config, SBIMRun

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5, "fp32_comp": 1e-5}
DEV = "cuda:0"


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def run_gpu(cfg_d, u_hist, precision, v_hist=None, tau_inf=None):
    cfg = Config.from_dict(cfg_d, precision=precision)
    sb = SBIM(cfg, device=DEV)
    dt = cfg.dtype
    out = np.empty(u_hist.shape)
    u_t = torch.tensor(u_hist, dtype=dt, device=DEV)
    v_t = torch.tensor(v_hist, dtype=dt, device=DEV) if v_hist is not None else None
    ti = torch.tensor(tau_inf, dtype=dt, device=DEV) if tau_inf is not None else None
    for n in range(u_hist.shape[0]):
        sb.push(u_t[n], None if v_t is None else v_t[n])
        out[n] = sb.tractions(None if ti is None else ti[n]).double().cpu().numpy()
    sb.close()
    return out


SMALL = {
    "square16_fixed": dict(n1=16, n3=16, window_cap=6, planes=[dict(side=1)]),
    "rect8x32_permode": dict(n1=8, n3=32, dx1=0.7, dx3=1.3, window_cap=9, window_mode="per_mode",
                             eta_w=0.5, planes=[dict(side=-1, mu=2.0, cs=0.8, cp=1.7)]),
    "two_planes_two_materials": dict(n1=16, n3=8, window_cap=5,
                                     planes=[dict(side=1), dict(side=-1, mu=1.5, cs=1.2, cp=2.5)]),
    "two_planes_shared": dict(n1=32, n3=16, window_cap=12, planes=[dict(side=1), dict(side=-1)]),
    "tiny4": dict(n1=4, n3=4, window_cap=3, planes=[dict(side=1), dict(side=-1)]),
}


def _inputs(cfg_d, steps, seed):
    rng = np.random.default_rng(seed)
    P = len(cfg_d["planes"])
    shape = (steps, P, 3, cfg_d["n1"], cfg_d["n3"])
    return rng.standard_normal(shape), rng.standard_normal(shape), rng.standard_normal(shape)


@pytest.mark.parametrize("name", sorted(SMALL))
@pytest.mark.parametrize("kind", ["absolute", "increment"])
def test_small_fp64(name, kind):
    cfg_d = dict(SMALL[name], input_kind=kind)
    u, v, ti = _inputs(cfg_d, 11, 1)
    ref = oracle.forward(cfg_d, u)
    got = run_gpu(cfg_d, u, "fp64")
    assert rel_l2(got, ref) < TOL["fp64"]
    # explicit velocity and far-field traction
    ref = oracle.forward(cfg_d, u, v, ti)
    got = run_gpu(cfg_d, u, "fp64", v, ti)
    assert rel_l2(got, ref) < TOL["fp64"]


@pytest.mark.parametrize("precision", ["fp32", "fp32_comp"])
@pytest.mark.parametrize("name", ["square16_fixed", "two_planes_two_materials", "rect8x32_permode"])
def test_small_fp32(name, precision):
    cfg_d = dict(SMALL[name], input_kind="increment")
    u, v, ti = _inputs(cfg_d, 11, 2)
    ref = oracle.forward(cfg_d, u, v, ti)
    got = run_gpu(cfg_d, u, precision, v, ti)
    assert rel_l2(got, ref) < TOL[precision]


@pytest.mark.parametrize("precision", ["fp64", "fp32_comp", "fp32"])
def test_workload_plane64_w100(precision):
    """The 64x64, W = 100, 200-step single-plane workload in full."""
    wl = workloads.WORKLOADS[1]
    du = workloads.Increments(wl).history(wl.steps)
    cfg_d = wl.config_dict()
    ref = oracle.forward(cfg_d, du)
    got = run_gpu(cfg_d, du, precision)
    err = rel_l2(got, ref)
    print(f"plane64_w100 {precision}: rel-L2 {err:.3e}")
    assert err < TOL[precision]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_kernel_tables_match_oracle(precision):
    cfg_d = dict(n1=64, n3=32, dx1=1.0, dx3=2.0, dt=0.2, window_cap=150, window_mode="per_mode",
                 eta_w=3.0, planes=[dict(side=1), dict(side=-1, mu=1.0, cs=0.7, cp=1.5)])
    sb = SBIM(Config.from_dict(cfg_d, precision=precision), device=DEV)
    ocfg = oracle.Config.from_dict(cfg_d)
    q, _, _ = oracle.mode_geometry(ocfg)
    rng = np.random.default_rng(3)
    picks = [(0, 1), (1, 0), (32, 16), (63, 5), (17, 9)] + [tuple(x) for x in rng.integers(0, [64, 17], (10, 2))]
    for p in range(2):
        pl = ocfg.planes[p]
        for i1, i3 in picks:
            W = int(oracle.mode_window(q[i1, i3], pl.cs, ocfg.dt, ocfg))
            w_gpu, tab = sb.mode_kernel(p, i1, i3, 400)
            assert w_gpu == W, (p, i1, i3)
            if W == 0:
                continue
            ref = oracle.kernels.lag_weights(q[i1, i3], pl.cs, ocfg.dt, W, pl.cp / pl.cs)
            if precision == "fp64":
                np.testing.assert_allclose(tab, ref, rtol=0, atol=1e-15)
            else:
                np.testing.assert_allclose(tab, ref.astype(np.float32), rtol=0,
                                           atol=1e-7 * np.abs(ref).max())
    sb.close()


@pytest.mark.parametrize("kind", ["absolute", "increment"])
@pytest.mark.parametrize("with_v", [False, True])
def test_adjoint_fp64(kind, with_v):
    cfg_d = dict(SMALL["two_planes_two_materials"], input_kind=kind, window_mode="per_mode",
                 eta_w=0.8)
    u, v, _ = _inputs(cfg_d, 9, 4)
    g = np.random.default_rng(5).standard_normal(u.shape)
    du_ref, dv_ref = oracle.adjoint(cfg_d, g, with_velocity=with_v)
    sb = SBIM(Config.from_dict(cfg_d, precision="fp64"), device=DEV)
    ut = torch.tensor(u, device=DEV, requires_grad=True)
    vt = torch.tensor(v, device=DEV, requires_grad=True) if with_v else None
    tau = SBIMRun.apply(sb, ut, vt)
    (tau * torch.tensor(g, device=DEV)).sum().backward()
    assert rel_l2(ut.grad.cpu().numpy(), du_ref) < 1e-12
    if with_v:
        assert rel_l2(vt.grad.cpu().numpy(), dv_ref) < 1e-12
    sb.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_count_nonfinite(precision):
    """The library's non-finite count of a field: zero for finite values, the number of
    planted infinities and NaNs otherwise, and a NaN pushed into the history shows up in
    the tractions."""
    cfg_d = SMALL["two_planes_shared"]
    sb = SBIM(Config.from_dict(cfg_d, precision=precision), device=DEV)
    u = torch.randn(sb.shape, dtype=sb.dtype, device=DEV)
    assert sb.count_nonfinite(u) == 0
    bad = u.clone()
    flat = bad.view(-1)
    flat[0], flat[17], flat[-1] = float("nan"), float("inf"), float("-inf")
    flat[1000] = float("nan")
    assert sb.count_nonfinite(bad) == 4
    sb.push(u)
    assert sb.count_nonfinite(sb.tractions()) == 0
    sb.push(bad)
    assert sb.count_nonfinite(sb.tractions()) > 0
    sb.close()


def test_deterministic_bitwise():
    cfg_d = dict(SMALL["two_planes_shared"], input_kind="increment")
    u, _, _ = _inputs(cfg_d, 15, 6)
    a = run_gpu(cfg_d, u, "fp32_comp")
    b = run_gpu(cfg_d, u, "fp32_comp")
    assert np.array_equal(a, b)


# Several 64-mode blocks with ragged per-mode windows, run long enough for
# every block to sweep many times: exercises the split of each history sum
# into the block's last sweep and the newer lags, at every sweep depth.
SWEEP_CFG = dict(n1=32, n3=64, dx1=1.0, dx3=0.8, dt=0.2, window_cap=40, window_mode="per_mode",
                 eta_w=1.5, input_kind="increment", planes=[dict(side=1), dict(side=-1)])


# Windows of one and two lags (blocks whose capacity is below the sweep depth)
# next to windows up to the cap.
TINYWIN_CFG = dict(n1=32, n3=16, dx1=1.0, dx3=1.0, dt=0.2, window_cap=5, window_mode="per_mode",
                   eta_w=0.04, input_kind="absolute", planes=[dict(side=1), dict(side=-1)])
SWEEP_CASES = {"ragged40": (SWEEP_CFG, 90, 7), "tinywin": (TINYWIN_CFG, 30, 9)}


@pytest.fixture(scope="module")
def sweep_refs():
    out = {}
    for name, (cfg, steps, seed) in SWEEP_CASES.items():
        u, _, _ = _inputs(cfg, steps, seed)
        out[name] = (u, oracle.forward(cfg, u))
    return out


@pytest.mark.parametrize("case", sorted(SWEEP_CASES))
@pytest.mark.parametrize("depth", [1, 2, 4, 6, 8, 12, 16])
@pytest.mark.parametrize("precision", ["fp64", "fp32_comp", "fp32"])
def test_sweep_depths(sweep_refs, case, depth, precision, monkeypatch):
    monkeypatch.setenv("SBIM_SWEEP_DEPTH", str(depth))
    cfg = SWEEP_CASES[case][0]
    u, ref = sweep_refs[case]
    sb = SBIM(Config.from_dict(cfg, precision=precision), device=DEV)
    assert sb.info()["sweep_depth"] == depth
    sb.close()
    got = run_gpu(cfg, u, precision)
    err = rel_l2(got, ref)
    print(f"{case} sweep depth {depth} {precision}: rel-L2 {err:.3e}")
    assert err < TOL[precision]


@pytest.mark.parametrize("precision,long_depth", [("fp32", 8), ("fp32_comp", 12), ("fp64", 12)])
def test_default_sweep_depth(precision, long_depth, monkeypatch):
    """Long windows: 8 steps per sweep for float32 (12 from 1500 lags), 12 (two lanes per
    mode) for float64 and the compensated form; per-mode windows averaging under 64 lags
    (here 18): 6."""
    monkeypatch.delenv("SBIM_SWEEP_DEPTH", raising=False)
    long_w = dict(n1=64, n3=64, window_cap=100, planes=[dict(side=1)])
    short_w = dict(n1=64, n3=64, window_cap=400, window_mode="per_mode", eta_w=1.0,
                   planes=[dict(side=1), dict(side=-1)])
    longer_w = dict(n1=16, n3=16, window_cap=1600, planes=[dict(side=1)])
    for cfg, want in ((long_w, long_depth), (short_w, 6), (longer_w, 12)):
        sb = SBIM(Config.from_dict(cfg, precision=precision), device=DEV)
        assert sb.info()["sweep_depth"] == want, (cfg["window_mode"] if "window_mode" in cfg else "fixed")
        sb.close()


def test_tractions_repeatable_and_snapshots_mid_rotation():
    """tractions() changes no state; a snapshot taken at a step that is not a
    multiple of the sweep depth restores the pending sums exactly."""
    sb = SBIM(Config.from_dict(SWEEP_CFG, precision="fp32"), device=DEV)
    depth = sb.info()["sweep_depth"]
    steps = 3 * depth + 20
    u = _inputs(SWEEP_CFG, steps, 8)[0]
    ut = torch.tensor(u, dtype=torch.float32, device=DEV)
    snap = torch.empty(sb.state_bytes(), dtype=torch.uint8, device=DEV)
    cut = 2 * depth + 3
    first = []
    for n in range(steps):
        sb.push(ut[n])
        a = sb.tractions().clone()
        b = sb.tractions().clone()
        assert torch.equal(a, b), n
        first.append(a)
        if n == cut:
            sb.save_state(snap)
    sb.load_state(snap)
    for n in range(cut + 1, steps):
        sb.push(ut[n])
        assert torch.equal(sb.tractions(), first[n]), n
    sb.close()


@pytest.mark.parametrize("depth", [1, 2, 6, 8, 12, 16])
@pytest.mark.parametrize("kind", ["absolute", "increment"])
def test_adjoint_sweep_depths(depth, kind, monkeypatch):
    """The adjoint runs the same sweep on its own history: exact transpose at every depth."""
    monkeypatch.setenv("SBIM_SWEEP_DEPTH", str(depth))
    cfg_d = dict(SWEEP_CFG, input_kind=kind)
    u, _, _ = _inputs(cfg_d, 30, 10)
    g = np.random.default_rng(11).standard_normal(u.shape)
    du_ref, _ = oracle.adjoint(cfg_d, g)
    sb = SBIM(Config.from_dict(cfg_d, precision="fp64"), device=DEV)
    assert sb.info()["sweep_depth"] == depth
    ut = torch.tensor(u, device=DEV, requires_grad=True)
    tau = SBIMRun.apply(sb, ut)
    (tau * torch.tensor(g, device=DEV)).sum().backward()
    err = rel_l2(ut.grad.cpu().numpy(), du_ref)
    print(f"adjoint depth {depth} {kind}: rel-L2 {err:.3e}")
    assert err < 1e-12
    sb.close()


def test_oversize_ring_is_refused_before_allocating():
    """A window whose ring cannot fit in device memory: SBIM_E_OOM from sbim_init, with
    nothing allocated, and the device stays usable."""
    from paper_2102_08756_amd import SBIMError
    free0, _ = torch.cuda.mem_get_info()
    cfg = Config.from_dict(dict(n1=4096, n3=4096, window_cap=1 << 20,
                                planes=[dict(side=1), dict(side=-1)]), precision="fp64")
    with pytest.raises(SBIMError, match="SBIM_E_OOM"):
        SBIM(cfg, device=DEV)
    free1, _ = torch.cuda.mem_get_info()
    assert abs(free1 - free0) < 64 << 20
    cfg_d = dict(SMALL["tiny4"], input_kind="absolute")
    u, _, _ = _inputs(cfg_d, 3, 5)
    np.testing.assert_allclose(run_gpu(cfg_d, u, "fp64"), oracle.forward(cfg_d, u), rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("every", [1, 3])
def test_launch_timing_every_nth(every):
    """sbim_profile_conv(h, n) brackets the first step launch after the call and every n-th
    after it; timing changes no result; n < 0 is refused."""
    from paper_2102_08756_amd import SBIMError
    cfg_d = dict(SMALL["two_planes_shared"], input_kind="increment")
    u, _, _ = _inputs(cfg_d, 10, 11)
    sb = SBIM(Config.from_dict(cfg_d, precision="fp32_comp"), device=DEV)
    u_t = torch.tensor(u, dtype=torch.float32, device=DEV)
    sb.profile_conv(True, every)
    out = np.empty(u.shape)
    for n in range(u.shape[0]):
        sb.push(u_t[n])
        out[n] = sb.tractions().double().cpu().numpy()
    ms, launches = sb.conv_timing()
    assert launches == (u.shape[0] + every - 1) // every
    assert ms > 0.0
    with pytest.raises(SBIMError, match="SBIM_E_INVALID"):
        sb.profile_conv(True, -1)
    sb.profile_conv(False)
    sb.push(u_t[0])
    assert sb.conv_timing() == (0.0, 0)
    sb.close()
    assert np.array_equal(out, run_gpu(cfg_d, u, "fp32_comp"))
