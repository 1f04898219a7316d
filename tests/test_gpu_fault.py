"""GPU parity of the frictional fault (``sbim_fault_*``) against the oracle's rupture.

Every case runs the library's explicit step (push without damping, inverse
transform, interface solve) and ``oracle.fault.rupture`` on the same seeded
workload and compares, per step and cell, the fault traction, the slip rate,
the slip and both sides' displacement and velocity.  Bars,
relative to each field's largest magnitude over the run: float64 1e-12 (measured
1e-14 to 2e-14: the transforms and history sums agree to ~1e-15 of the field,
and the stick/slip choice and the weakening amplify that by the ratio of shear
modulus to strength drop), and the set of slipping cells must agree exactly.  The float32 forms carry the
traction functional in float32 (relative error ~1e-7 of its field); a cell
whose stick/slip choice falls within that error of the strength could switch a
step early or late, so they are compared by relative L2 over the run (bar
1e-5, the bar of the traction update's float32 forms) and by the step at
which each cell first slips (within one step).
"""
import math

import numpy as np
import pytest
import torch

import workloads
from oracle import fault as ofault
from oracle.sbim import Config as OConfig
from paper_2102_08756_amd import SBIM, Config, Fault, SBIMError

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

_REF = {}


def oracle_run(name, steps=None):
    wl = workloads.FAULTS[name]
    steps = steps or wl.steps
    key = (name, steps)
    if key not in _REF:
        tau0, mu_s, mu_k, d_c = wl.params()
        _REF[key] = ofault.rupture(OConfig.from_dict(dict(wl.config_dict(), input_kind="absolute")),
                                   ofault.FaultParams(tau0, mu_s, mu_k, d_c), steps)
    return _REF[key]


def make_fault(wl, precision, kind, params=None):
    cfg = Config.from_dict(wl.config_dict(), precision=precision, input_kind=kind)
    sb = SBIM(cfg, device=DEV)
    p = params if params is not None else wl.params()
    t = [torch.tensor(a, dtype=torch.float64, device=DEV).contiguous() for a in p]
    return sb, Fault(sb, *t)


def gpu_run(name, precision, kind, steps=None):
    wl = workloads.FAULTS[name]
    steps = steps or wl.steps
    sb, f = make_fault(wl, precision, kind)
    out = {k: [] for k in ("traction", "slip_rate", "slip", "v_plus", "v_minus", "u_plus")}
    for n in range(steps):
        f.step()
        out["traction"].append(f.read("traction"))
        out["slip_rate"].append(f.read("slip_rate"))
        out["slip"].append(f.read("slip"))
        v = f.read("velocity")
        out["v_plus"].append(v[:3])
        out["v_minus"].append(v[3:])
        out["u_plus"].append(f.read("displacement")[:3])
    res = {k: torch.stack(v).cpu().numpy() for k, v in out.items()}
    f.close()
    sb.close()
    return res


def first_slip(rate):
    V = np.sqrt((rate ** 2).sum(1))
    s = V > 0
    return np.where(s.any(0), np.argmax(s, axis=0), -1)


CASES = ["tpv3_coarse16", "tpv3_coarse32", "tpv3_rect32x16", "bimaterial32"]


@pytest.mark.parametrize("kind", ["absolute", "increment"])
@pytest.mark.parametrize("name", CASES)
def test_fault_fp64_matches_oracle(name, kind):
    wl = workloads.FAULTS[name]
    ref = oracle_run(name)
    got = gpu_run(name, "fp64", kind)
    worst = {}
    for key in ("traction", "slip_rate", "slip", "v_plus", "v_minus"):
        scale = max(np.abs(ref[key]).max(), 1e-300)
        worst[key] = float(np.abs(got[key] - ref[key]).max() / scale)
    # displacement of the upper side: the running sum of dt v+
    u_ref = np.cumsum(ref["v_plus"], axis=0) * wl.dt
    worst["u_plus"] = float(np.abs(got["u_plus"] - u_ref).max() / np.abs(u_ref).max())
    print(f"[fault] {name} fp64 {kind}: " + ", ".join(f"{k} {v:.2e}" for k, v in worst.items()), flush=True)
    np.testing.assert_array_equal(first_slip(got["slip_rate"]), first_slip(ref["slip_rate"]))
    np.testing.assert_array_equal(got["slip_rate"] > 0, ref["slip_rate"] > 0)
    for key, w in worst.items():
        assert w < 1e-12, (key, w)


@pytest.mark.parametrize("precision", ["fp32", "fp32_comp"])
@pytest.mark.parametrize("name", ["tpv3_coarse32", "bimaterial32"])
def test_fault_fp32_forms_against_oracle(name, precision):
    ref = oracle_run(name)
    got = gpu_run(name, precision, "increment")
    errs = {}
    for key in ("traction", "slip_rate", "slip"):
        errs[key] = float(np.linalg.norm(got[key] - ref[key]) / np.linalg.norm(ref[key]))
    fg, fr = first_slip(got["slip_rate"]), first_slip(ref["slip_rate"])
    both = (fg >= 0) & (fr >= 0)
    print(f"[fault] {name} {precision}: rel-L2 " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items())
          + f"; first-slip steps differ at {int((fg != fr).sum())} cells (max {int(np.abs(fg - fr)[both].max())})",
          flush=True)
    assert np.array_equal(fg >= 0, fr >= 0)
    assert np.abs(fg - fr)[both].max() <= 1
    for key, e in errs.items():
        assert e < 1e-5, (key, e)


def test_fault_uniform_and_locked_edge_cases():
    """k = 0 only (uniform stress above strength) and a fault that never slips."""
    wl = workloads.FaultWorkload("uniform8x4", 8, 4, 375.0, 40, region=(1e9, 1e9))
    tau0, mu_s, mu_k, d_c = wl.params()
    tau0[0] = (workloads.TPV3["mu_s"] + 0.01) * workloads.TPV3["sigma0"]   # everywhere above strength
    cfg_o = OConfig.from_dict(dict(wl.config_dict(), input_kind="absolute"))
    ref = ofault.rupture(cfg_o, ofault.FaultParams(tau0, mu_s, mu_k, d_c), wl.steps)
    sb, f = make_fault(wl, "fp64", "increment", (tau0, mu_s, mu_k, d_c))
    tau, rate = f.run(wl.steps)
    # x3 components are round-off around zero on both sides
    np.testing.assert_allclose(rate.cpu().numpy(), ref["slip_rate"], rtol=1e-12,
                               atol=1e-12 * np.abs(ref["slip_rate"]).max())
    np.testing.assert_allclose(tau.cpu().numpy(), ref["traction"], rtol=1e-12,
                               atol=1e-12 * np.abs(ref["traction"]).max())
    assert (ref["slip_rate"][:, 0] > 0).all()
    f.close()
    sb.close()
    # locked: the background stays below strength everywhere
    tau0[0] = 0.5 * workloads.TPV3["tau0"]
    sb, f = make_fault(wl, "fp32_comp", "increment", (tau0, mu_s, mu_k, d_c))
    tau, rate = f.run(10)
    assert float(rate.abs().max()) == 0.0
    # the impedance-weighted mean of two equal values is that value to an ulp
    np.testing.assert_allclose(tau[-1].cpu().numpy(), tau0, rtol=1e-15)
    assert float(f.read("displacement").abs().max()) < 1e-12
    f.close()
    sb.close()


def test_fault_reset_repeats_and_outputs_agree():
    wl = workloads.FAULTS["tpv3_rect32x16"]
    sb, f = make_fault(wl, "fp32_comp", "increment")
    tau_a, rate_a = f.run(30)
    slip_a = f.read("slip")
    f.reset()
    tau_b, rate_b = f.run(30)
    assert torch.equal(tau_a, tau_b) and torch.equal(rate_a, rate_b)
    assert torch.equal(slip_a, f.read("slip"))
    # the outputs passed to step equal the stored fields of the same step
    assert torch.equal(tau_b[-1], f.read("traction")) and torch.equal(rate_b[-1], f.read("slip_rate"))
    f.close()
    sb.close()


def test_fault_argument_errors():
    wl = workloads.FAULTS["tpv3_coarse16"]
    tau0, mu_s, mu_k, d_c = wl.params()
    bad = d_c.copy()
    bad[3, 5] = 0.0
    with pytest.raises(SBIMError, match=r"i1=3, i3=5"):
        make_fault(wl, "fp64", "increment", (tau0, mu_s, mu_k, bad))
    bad = mu_k.copy()
    bad[7, 1] = 2.0 * mu_s[7, 1]
    with pytest.raises(SBIMError, match=r"i1=7, i3=1"):
        make_fault(wl, "fp64", "increment", (tau0, mu_s, bad, d_c))
    t = tau0.copy()
    t[2, 0, 0] = np.nan
    with pytest.raises(SBIMError, match=r"i1=0, i3=0"):
        make_fault(wl, "fp64", "increment", (t, mu_s, mu_k, d_c))
    # planes must be (+1) or (+1, -1)
    cfg = Config.from_dict(dict(wl.config_dict(), planes=[dict(wl.upper(), side=-1)]))
    sb = SBIM(cfg, device=DEV)
    args = [torch.tensor(a, dtype=torch.float64, device=DEV) for a in (tau0, mu_s, mu_k, d_c)]
    with pytest.raises(SBIMError, match="SBIM_E_INVALID"):
        Fault(sb, *args)
    sb.close()
    # the handle must be at step 0, and only the fault may step it
    sb = SBIM(Config.from_dict(wl.config_dict()), device=DEV)
    sb.push(sb.new_field().zero_())
    with pytest.raises(SBIMError, match="SBIM_E_STATE"):
        Fault(sb, *args)
    sb.reset()
    f = Fault(sb, *args)
    f.step()
    sb.push(sb.new_field().zero_())
    with pytest.raises(SBIMError, match="SBIM_E_STATE"):
        f.step()
    f.close()
    sb.close()


def test_fault_tiny_grid_partial_tile():
    """4 x 8 cells: fewer cells than one work-group of the interface kernel."""
    wl = workloads.FaultWorkload("tiny4x8", 4, 8, 750.0, 30, region=(2250.0, 4500.0), patch=1500.0)
    tau0, mu_s, mu_k, d_c = wl.params()
    cfg_o = OConfig.from_dict(dict(wl.config_dict(), input_kind="absolute"))
    ref = ofault.rupture(cfg_o, ofault.FaultParams(tau0, mu_s, mu_k, d_c), wl.steps)
    assert (ref["slip_rate"] > 0).any()
    sb, f = make_fault(wl, "fp64", "absolute")
    tau, rate = f.run(wl.steps)
    scale = np.abs(ref["traction"]).max()
    assert np.abs(tau.cpu().numpy() - ref["traction"]).max() < 1e-12 * scale
    np.testing.assert_array_equal(rate.cpu().numpy() > 0, ref["slip_rate"] > 0)
    f.close()
    sb.close()


def _full_run(fw, precision):
    """The whole run, recording the step at which each cell first slips."""
    sb, f = make_fault(fw, precision, "increment")
    n1, n3 = fw.n1, fw.n3
    first = torch.full((n1, n3), -1, dtype=torch.int32, device=DEV)
    rate = torch.empty((2, n1, n3), dtype=torch.float64, device=DEV)
    for n in range(fw.steps):
        f.step(slip_rate=rate)
        moving = (rate[0] != 0) | (rate[1] != 0)
        first = torch.where(moving & (first < 0), torch.full_like(first, n), first)
    slip = f.read("slip").cpu().numpy()
    first = first.cpu().numpy()
    f.close()
    sb.close()
    torch.cuda.empty_cache()
    return first, slip


def test_tpv3_full_size_invariants():
    """1024 x 1024 cells of 50 m, 2000 steps (the paper's resolution and setup):
    causality (no cell slips before a P wave from the patch reaches it), locked
    cells never slip, the rupture runs across the whole rupture region, and the
    compensated float32 form follows float64 (rupture time within a step at
    almost every cell; final slip within 1e-3 relative L2)."""
    fw = workloads.FAULTS["tpv3_1024"]
    f64, s64 = _full_run(fw, "fp64")
    f32, s32 = _full_run(fw, "fp32_comp")
    patch, region = fw.masks()
    X1, X3 = fw.coords()
    h = fw.patch / 2
    dist = np.hypot(np.maximum(np.abs(X1) - h, 0), np.maximum(np.abs(X3) - h, 0))
    cp = workloads.TPV3["cp"]
    for first in (f64, f32):
        ever = first >= 0
        assert (first[patch] == 0).all()
        assert not ever[~region].any()
        assert ever[region].all()
        assert np.all(dist[ever] <= cp * (first[ever] + 1) * fw.dt + 1e-6)
    both = (f64 >= 0) & (f32 >= 0)
    diff = np.abs(f64 - f32)[both]
    rel = float(np.linalg.norm(s32 - s64) / np.linalg.norm(s64))
    edge = first_edge = int(f64[fw.n1 // 2 + int(14500 / fw.dx), fw.n3 // 2])
    print(f"[fault] tpv3_1024: rupture reaches x1 = 14.5 km at step {edge} "
          f"({edge * fw.dt:.2f} s); fp32_comp vs fp64: rupture step differs at "
          f"{int((diff > 0).sum())} of {int(both.sum())} cells (max {int(diff.max())}), "
          f"final slip rel-L2 {rel:.2e}", flush=True)
    assert first_edge > 0
    assert (diff <= 1).mean() > 0.999
    assert rel < 1e-3
