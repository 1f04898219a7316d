"""GPU parity of the hybrid finite-element strip (``sbim_strip_*``) against the oracle.

Each case runs the library's step (predictor, S+ push and tractions, stencil
forces, fault solve, corrector) and ``oracle.hybrid.hybrid_rupture`` (element
loop, naive transforms, direct history sums) on the same workload, and
compares per step: fault traction, slip rate, slip, the set of sliding nodes,
and the S+ layer's displacement.  Bars relative to each field's largest value
over the run: float64 1e-12 (measured 5e-15 to 3e-13) with identical sliding sets; float32 forms
(boundary relation in float32, strip in float64) 1e-5 relative L2 with rupture
onset within one step.  At full size (1024 x 1024 cells of 50 m) the hybrid
rupture is compared with the stand-alone boundary-integral rupture of the same
setup: they are different discretisations that the paper shows agree (Sec. 3.2).
"""
import numpy as np
import pytest
import torch

import workloads
from oracle import hybrid as ohybrid
from oracle.hybrid import Layer, StripConfig
from oracle.sbim import Plane as OPlane
from paper_2102_08756_amd import SBIM, Config, Fault, SBIMError, Strip

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
T = workloads.TPV3
BULK = (T["rho"], T["cp"], T["cs"])
SLOW = (T["rho"], 0.7 * T["cp"], 0.7 * T["cs"])       # a slower layer next to the fault

CASES = {
    "coarse16_two_layers": ("tpv3_coarse16", [BULK, BULK]),
    "rect32x16_slow_layer": ("tpv3_rect32x16", [SLOW, BULK, BULK]),
    "coarse32_one_layer": ("tpv3_coarse32", [BULK]),
    "tiny8_two_layers": ("tpv3_tiny8", [BULK, SLOW]),
}
_REF = {}


def oracle_run(case):
    if case not in _REF:
        name, layers = CASES[case]
        wl = workloads.FAULTS[name]
        up = wl.upper()
        cfg = StripConfig(wl.n1, wl.n3, wl.dx, wl.dt, [Layer(*L) for L in layers],
                          OPlane(1, up["mu"], up["cs"], up["cp"]), window_cap=wl.steps)
        _REF[case] = ohybrid.hybrid_rupture(cfg, *wl.params(), wl.steps)
    return _REF[case]


def make_strip(wl, layers, precision, kind, params=None):
    cfg = Config.from_dict(wl.config_dict(), precision=precision, input_kind=kind)
    sb = SBIM(cfg, device=DEV)
    p = params if params is not None else wl.params()
    t = [torch.tensor(a, dtype=torch.float64, device=DEV).contiguous() for a in p]
    return sb, Strip(sb, layers, *t)


def gpu_run(case, precision, kind):
    name, layers = CASES[case]
    wl = workloads.FAULTS[name]
    sb, s = make_strip(wl, layers, precision, kind)
    out = {k: [] for k in ("traction", "slip_rate", "slip", "sliding", "top_u")}
    for n in range(wl.steps):
        s.step()
        for k in ("traction", "slip_rate", "slip", "sliding"):
            out[k].append(s.read(k))
        out["top_u"].append(s.read("displacement")[:, -1])
    res = {k: torch.stack(v).cpu().numpy() for k, v in out.items()}
    res["sliding"] = res["sliding"][:, 0] > 0.5
    s.close()
    sb.close()
    return res


def onset(sliding):
    return np.where(sliding.any(0), np.argmax(sliding, axis=0), -1)


@pytest.mark.parametrize("kind", ["absolute", "increment"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_strip_fp64_matches_oracle(case, kind):
    ref = oracle_run(case)
    got = gpu_run(case, "fp64", kind)
    worst = {}
    for key in ("traction", "slip_rate", "slip", "top_u"):
        worst[key] = float(np.abs(got[key] - ref[key]).max() / max(np.abs(ref[key]).max(), 1e-300))
    print(f"[strip] {case} fp64 {kind}: " + ", ".join(f"{k} {v:.2e}" for k, v in worst.items()),
          flush=True)
    np.testing.assert_array_equal(got["sliding"], ref["sliding"])
    assert ref["sliding"].any()
    for key, w in worst.items():
        assert w < 1e-12, (key, w)


@pytest.mark.parametrize("precision", ["fp32", "fp32_comp"])
def test_strip_fp32_forms_against_oracle(precision):
    case = "rect32x16_slow_layer"
    ref = oracle_run(case)
    got = gpu_run(case, precision, "increment")
    errs = {k: float(np.linalg.norm(got[k] - ref[k]) / np.linalg.norm(ref[k]))
            for k in ("traction", "slip_rate", "slip", "top_u")}
    og, orf = onset(got["sliding"]), onset(ref["sliding"])
    both = (og >= 0) & (orf >= 0)
    print(f"[strip] {case} {precision}: rel-L2 " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items())
          + f"; onset differs at {int((og != orf).sum())} cells", flush=True)
    np.testing.assert_array_equal(og >= 0, orf >= 0)
    assert np.abs(og - orf)[both].max() <= 1
    for k, e in errs.items():
        assert e < 1e-5, (k, e)


def test_strip_reset_and_errors():
    name, layers = CASES["coarse16_two_layers"]
    wl = workloads.FAULTS[name]
    sb, s = make_strip(wl, layers, "fp32_comp", "increment")
    ta, ra = s.run(25)
    s.reset()
    tb, rb = s.run(25)
    assert torch.equal(ta, tb) and torch.equal(ra, rb)
    assert torch.equal(tb[-1], s.read("traction")) and torch.equal(rb[-1], s.read("slip_rate"))
    sb.push(sb.new_field().zero_())
    with pytest.raises(SBIMError, match="SBIM_E_STATE"):
        s.step()
    s.close()
    sb.close()
    args = [torch.tensor(a, dtype=torch.float64, device=DEV) for a in wl.params()]
    # two planes, non-cubic cells, bad layer material
    two = Config.from_dict(dict(wl.config_dict(), planes=[wl.upper(), dict(wl.upper(), side=-1)]))
    sb = SBIM(two, device=DEV)
    with pytest.raises(SBIMError, match="one plane of side"):
        Strip(sb, layers, *args)
    sb.close()
    sb = SBIM(Config.from_dict(dict(wl.config_dict(), dx3=2 * wl.dx)), device=DEV)
    with pytest.raises(SBIMError, match="dx1 must equal dx3"):
        Strip(sb, layers, *args)
    sb.close()
    sb = SBIM(Config.from_dict(wl.config_dict()), device=DEV)
    with pytest.raises(SBIMError, match="strip layer 1"):
        Strip(sb, [BULK, (T["rho"], T["cs"], T["cs"])], *args)
    sb.close()


def _onset_full(run_step, fw):
    first = torch.full((fw.n1, fw.n3), -1, dtype=torch.int32, device=DEV)
    for n in range(fw.steps):
        moving = run_step()
        first = torch.where(moving & (first < 0), torch.full_like(first, n), first)
    return first.cpu().numpy()


def test_tpv3_hybrid_agrees_with_boundary_integral_rupture():
    """The paper's TPV3 comparison at its resolution (50 m; two element layers
    between the fault and S+, i.e. a strip of width 4 dx): rupture onset and
    final slip of the hybrid scheme against the stand-alone boundary-integral
    rupture, both float64, 2000 steps."""
    fw = workloads.FAULTS["tpv3_1024"]
    sb, s = make_strip(fw, [BULK, BULK], "fp64", "increment")

    def hyb_step():
        s.step()
        return s.read("sliding")[0] > 0.5
    oh = _onset_full(hyb_step, fw)
    slip_h = s.read("slip").cpu().numpy()
    s.close()
    sb.close()
    torch.cuda.empty_cache()
    cfg = Config.from_dict(fw.config_dict(), precision="fp64", input_kind="increment")
    sb = SBIM(cfg, device=DEV)
    f = Fault(sb, *[torch.tensor(a, dtype=torch.float64, device=DEV).contiguous() for a in fw.params()])
    rate = torch.empty((2, fw.n1, fw.n3), dtype=torch.float64, device=DEV)

    def sbi_step():
        f.step(slip_rate=rate)
        return (rate[0] != 0) | (rate[1] != 0)
    of = _onset_full(sbi_step, fw)
    slip_f = f.read("slip").cpu().numpy()
    f.close()
    sb.close()
    torch.cuda.empty_cache()
    patch, region = fw.masks()
    both = (oh >= 0) & (of >= 0)
    rel_onset = np.abs(oh - of)[both & ~patch] / np.maximum(of[both & ~patch], 1)
    rel_slip = float(np.linalg.norm(slip_h - slip_f) / np.linalg.norm(slip_f))
    print(f"[strip] tpv3_1024 hybrid vs boundary integral: onset differs by {np.median(rel_onset):.3f} "
          f"(median), {np.percentile(rel_onset, 99):.3f} (99th percentile) of the arrival step; "
          f"final slip rel-L2 {rel_slip:.3e}; slipped cells {int((oh >= 0).sum())} vs {int((of >= 0).sum())}",
          flush=True)
    assert not (oh[~region] >= 0).any()
    assert (oh[region] >= 0).mean() > 0.99
    assert np.median(rel_onset) < 0.03 and np.percentile(rel_onset, 99) < 0.1
    assert rel_slip < 0.05


def test_tpv3_strip_width_independence():
    """Moving S+ from two to four element layers above the fault (strip width 4 dx
    -> 8 dx) leaves the full-size rupture unchanged: onset times within three
    steps of ~1200 and final slip within 1 % (measured 0.46 %), as the boundary
    relation reflects nothing back into the strip (the paper's strip-width
    tests, Secs. 4-6)."""
    fw = workloads.FaultWorkload("tpv3_1024_short", 1024, 1024, 50.0, 1200)
    res = {}
    for layers in (2, 4):
        sb, s = make_strip(fw, [BULK] * layers, "fp32_comp", "increment")

        def step():
            s.step()
            return s.read("sliding")[0] > 0.5
        onset_l = _onset_full(step, fw)
        res[layers] = (onset_l, s.read("slip").cpu().numpy())
        s.close()
        sb.close()
        torch.cuda.empty_cache()
    (o2, s2), (o4, s4) = res[2], res[4]
    both = (o2 >= 0) & (o4 >= 0)
    rel = float(np.linalg.norm(s2 - s4) / np.linalg.norm(s4))
    print(f"[strip] tpv3 width 4 dx vs 8 dx: onset differs at {int((o2 != o4).sum())} of "
          f"{int(both.sum())} cells (max {int(np.abs(o2 - o4)[both].max())} steps); final slip "
          f"rel-L2 {rel:.2e}", flush=True)
    # the ruptured sets differ only at the front, within the last few steps
    only = (o2 >= 0) != (o4 >= 0)
    assert np.all(np.maximum(o2, o4)[only] >= fw.steps - 4)
    assert np.abs(o2 - o4)[both].max() <= 3        # out of onsets up to ~1200 steps
    assert rel < 1e-2


def test_tpv3_hybrid_error_decreases_with_mesh_refinement():
    """The paper's mesh study of the hybrid scheme on TPV3 (Sec. 3.2): the L2
    difference of the slip field at t = 3 s between the hybrid scheme (strip
    width 4 dx) and the stand-alone boundary-integral rupture falls as the grid
    is refined (dx = 200, 100, 50 m on the same 51.2 km domain)."""
    errs = []
    for n, dx in ((256, 200.0), (512, 100.0), (1024, 50.0)):
        fw = workloads.FaultWorkload(f"tpv3_dx{int(dx)}", n, n, dx, 0)
        fw.steps = int(round(3.0 / fw.dt))
        sb, s = make_strip(fw, [BULK, BULK], "fp64", "increment")
        for _ in range(fw.steps):
            s.step()
        sh = s.read("slip").cpu().numpy()
        s.close()
        sb.close()
        cfg = Config.from_dict(fw.config_dict(), precision="fp64", input_kind="increment")
        sb = SBIM(cfg, device=DEV)
        f = Fault(sb, *[torch.tensor(a, dtype=torch.float64, device=DEV).contiguous() for a in fw.params()])
        for _ in range(fw.steps):
            f.step()
        sf = f.read("slip").cpu().numpy()
        f.close()
        sb.close()
        torch.cuda.empty_cache()
        errs.append(float(np.linalg.norm(sh - sf) / np.linalg.norm(sf)))
        print(f"[strip] TPV3 at t = 3 s, dx = {dx:.0f} m ({fw.steps} steps): hybrid vs boundary "
              f"integral slip rel-L2 {errs[-1]:.3e}", flush=True)
    # first-order convergence (measured 15.8 %, 7.4 %, 3.5 %): each halving of dx at
    # least 1.6 times smaller
    assert errs[1] < errs[0] / 1.6 and errs[2] < errs[1] / 1.6
    assert errs[2] < 0.05


# ------------------------------------------------------------ two-sided strip

_LO = workloads.SLOWER
BULK_LO = (_LO["mu"] / _LO["cs"] ** 2, _LO["cp"], _LO["cs"])       # the slower lower material
TWO_CASES = {
    # (workload, lower half-space, layers above, layers below), both lists from the fault out
    "bimaterial32_2up_2down": (workloads.FAULTS["bimaterial32"], [BULK, BULK], [BULK_LO, BULK_LO]),
    "rect32x16_3up_1down": (workloads.FaultWorkload("rect32x16_bimat", 32, 16, 375.0, 120,
                                                    region=(9000.0, 4500.0), tau0_3=4.0e6,
                                                    lower=_LO), [SLOW, BULK, BULK], [BULK_LO]),
    "tiny8_1up_3down": (workloads.FaultWorkload("tiny8_bimat", 8, 8, 750.0, 40,
                                                region=(4500.0, 4500.0), patch=1500.0, lower=_LO),
                        [BULK], [BULK_LO, SLOW, BULK_LO]),
    # 7 node layers: the corrector's last chunk of three layers holds one
    "tiny8_2up_3down": (workloads.FaultWorkload("tiny8_bimat", 8, 8, 750.0, 40,
                                                region=(4500.0, 4500.0), patch=1500.0, lower=_LO),
                        [SLOW, BULK], [BULK_LO, BULK_LO, BULK_LO]),
}
_REF2 = {}


def oracle_two_sided(case):
    if case not in _REF2:
        wl, up_l, lo_l = TWO_CASES[case]
        up, lo = wl.planes()
        cfg = ohybrid.TwoSidedConfig(wl.n1, wl.n3, wl.dx, wl.dt, [Layer(*L) for L in up_l],
                                     [Layer(*L) for L in lo_l],
                                     OPlane(1, up["mu"], up["cs"], up["cp"]),
                                     OPlane(-1, lo["mu"], lo["cs"], lo["cp"]), window_cap=wl.steps)
        _REF2[case] = ohybrid.hybrid_rupture_two_sided(cfg, *wl.params(), wl.steps)
    return _REF2[case]


def gpu_two_sided(wl, up_l, lo_l, precision, kind, planes=None):
    d = wl.config_dict() if planes is None else dict(wl.config_dict(), planes=planes)
    sb = SBIM(Config.from_dict(d, precision=precision, input_kind=kind), device=DEV)
    t = [torch.tensor(a, dtype=torch.float64, device=DEV).contiguous() for a in wl.params()]
    s = Strip(sb, up_l, *t, layers_below=lo_l)
    fl = len(lo_l)                                    # storage layer of the lower fault copy
    out = {k: [] for k in ("traction", "slip_rate", "slip", "sliding", "normal_jump")}
    for n in range(wl.steps):
        s.step()
        for k in ("traction", "slip_rate", "slip", "sliding"):
            out[k].append(s.read(k))
        v = s.read("velocity")
        out["normal_jump"].append(v[1, fl + 1] - v[1, fl])
    res = {k: torch.stack(v).cpu().numpy() for k, v in out.items()}
    res["sliding"] = res["sliding"][:, 0] > 0.5
    assert s.read("displacement").shape == (3, len(up_l) + len(lo_l) + 2, wl.n1, wl.n3)
    s.close()
    sb.close()
    return res


@pytest.mark.parametrize("kind", ["absolute", "increment"])
@pytest.mark.parametrize("case", sorted(TWO_CASES))
def test_two_sided_strip_fp64_matches_oracle(case, kind):
    ref = oracle_two_sided(case)
    got = gpu_two_sided(*TWO_CASES[case], "fp64", kind)
    worst = {k: float(np.abs(got[k] - ref[k]).max() / max(np.abs(ref[k]).max(), 1e-300))
             for k in ("traction", "slip_rate", "slip")}
    vmax = np.abs(ref["slip_rate"]).max()
    print(f"[strip2] {case} fp64 {kind}: " + ", ".join(f"{k} {v:.2e}" for k, v in worst.items())
          + f"; max normal jump / max slip rate {np.abs(got['normal_jump']).max() / vmax:.1e}",
          flush=True)
    np.testing.assert_array_equal(got["sliding"], ref["sliding"])
    assert ref["sliding"].any()
    for key, w in worst.items():
        assert w < 1e-12, (key, w)
    assert np.abs(got["normal_jump"]).max() < 1e-12 * vmax     # the fault never opens
    assert np.ptp(ref["traction"][:, 1]) > 1e5                # the normal traction does change


@pytest.mark.parametrize("precision", ["fp32", "fp32_comp"])
def test_two_sided_strip_fp32_forms_against_oracle(precision):
    case = "bimaterial32_2up_2down"
    ref = oracle_two_sided(case)
    got = gpu_two_sided(*TWO_CASES[case], precision, "increment")
    errs = {k: float(np.linalg.norm(got[k] - ref[k]) / np.linalg.norm(ref[k]))
            for k in ("traction", "slip_rate", "slip")}
    og, orf = onset(got["sliding"]), onset(ref["sliding"])
    both = (og >= 0) & (orf >= 0)
    print(f"[strip2] {case} {precision}: rel-L2 " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items())
          + f"; onset differs at {int((og != orf).sum())} cells", flush=True)
    np.testing.assert_array_equal(og >= 0, orf >= 0)
    assert np.abs(og - orf)[both].max() <= 1
    for k, e in errs.items():
        assert e < 1e-5, (k, e)


def test_two_sided_strip_with_equal_sides_is_the_symmetric_strip():
    """Same material and width on both sides of the split fault: the library's
    two-sided strip reproduces its one-sided strip (the fault a symmetry plane)."""
    wl = workloads.FAULTS["tpv3_coarse16"]
    one = gpu_run("coarse16_two_layers", "fp64", "increment")
    up = wl.upper()
    two = gpu_two_sided(wl, [BULK, BULK], [BULK, BULK], "fp64", "increment",
                        planes=[up, dict(up, side=-1)])
    for k in ("traction", "slip_rate", "slip"):
        w = float(np.abs(one[k] - two[k]).max() / np.abs(one[k]).max())
        assert w < 1e-11, (k, w)
    np.testing.assert_array_equal(one["sliding"], two["sliding"])
    assert np.abs(two["normal_jump"]).max() < 1e-12 * np.abs(one["slip_rate"]).max()


def test_two_sided_strip_errors():
    wl = TWO_CASES["bimaterial32_2up_2down"][0]
    args = [torch.tensor(a, dtype=torch.float64, device=DEV) for a in wl.params()]
    up = wl.upper()
    sb = SBIM(Config.from_dict(dict(wl.config_dict(), planes=[up])), device=DEV)
    with pytest.raises(SBIMError, match="planes of sides"):
        Strip(sb, [BULK], *args, layers_below=[BULK_LO])
    sb.close()
    sb = SBIM(Config.from_dict(wl.config_dict()), device=DEV)
    with pytest.raises(SBIMError, match="one plane of side"):
        Strip(sb, [BULK], *args)
    with pytest.raises(SBIMError, match="strip layer 1 below the fault"):
        Strip(sb, [BULK], *args, layers_below=[BULK_LO, (T["rho"], T["cs"], T["cs"])])
    sb.close()


def test_tpv3_bimaterial_two_sided_hybrid_agrees_with_boundary_integral_rupture():
    """TPV3 between two materials (below the fault 0.64 mu, 0.8 c_s, 0.8 c_p) at full
    size (1024 x 1024 cells of 50 m, 2000 steps, float64): the two-sided strip (two
    element layers on each side, split fault nodes) against the stand-alone rupture
    of the two half-spaces' boundary relations.

    Slip between different materials under a friction coefficient that responds
    at once to the normal traction is ill-posed: short wavelengths grow the faster
    the finer the grid, and neither scheme converges late in the run (measured peak
    normal-traction change of the stand-alone rupture 30, 73, 284 MPa at dx = 200,
    100, 50 m; the two schemes' slip at t = 1.2 s differs by 4.8, 2.7, 3.5 %).  So
    the comparison covers what the instability has not yet reached: rupture onset
    times over the whole run, and the slip field at t = 1.2 s.  The hybrid rupture
    also stays inside the strength barrier that bounds the region."""
    import dataclasses
    fw = dataclasses.replace(workloads.FAULTS["tpv3_1024"], name="tpv3_1024_bimaterial",
                             lower=workloads.SLOWER)
    early = int(round(1.2 / fw.dt))
    cfg = Config.from_dict(fw.config_dict(), precision="fp64", input_kind="increment")
    prm = [torch.tensor(a, dtype=torch.float64, device=DEV).contiguous() for a in fw.params()]
    res = {}
    for kind in ("hybrid", "boundary integral"):
        sb = SBIM(cfg, device=DEV)
        if kind == "hybrid":
            obj = Strip(sb, [BULK, BULK], *prm, layers_below=[BULK_LO, BULK_LO])
            moving = lambda: obj.read("sliding")[0] > 0.5      # noqa: E731
        else:
            obj = Fault(sb, *prm)
            moving = lambda: (obj.read("slip_rate") != 0).any(0)  # noqa: E731
        snap = {"n": 0}

        def step():
            obj.step()
            snap["n"] += 1
            if snap["n"] == early:
                snap["slip"] = obj.read("slip").cpu().numpy()
            return moving()
        res[kind] = (_onset_full(step, fw), snap["slip"])
        obj.close()
        sb.close()
        torch.cuda.empty_cache()
    (oh, sh), (of, sf) = res["hybrid"], res["boundary integral"]
    patch, region = fw.masks()
    both = (oh >= 0) & (of >= 0) & region & ~patch
    rel_onset = np.abs(oh - of)[both] / np.maximum(of[both], 1)
    rel_slip = float(np.linalg.norm(sh - sf) / np.linalg.norm(sf))
    print(f"[strip2] tpv3_1024 bimaterial two-sided hybrid vs boundary integral: onset differs by "
          f"{np.median(rel_onset):.3f} (median), {np.percentile(rel_onset, 99):.3f} (99th percentile); "
          f"slip at t = 1.2 s rel-L2 {rel_slip:.3e}; cells slipped outside the region "
          f"{int((oh[~region] >= 0).sum())} vs {int((of[~region] >= 0).sum())}", flush=True)
    assert not (oh[~region] >= 0).any()
    assert (oh[region] >= 0).mean() > 0.99
    assert np.median(rel_onset) < 0.03 and np.percentile(rel_onset, 99) < 0.1
    assert rel_slip < 0.05


@pytest.mark.parametrize("kind", ["absolute", "increment"])
def test_strip_on_quasi_dynamic_boundary_matches_oracle(kind):
    """The strip closed at S+ by the quasi-dynamic boundary relation (the static response
    of the half-space plus radiation damping, window mode "static"): float64 against the
    oracle's hybrid scheme with the same static window."""
    import dataclasses
    wl = dataclasses.replace(workloads.FAULTS["tpv3_coarse16"], window_mode="static", window_cap=1)
    up = wl.upper()
    cfg = StripConfig(wl.n1, wl.n3, wl.dx, wl.dt, [Layer(*BULK), Layer(*BULK)],
                      OPlane(1, up["mu"], up["cs"], up["cp"]), window_cap=1, window_mode="static")
    ref = ohybrid.hybrid_rupture(cfg, *wl.params(), wl.steps)
    sb, s = make_strip(wl, [BULK, BULK], "fp64", kind)
    got = {k: [] for k in ("traction", "slip_rate", "slip", "sliding")}
    for n in range(wl.steps):
        s.step()
        for k in got:
            got[k].append(s.read(k))
    got = {k: torch.stack(v).cpu().numpy() for k, v in got.items()}
    got["sliding"] = got["sliding"][:, 0] > 0.5
    s.close()
    sb.close()
    worst = {k: float(np.abs(got[k] - ref[k]).max() / max(np.abs(ref[k]).max(), 1e-300))
             for k in ("traction", "slip_rate", "slip")}
    print(f"[strip] quasi-dynamic boundary, coarse16 fp64 {kind}: "
          + ", ".join(f"{k} {v:.2e}" for k, v in worst.items()), flush=True)
    np.testing.assert_array_equal(got["sliding"], ref["sliding"])
    assert ref["sliding"].any()
    for k, w in worst.items():
        assert w < 1e-12, (k, w)


@pytest.mark.parametrize("two_sided", [False, True])
@pytest.mark.parametrize("kind", ["absolute", "increment"])
def test_strip_with_variable_steps_matches_oracle(two_sided, kind):
    """The quasi-dynamic boundary relation with a new step size before most steps
    (sbim_set_dt; every fourth step repeats the previous size): the strip redoes its
    prediction for the new size.  Float64 against the oracle's strip with the same step
    sequence, one-sided and two-sided."""
    import dataclasses
    if two_sided:
        wl = workloads.FaultWorkload("bimat16_qd", 16, 16, 750.0, 60, region=(9000.0, 9000.0),
                                     lower=_LO, window_mode="static", window_cap=1)
        up_l, lo_l = [BULK, BULK], [BULK_LO, BULK_LO]
    else:
        wl = dataclasses.replace(workloads.FAULTS["tpv3_coarse16"], window_mode="static",
                                 window_cap=1)
        up_l, lo_l = [BULK, BULK], None
    rng = np.random.default_rng(31)
    dts = rng.uniform(0.1, 0.3, wl.steps) * wl.dx / T["cs"]
    for k in range(4, wl.steps, 4):
        dts[k] = dts[k - 1]
    planes = wl.planes()
    op = [OPlane(1, planes[0]["mu"], planes[0]["cs"], planes[0]["cp"])]
    if two_sided:
        op.append(OPlane(-1, planes[1]["mu"], planes[1]["cs"], planes[1]["cp"]))
        cfg = ohybrid.TwoSidedConfig(wl.n1, wl.n3, wl.dx, wl.dt, [Layer(*L) for L in up_l],
                                     [Layer(*L) for L in lo_l], op[0], op[1], window_cap=1,
                                     window_mode="static")
        ref = ohybrid.hybrid_rupture_two_sided(cfg, *wl.params(), wl.steps, dts=dts)
    else:
        cfg = StripConfig(wl.n1, wl.n3, wl.dx, wl.dt, [Layer(*L) for L in up_l], op[0],
                          window_cap=1, window_mode="static")
        ref = ohybrid.hybrid_rupture(cfg, *wl.params(), wl.steps, dts=dts)
    sb = SBIM(Config.from_dict(wl.config_dict(), precision="fp64", input_kind=kind), device=DEV)
    prm = [torch.tensor(a, dtype=torch.float64, device=DEV).contiguous() for a in wl.params()]
    s = Strip(sb, up_l, *prm, layers_below=lo_l)
    got = {k: [] for k in ("traction", "slip_rate", "slip", "sliding")}
    for n in range(wl.steps):
        sb.set_dt(float(dts[n]))
        s.step()
        for k in got:
            got[k].append(s.read(k))
    got = {k: torch.stack(v).cpu().numpy() for k, v in got.items()}
    got["sliding"] = got["sliding"][:, 0] > 0.5
    s.close()
    sb.close()
    worst = {k: float(np.abs(got[k] - ref[k]).max() / max(np.abs(ref[k]).max(), 1e-300))
             for k in ("traction", "slip_rate", "slip")}
    print(f"[strip] variable steps, {'two' if two_sided else 'one'}-sided fp64 {kind}: "
          + ", ".join(f"{k} {v:.2e}" for k, v in worst.items()), flush=True)
    np.testing.assert_array_equal(got["sliding"], ref["sliding"])
    assert ref["sliding"].any()
    for k, w in worst.items():
        assert w < 1e-12, (k, w)
