"""GPU parity of the quasi-dynamic boundary relation (window mode "static") against the oracle.

The library keeps one history slot per mode and uses the kernels' static
integrals; the oracle applies the same limit through its own kernel
functions.  Bars as for the dynamic relation (float64 1e-12, float32 forms
1e-5 relative L2 over all steps), with per-step time steps set through
``sbim_set_dt``; the quasi-dynamic fault with variable time steps against the
oracle's rupture at 1e-12 of each field's largest value (float64) or 1e-5
relative L2 (compensated float32).
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
from oracle import fault as ofault
from paper_2102_08756_amd import SBIM, Config, Fault, SBIMError

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = {"fp64": 1e-12, "fp32": 1e-5, "fp32_comp": 1e-5}

CFG = dict(n1=16, n3=32, dx1=0.8, dx3=1.1, dt=0.2, window_mode="static", window_cap=7,
           planes=[dict(side=1), dict(side=-1, mu=1.7, cs=0.9, cp=2.0)])


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32_comp"])
@pytest.mark.parametrize("kind", ["absolute", "increment"])
def test_static_relation_matches_oracle_with_variable_steps(precision, kind):
    rng = np.random.default_rng(31)
    N = 9
    P = len(CFG["planes"])
    shape = (N, P, 3, CFG["n1"], CFG["n3"])
    u = rng.standard_normal(shape)
    dts = rng.uniform(0.05, 0.5, N)
    # the velocity the library forms without a pushed one, per step
    if kind == "absolute":
        prev = np.concatenate([np.zeros_like(u[:1]), u[:-1]])
        v = (u - prev) / dts[:, None, None, None, None]
    else:
        v = u / dts[:, None, None, None, None]
    cfg_d = dict(CFG, input_kind=kind)
    ref = oracle.forward(cfg_d, u, v)
    sb = SBIM(Config.from_dict(cfg_d, precision=precision), device=DEV)
    ut = torch.tensor(u, dtype=sb.dtype, device=DEV)
    got = np.empty_like(ref)
    for n in range(N):
        sb.set_dt(dts[n])
        sb.push(ut[n])
        got[n] = sb.tractions().double().cpu().numpy()
    assert sb.info()["ring_bytes"] > 0
    sb.close()
    err = rel_l2(got, ref)
    print(f"[static] {precision} {kind}: rel-L2 {err:.2e}", flush=True)
    assert err < TOL[precision]


def test_set_dt_only_for_static_handles():
    sb = SBIM(Config.from_dict(dict(CFG, window_mode="fixed")), device=DEV)
    with pytest.raises(SBIMError, match="SBIM_E_STATE"):
        sb.set_dt(0.1)
    sb.close()
    sb = SBIM(Config.from_dict(CFG), device=DEV)
    with pytest.raises(SBIMError, match="SBIM_E_INVALID"):
        sb.set_dt(-1.0)
    sb.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_comp"])
def test_quasi_dynamic_fault_with_variable_steps(precision):
    wl = workloads.FAULTS["tpv3_coarse32"]
    steps = 120
    rng = np.random.default_rng(5)
    dts = wl.dt * rng.uniform(0.5, 2.0, steps)
    cfg_d = dict(wl.config_dict(), window_mode="static")
    prm = wl.params()
    ref = ofault.rupture(oracle.Config.from_dict(dict(cfg_d, input_kind="absolute")),
                         ofault.FaultParams(*prm), steps, dts=dts)
    sb = SBIM(Config.from_dict(cfg_d, precision=precision, input_kind="increment"), device=DEV)
    f = Fault(sb, *[torch.tensor(a, device=DEV).contiguous() for a in prm])
    tau = torch.empty((steps, 3, wl.n1, wl.n3), dtype=torch.float64, device=DEV)
    rate = torch.empty((steps, 2, wl.n1, wl.n3), dtype=torch.float64, device=DEV)
    for n in range(steps):
        sb.set_dt(dts[n])
        f.step(tau[n], rate[n])
    slip = f.read("slip").cpu().numpy()
    f.close()
    sb.close()
    tau, rate = tau.cpu().numpy(), rate.cpu().numpy()
    if precision == "fp64":      # largest deviation over the field's largest value
        err = lambda a, b: np.abs(a - b).max() / np.abs(b).max()  # noqa: E731
    else:                        # relative L2, as for the dynamic float32 forms
        err = rel_l2
    e_tau, e_rate, e_slip = err(tau, ref["traction"]), err(rate, ref["slip_rate"]), err(slip, ref["slip"][-1])
    print(f"[static] fault {precision}: traction {e_tau:.2e}, slip rate {e_rate:.2e}, slip {e_slip:.2e}",
          flush=True)
    assert (ref["slip_rate"] > 0).any()
    bar = 1e-12 if precision == "fp64" else 1e-5
    np.testing.assert_array_equal(rate > 0, ref["slip_rate"] > 0)
    assert e_tau < bar and e_rate < bar and e_slip < bar
