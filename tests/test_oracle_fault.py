"""Pins of the oracle's frictional fault (``oracle.fault``).

Each pin is fixed by something other than the oracle's own formulas:
  * a spatially uniform fault (only the k = 0 mode): each side radiates a
    plane shear wave, so slip follows a closed-form geometric sequence under
    linear slip-weakening, then grows linearly at the kinetic level; with two
    different materials the side velocities split in the inverse ratio of
    the impedances;
  * a fault loaded below its strength everywhere never moves;
  * static limits of elasticity: a frictionless fault under a sinusoidal shear
    load settles (on time average) at the slip that cancels the load, which is
    2 A / (mu q) antiplane and 2 (1 - nu) A / (mu q) in-plane for equal
    materials (Boussinesq-Cerruti surface compliance of a half-space), and the
    solution of the two half-spaces' static 2x2 stiffnesses for a bimaterial;
  * two identical planes (+1, -1) give the same rupture as one plane with its
    mirror image;
  * causality: no cell slips before a P wave from the nucleation patch could
    reach it, and the locked cells never slip;
  * the workload constants are the ones the paper prints (``tests/golden``).
"""
import json
import math
import os

import numpy as np
import pytest

import workloads
from oracle import fault
from oracle.sbim import Config, Plane

HERE = os.path.dirname(os.path.abspath(__file__))


def _uniform_params(n, tau_sh, sigma, mu_s, mu_k, d_c, tau_3=0.0):
    tau0 = np.zeros((3, n, n))
    tau0[0], tau0[1], tau0[2] = tau_sh, -sigma, tau_3
    full = lambda v: np.full((n, n), float(v))  # noqa: E731
    return fault.FaultParams(tau0, full(mu_s), full(mu_k), full(d_c))


@pytest.mark.parametrize("lower", [None, Plane(-1, 0.6, 0.8, 0.8 * math.sqrt(3.0))])
def test_uniform_fault_closed_form(lower):
    """k = 0 only: V = (|tau0| - S(delta)) (1/Z+ + 1/Z-), Z = mu / c_s, so with
    S linear in the slip amplitude delta, delta^n = (A/B)((1 + B dt)^n - 1) until
    it passes d_c, then it grows by dt V_k per step."""
    planes = [Plane()] if lower is None else [Plane(), lower]
    dt, n, steps = 0.2, 4, 60
    cfg = Config(n1=n, n3=n, dt=dt, planes=planes, window_cap=steps)
    t1, t3, sigma, mu_s, mu_k, d_c = 0.65, 0.2, 1.0, 0.6, 0.5, 0.5
    out = fault.rupture(cfg, _uniform_params(n, t1, sigma, mu_s, mu_k, d_c, t3), steps)
    zp = 1.0
    zm = 1.0 if lower is None else lower.mu / lower.cs
    cz = 1.0 / zp + 1.0 / zm
    tmag = math.hypot(t1, t3)
    A = (tmag - sigma * mu_s) * cz
    B = sigma * (mu_s - mu_k) / d_c * cz
    delta = (A / B) * ((1 + B * dt) ** np.arange(steps, dtype=np.float64) - 1)   # delta^n, closed form
    k_star = int(np.argmax(delta >= d_c))     # first step that starts at or past d_c
    Vk = (tmag - sigma * mu_k) * cz
    expect = np.where(np.arange(steps) < k_star, delta, delta[k_star] + (np.arange(steps) - k_star) * dt * Vk)
    # the slip after step m is delta^{m+1}
    amp = np.hypot(out["slip"][:, 0], out["slip"][:, 1])
    got = amp[:, 0, 0]
    np.testing.assert_allclose(got[:k_star], expect[1:k_star + 1], rtol=1e-12)
    np.testing.assert_allclose(got[k_star:], expect[k_star] + np.arange(1, steps - k_star + 1) * dt * Vk,
                               rtol=1e-12)
    assert np.ptp(amp[-1]) <= 1e-13 * amp[-1].max()                 # stays uniform
    # slip along the background shear, side velocities split by impedance
    V = out["slip_rate"][:, :, 0, 0]
    np.testing.assert_allclose(V[:, 1] * t1, V[:, 0] * t3, atol=1e-15)
    tau_sh = out["traction"][:, [0, 2], 0, 0]
    drop = np.array([t1, t3])[None] - tau_sh                     # = V / cz
    np.testing.assert_allclose(out["v_plus"][:, [0, 2], 0, 0], drop / zp, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(out["v_minus"][:, [0, 2], 0, 0], -drop / zm, rtol=1e-12, atol=1e-15)
    assert 2 < k_star < steps - 10
    np.testing.assert_allclose(out["traction"][:, 1], -sigma, rtol=1e-14)
    assert np.abs(out["v_plus"][:, 1]).max() < 1e-14


def test_fault_below_strength_never_moves():
    rng = np.random.default_rng(3)
    n = 8
    cfg = Config(n1=n, n3=n, dt=0.2, planes=[Plane(), Plane(-1, 2.0, 1.3, 2.4)], window_cap=20)
    tau0 = np.zeros((3, n, n))
    tau0[0] = rng.uniform(-0.3, 0.3, (n, n))
    tau0[2] = rng.uniform(-0.3, 0.3, (n, n))
    tau0[1] = -1.0 - rng.uniform(0, 0.5, (n, n))
    prm = fault.FaultParams(tau0, np.full((n, n), 0.5), np.full((n, n), 0.1), np.full((n, n), 1.0))
    out = fault.rupture(cfg, prm, 20)
    assert np.abs(out["slip_rate"]).max() == 0.0
    # the impedance-weighted means of equal numbers round to within an ulp
    assert np.abs(out["v_plus"]).max() < 1e-15 and np.abs(out["v_minus"]).max() < 1e-15
    assert np.abs(out["slip"]).max() == 0.0
    np.testing.assert_allclose(out["traction"][-1], tau0, rtol=1e-14)


def _sinusoid_static(comp, planes, steps=500, n1=4, n3=4, avg=250):
    cfg = Config(n1=n1, n3=n3, dt=0.2, planes=planes, window_cap=steps)
    k = 2 * np.pi / n1
    A = 1e-3
    tau0 = np.zeros((3, n1, n3))
    tau0[1] = -1.0
    tau0[comp] = A * np.cos(k * np.arange(n1))[:, None]
    z = np.zeros((n1, n3))
    out = fault.rupture(cfg, fault.FaultParams(tau0, z, z, z + 1.0), steps)
    D = out["slip"][:, 0 if comp == 0 else 1, :, 0]                 # [N, n1]
    amp = (D * np.cos(k * np.arange(n1))).sum(-1) * 2 / n1
    return amp[-avg:].mean(), A, k, out


def test_static_limit_antiplane():
    """Slip along x3 varying along x1: the traction of slip D cos(k x1) on an
    antiplane fault is -mu k D / 2, so the load A is cancelled at D = 2A/(mu k)."""
    mean, A, k, _ = _sinusoid_static(2, [Plane()])
    assert abs(mean / (2 * A / k) - 1) < 0.02


def test_static_limit_inplane():
    """Slip along x1 varying along x1: with the normal traction unchanged the
    half-space compliance is (1 - nu)/(mu k); nu = 1/4 for c_p/c_s = sqrt 3."""
    nu = 0.25
    mean, A, k, _ = _sinusoid_static(0, [Plane()])
    assert abs(mean / (2 * (1 - nu) * A / k) - 1) < 0.02
    mean2, _, _, _ = _sinusoid_static(0, [Plane(), Plane(-1)])
    assert abs(mean2 - mean) < 1e-12 * abs(mean)


def test_static_limit_bimaterial():
    """Frictionless in-plane slip between two different half-spaces.  Static
    surface stiffness of a half-space (Boussinesq-Cerruti, wavevector frame,
    upper side): tau_L = -mu q [K11 u_L + i K12 u_N], tau_N = -mu q [K22 u_N -
    i K12 u_L] with K11 = K22 = 2 eta^2/(eta^2 + 1), K12 = -2/(eta^2 + 1); the
    lower side is its mirror image.  Zero shear traction change on both sides,
    equal normal traction change and a common normal displacement fix the slip."""
    lower = Plane(-1, 0.5, 0.8, 0.8 * 1.9)
    planes = [Plane(), lower]
    mean, A, k, out = _sinusoid_static(0, planes, steps=700, avg=400)

    def K(pl):
        e2 = (pl.cp / pl.cs) ** 2
        return 2 * e2 / (e2 + 1), -2 / (e2 + 1)
    K11p, K12p = K(planes[0])
    K11m, K12m = K(lower)
    mp, mm = planes[0].mu * k, lower.mu * k
    # unknowns (a = u_L+, b = u_L-, w = u_N); load A on the L component
    M = np.array([[-mp * K11p, 0, -1j * mp * K12p],
                  [0, mm * K11m, -1j * mm * K12m],
                  [1j * mp * K12p, -1j * mm * K12m, -mp * K11p - mm * K11m]], dtype=complex)
    rhs = np.array([-A, -A, 0], dtype=complex)
    a, b, w = np.linalg.solve(M, rhs)
    expect = (a - b).real
    assert abs(mean / expect - 1) < 0.02
    # the normal velocities of the two sides agree at every step (no opening)
    np.testing.assert_allclose(out["v_plus"][:, 1], out["v_minus"][:, 1], rtol=0,
                               atol=1e-12 * np.abs(out["v_plus"]).max())


def test_mirror_plane_equals_two_identical_planes():
    wl = workloads.FAULTS["tpv3_coarse16"]
    tau0, mu_s, mu_k, d_c = wl.params()
    prm = fault.FaultParams(tau0, mu_s, mu_k, d_c)
    cfg1 = wl.config_dict()
    cfg2 = dict(cfg1, planes=cfg1["planes"] + [dict(cfg1["planes"][0], side=-1)])
    a = fault.rupture(Config.from_dict(cfg1), prm, 40)
    b = fault.rupture(Config.from_dict(cfg2), prm, 40)
    for key in a:
        scale = max(np.abs(a[key]).max(), 1e-300)
        assert np.abs(a[key] - b[key]).max() <= 1e-12 * scale, key
    assert np.abs(a["slip_rate"]).max() > 0


def test_nucleated_rupture_causal_and_confined():
    wl = workloads.FAULTS["tpv3_coarse16"]
    tau0, mu_s, mu_k, d_c = wl.params()
    out = fault.rupture(Config.from_dict(wl.config_dict()), fault.FaultParams(tau0, mu_s, mu_k, d_c),
                        wl.steps)
    patch, region = wl.masks()
    V = np.sqrt((out["slip_rate"] ** 2).sum(1))                   # [N, n1, n3]
    slipping = V > 0
    assert slipping[0][patch].all() and not slipping[0][~patch].any()
    assert not slipping[:, ~region].any()                         # locked cells stay locked
    ever = slipping.any(0)
    assert ever[region & ~patch].sum() > 0.5 * (region & ~patch).sum()   # the rupture spreads
    X1, X3 = wl.coords()
    h = wl.patch / 2
    dist = np.hypot(np.maximum(np.abs(X1) - h, 0), np.maximum(np.abs(X3) - h, 0))
    first = np.argmax(slipping, axis=0)
    cp = workloads.TPV3["cp"]
    t_first = first * wl.dt
    assert np.all(dist[ever] <= cp * (t_first[ever] + wl.dt) + 1e-9)
    np.testing.assert_array_equal(out["traction"][:, 1], np.broadcast_to(tau0[1], out["traction"][:, 1].shape))
    # the shear traction never exceeds the strength of the step
    tau_sh = np.hypot(out["traction"][:, 0], out["traction"][:, 2])
    amp = np.hypot(out["slip"][:, 0], out["slip"][:, 1])
    delta_before = np.concatenate([np.zeros((1,) + mu_s.shape), amp[:-1]])
    mu = np.where(delta_before < d_c, mu_s - (mu_s - mu_k) * delta_before / d_c, mu_k)
    assert np.all(tau_sh <= -tau0[1] * mu * (1 + 1e-12))


def test_fault_workload_constants_are_the_papers():
    with open(os.path.join(HERE, "golden", "tpv3_fault.json")) as f:
        g = json.load(f)
    with open(os.path.join(HERE, "golden", "tpv3_material.json")) as f:
        m = json.load(f)
    t = workloads.TPV3
    assert (t["mu_s"], t["mu_k"], t["d_c"]) == (g["mu_s"], g["mu_k"], g["d_c_m"])
    assert (t["tau0"], t["sigma0"]) == (g["tau0_shear_pa"], g["sigma0_normal_pa"])
    assert t["patch"] == g["nucleation_patch_m"] and list(t["region"]) == g["rupture_region_m"]
    assert (t["rho"], t["cp"], t["cs"], t["dx"]) == (m["rho_kg_m3"], m["cp_m_s"], m["cs_m_s"], m["dx_m"])
    wl = workloads.FAULTS["tpv3_1024"]
    patch, region = wl.masks()
    assert patch.sum() == (3000 // 50) ** 2 and region.sum() == (30000 // 50) * (15000 // 50)


def test_fault_impedances_are_the_boundary_relations_damping():
    """The interface solve's Z must be the damping coefficient of each side's
    boundary relation: adding a velocity v to a side's push changes its traction
    by -Z v (upper side) or +Z v (lower side), component by component.  That
    damping is itself pinned by the plane-wave (k = 0) test of the pipeline."""
    from oracle.sbim import PlaneOperator
    planes = [Plane(1, 1.3, 0.9, 1.7), Plane(-1, 0.6, 0.8, 1.5)]
    cfg = Config(n1=8, n3=8, dt=0.2, planes=planes, window_cap=3)
    zp, zm = fault.impedances(cfg)
    rng = np.random.default_rng(11)
    U = rng.standard_normal((2, 3, 8 * 5)) + 1j * rng.standard_normal((2, 3, 8 * 5))
    V = rng.standard_normal((3, 8 * 5)) + 1j * rng.standard_normal((3, 8 * 5))
    for p, (z, sign) in enumerate(((zp, -1.0), (zm, 1.0))):
        op = PlaneOperator(cfg, p)
        with_v = op.apply_last(U, V)
        without = op.apply_last(U, np.zeros_like(V))
        np.testing.assert_allclose(with_v - without, sign * z[:, None] * V, rtol=1e-13, atol=1e-13)
