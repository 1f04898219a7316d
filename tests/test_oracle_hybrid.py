"""Pins of the oracle's hybrid finite-element / boundary-integral rupture (``oracle.hybrid``).

Fixed by facts outside the oracle's own formulas:
  * the hexahedral element stiffness is symmetric, has exactly the six rigid-
    body motions as null space, and passes the patch test: a uniform strain
    gives the face forces sigma . n h^2 of linear elasticity (Eq. linelasticity);
  * in the periodic strip a displacement linear in x2 loads only the two
    boundary layers, with the stress times the node area;
  * a spatially uniform fault (k = 0) settles at the slip rate of a plane shear
    wave leaving each side, 2 (tau0 - tau_k) c_s / mu, once the strip's
    transients have passed through S+ (the boundary relation absorbs them);
  * a fault below strength everywhere never moves;
  * moving the S+ boundary away from the fault (two versus four element
    layers) leaves the rupture unchanged to within a few percent (the paper's
    strip-width independence test, Secs. 4-6);
  * with mesh refinement the hybrid rupture approaches the stand-alone
    boundary-integral rupture on the same grid (Sec. 3.2: TPV3 agreement,
    error decreasing with the mesh size).
"""
import numpy as np
import pytest

import workloads
from oracle import fault, hybrid
from oracle.hybrid import CORNERS, Layer, StripConfig, hex8_stiffness
from oracle.sbim import Config, Plane

T = workloads.TPV3
RHO, CP, CS = T["rho"], T["cp"], T["cs"]
MU = RHO * CS * CS


def test_hex8_stiffness_symmetry_and_rigid_modes():
    h, lam, mu = 2.0, 1.3, 0.7
    K = hex8_stiffness(h, lam, mu)
    assert np.abs(K - K.T).max() < 1e-14 * np.abs(K).max()
    w = np.linalg.eigvalsh(K)
    assert np.all(np.abs(w[:6]) < 1e-12 * w[-1]) and w[6] > 1e-3 * w[-1]
    X = CORNERS * h
    rigid = []
    for c in range(3):
        t = np.zeros((8, 3))
        t[:, c] = 1.0
        rigid.append(t)
    for a, b in ((0, 1), (1, 2), (0, 2)):
        r = np.zeros((8, 3))
        r[:, a], r[:, b] = -X[:, b], X[:, a]
        rigid.append(r)
    for r in rigid:
        assert np.abs(K @ r.ravel()).max() < 1e-13 * np.abs(K).max()


@pytest.mark.parametrize("grad", [(0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (0, 2)])
def test_hex8_patch_test(grad):
    """u_i = x_j (one displacement gradient entry): nodal forces summed over each
    face equal sigma . n h^2 with sigma from Eq. linelasticity."""
    h, lam, mu = 1.5, 0.8, 1.1
    i, j = grad
    K = hex8_stiffness(h, lam, mu)
    X = CORNERS * h
    u = np.zeros((8, 3))
    u[:, i] = X[:, j]
    f = (K @ u.ravel()).reshape(8, 3)
    G = np.zeros((3, 3))
    G[i, j] = 1.0
    eps = 0.5 * (G + G.T)
    sigma = lam * np.trace(eps) * np.eye(3) + 2 * mu * eps
    # each corner collects a quarter of the traction sigma . n h^2 of each of its
    # three faces (a uniform stress has a bilinear-exact consistent load)
    expect = np.zeros((8, 3))
    for a in range(8):
        for axis in range(3):
            n = np.zeros(3)
            n[axis] = 1.0 if CORNERS[a, axis] else -1.0
            expect[a] += sigma @ n * h * h / 4.0
    np.testing.assert_allclose(f, expect, rtol=1e-12, atol=1e-12 * np.abs(expect).max())


def test_strip_linear_field_loads_only_boundary_layers():
    cfg = StripConfig(4, 8, 2.0, 0.1, [Layer(1.0, 2.0, 1.1)] * 3, Plane())
    strip = hybrid.Strip(cfg)
    L = cfg.layers[0]
    eps = 1e-3
    u = np.zeros(strip.shape)
    x2 = np.arange(cfg.n2 + 1) * cfg.h
    u[0] = eps * x2[:, None, None]                   # u1 = eps x2: shear strain eps/2
    f = strip.internal_force(u)
    sigma12 = L.mu * eps
    A = cfg.h ** 2
    np.testing.assert_allclose(f[0, 0], -sigma12 * A, rtol=1e-12)
    np.testing.assert_allclose(f[0, -1], sigma12 * A, rtol=1e-12)
    assert np.abs(f[0, 1:-1]).max() < 1e-12 * sigma12 * A
    assert np.abs(f[1:]).max() < 1e-12 * sigma12 * A


def _uniform(n, t1, mus, muk, dc=0.4):
    tau0 = np.zeros((3, n, n))
    tau0[0], tau0[1] = t1, -120e6
    full = lambda x: np.full((n, n), float(x))  # noqa: E731
    return tau0, full(mus), full(muk), full(dc)


@pytest.mark.parametrize("n2", [1, 2])
def test_uniform_fault_reaches_plane_wave_slip_rate(n2):
    n, h = 4, 375.0
    dt = 0.25 * h / CS
    cfg = StripConfig(n, n, h, dt, [Layer(RHO, CP, CS)] * n2, Plane(1, MU, CS, CP), window_cap=4)
    tau0, mus, muk, dc = _uniform(n, 80e6, 0.6, 0.6)
    out = hybrid.hybrid_rupture(cfg, tau0, mus, muk, dc, 400)
    V = out["slip_rate"][:, 0]
    expect = 2 * (80e6 - 0.6 * 120e6) * CS / MU
    assert np.abs(V[-50:] / expect - 1).max() < 2e-3
    assert out["sliding"][-50:].all()
    assert np.abs(out["slip_rate"][:, 1]).max() < 1e-9 * expect


def test_fault_below_strength_never_moves():
    n, h = 8, 375.0
    cfg = StripConfig(n, n, h, 0.25 * h / CS, [Layer(RHO, CP, CS)] * 2, Plane(1, MU, CS, CP),
                      window_cap=10)
    rng = np.random.default_rng(5)
    tau0, mus, muk, dc = _uniform(n, 0.0, 0.6, 0.5)
    tau0[0] = rng.uniform(-50e6, 50e6, (n, n))
    out = hybrid.hybrid_rupture(cfg, tau0, mus, muk, dc, 20)
    assert not out["sliding"].any()
    assert np.abs(out["slip_rate"]).max() == 0.0 and np.abs(out["top_u"]).max() == 0.0
    np.testing.assert_array_equal(out["traction"][-1], tau0)


def _strip_for(wl, n2):
    return StripConfig(wl.n1, wl.n3, wl.dx, wl.dt, [Layer(RHO, CP, CS)] * n2, Plane(1, MU, CS, CP),
                       window_cap=wl.steps)


def _onset(sliding):
    return np.where(sliding.any(0), np.argmax(sliding, axis=0), -1)


def test_strip_width_independence():
    wl = workloads.FAULTS["tpv3_coarse16"]
    prm = wl.params()
    a = hybrid.hybrid_rupture(_strip_for(wl, 2), *prm, wl.steps)
    b = hybrid.hybrid_rupture(_strip_for(wl, 4), *prm, wl.steps)
    oa, ob = _onset(a["sliding"]), _onset(b["sliding"])
    np.testing.assert_array_equal(oa >= 0, ob >= 0)
    assert np.abs(oa - ob).max() <= 1                  # rupture onset within one step
    rel = np.linalg.norm(a["slip"][-1] - b["slip"][-1]) / np.linalg.norm(b["slip"][-1])
    assert rel < 0.03
    patch, region = wl.masks()
    assert (_onset(a["sliding"])[region & ~patch] > 0).mean() > 0.5


def test_hybrid_converges_to_boundary_integral_rupture():
    errs = []
    for n in (16, 32):
        dx = 12000.0 / n
        wl = workloads.FaultWorkload(f"conv{n}", n, n, dx, int(round(72 * 750 / dx)),
                                     region=(9000.0, 9000.0))
        prm = wl.params()
        ref = fault.rupture(Config.from_dict(dict(wl.config_dict(), input_kind="absolute")),
                            fault.FaultParams(*prm), wl.steps)
        hyb = hybrid.hybrid_rupture(_strip_for(wl, 2), *prm, wl.steps)
        errs.append(np.linalg.norm(hyb["slip"][-1] - ref["slip"][-1]) / np.linalg.norm(ref["slip"][-1]))
        # no slip outside the rupture region, the same locked cells
        patch, region = wl.masks()
        assert not hyb["sliding"][:, ~region].any()
    assert errs[1] < 0.5 * errs[0] and errs[1] < 0.15, errs


# ---------------------------------------------------------------- two-sided strip

def _two_sided_materials():
    lo = workloads.SLOWER
    Bu = Layer(RHO, CP, CS)
    Bl = Layer(lo["mu"] / lo["cs"] ** 2, lo["cp"], lo["cs"])
    return Bu, Bl, Plane(1, MU, CS, CP), Plane(-1, lo["mu"], lo["cs"], lo["cp"])


def test_two_sided_strip_with_equal_sides_is_the_symmetric_strip():
    """Equal materials and widths on both sides: the split-node scheme must
    reproduce the one-sided scheme that models the fault as a symmetry plane."""
    from oracle.hybrid import TwoSidedConfig
    wl = workloads.FAULTS["tpv3_coarse16"]
    Bu = Layer(RHO, CP, CS)
    a = hybrid.hybrid_rupture(_strip_for(wl, 2), *wl.params(), wl.steps)
    b = hybrid.hybrid_rupture_two_sided(
        TwoSidedConfig(wl.n1, wl.n3, wl.dx, wl.dt, [Bu] * 2, [Bu] * 2, Plane(1, MU, CS, CP),
                       Plane(-1, MU, CS, CP), window_cap=wl.steps), *wl.params(), wl.steps)
    for k in ("traction", "slip_rate", "slip"):
        assert np.abs(a[k] - b[k]).max() < 1e-12 * np.abs(a[k]).max(), k
    np.testing.assert_array_equal(a["sliding"], b["sliding"])
    assert np.abs(b["normal_jump"]).max() < 1e-12


def test_two_sided_uniform_bimaterial_fault_reaches_plane_wave_slip_rate():
    """k = 0 between two materials: each side radiates its own plane shear wave,
    V = (tau0 - tau_k)(c_s+/mu+ + c_s-/mu-), and the normal traction stays put."""
    from oracle.hybrid import TwoSidedConfig
    Bu, Bl, Pu, Pl = _two_sided_materials()
    n, h = 4, 375.0
    cfg = TwoSidedConfig(n, n, h, 0.25 * h / CS, [Bu] * 2, [Bl] * 2, Pu, Pl, window_cap=4)
    tau0, mus, muk, dc = _uniform(n, 80e6, 0.6, 0.6)
    out = hybrid.hybrid_rupture_two_sided(cfg, tau0, mus, muk, dc, 500)
    expect = (80e6 - 0.6 * 120e6) * (CS / MU + Pl.cs / Pl.mu)
    assert np.abs(out["slip_rate"][-50:, 0] / expect - 1).max() < 2e-3
    np.testing.assert_allclose(out["traction"][:, 1], -120e6, rtol=1e-9)


def test_two_sided_hybrid_converges_to_bimaterial_boundary_integral_rupture():
    """Different materials across the fault (the lower one slower): with mesh
    refinement the hybrid rupture approaches the stand-alone two-plane rupture, and
    the fault never opens (equal normal velocities of the two copies)."""
    from oracle.hybrid import TwoSidedConfig
    Bu, Bl, Pu, Pl = _two_sided_materials()
    errs = []
    for n in (16, 32):
        dx = 12000.0 / n
        wl = workloads.FaultWorkload(f"bimat{n}", n, n, dx, int(round(72 * 750 / dx)),
                                     region=(9000.0, 9000.0), lower=workloads.SLOWER)
        prm = wl.params()
        ref = fault.rupture(Config.from_dict(dict(wl.config_dict(), input_kind="absolute")),
                            fault.FaultParams(*prm), wl.steps)
        hyb = hybrid.hybrid_rupture_two_sided(
            TwoSidedConfig(n, n, dx, wl.dt, [Bu] * 2, [Bl] * 2, Pu, Pl, window_cap=wl.steps),
            *prm, wl.steps)
        errs.append(np.linalg.norm(hyb["slip"][-1] - ref["slip"][-1]) / np.linalg.norm(ref["slip"][-1]))
        v = np.abs(hyb["slip_rate"]).max()
        assert np.abs(hyb["normal_jump"]).max() < 1e-9 * v
        assert np.ptp(hyb["traction"][:, 1]) > 1e6          # the bimaterial normal-stress change
    assert errs[1] < 0.5 * errs[0] and errs[1] < 0.15, errs


# ------------------------------------------------- variable time steps (quasi-dynamic)

def test_constant_step_sizes_reproduce_the_fixed_step_run():
    from oracle.hybrid import TwoSidedConfig
    wl = workloads.FAULTS["tpv3_tiny8"]
    one = StripConfig(wl.n1, wl.n3, wl.dx, wl.dt, [Layer(RHO, CP, CS)] * 2, Plane(1, MU, CS, CP),
                      window_cap=1, window_mode="static")
    a = hybrid.hybrid_rupture(one, *wl.params(), 30)
    b = hybrid.hybrid_rupture(one, *wl.params(), 30, dts=[wl.dt] * 30)
    for k in a:
        np.testing.assert_array_equal(a[k], b[k])
    Bu, Bl, Pu, Pl = _two_sided_materials()
    two = TwoSidedConfig(wl.n1, wl.n3, wl.dx, wl.dt, [Bu] * 2, [Bl], Pu, Pl, window_cap=1,
                         window_mode="static")
    a = hybrid.hybrid_rupture_two_sided(two, *wl.params(), 30)
    b = hybrid.hybrid_rupture_two_sided(two, *wl.params(), 30, dts=[wl.dt] * 30)
    for k in a:
        np.testing.assert_array_equal(a[k], b[k])
    with pytest.raises(ValueError):
        hybrid.hybrid_rupture(StripConfig(wl.n1, wl.n3, wl.dx, wl.dt, [Layer(RHO, CP, CS)],
                                          Plane(1, MU, CS, CP)), *wl.params(), 3, dts=[wl.dt] * 3)


@pytest.mark.parametrize("two_sided", [False, True])
def test_variable_steps_keep_locked_cells_stuck(two_sided):
    """Random step sizes with the quasi-dynamic boundary relation: cells locked by a huge
    static friction keep exactly zero slip while the waves of the sliding nucleation
    patch pass over them (the stick traction, predictor and corrector of each step use
    that step's size; any mismatch leaves the locked nodes moving)."""
    from oracle.hybrid import TwoSidedConfig
    wl = workloads.FAULTS["tpv3_tiny8"]
    tau0, mus, muk, dc = wl.params()
    patch, _ = wl.masks()
    mus = np.where(patch, mus, workloads.LOCKED_MU_S)
    dts = np.random.default_rng(13).uniform(0.1, 0.3, 60) * wl.dx / CS
    if two_sided:
        Bu, Bl, Pu, Pl = _two_sided_materials()
        cfg = TwoSidedConfig(wl.n1, wl.n3, wl.dx, wl.dt, [Bu] * 2, [Bl] * 2, Pu, Pl,
                             window_cap=1, window_mode="static")
        out = hybrid.hybrid_rupture_two_sided(cfg, tau0, mus, muk, dc, 60, dts=dts)
    else:
        cfg = StripConfig(wl.n1, wl.n3, wl.dx, wl.dt, [Layer(RHO, CP, CS)] * 2,
                          Plane(1, MU, CS, CP), window_cap=1, window_mode="static")
        out = hybrid.hybrid_rupture(cfg, tau0, mus, muk, dc, 60, dts=dts)
    moving = np.abs(out["slip"][:, :, patch]).max()
    assert moving > 1e-3                                   # the patch slides
    assert np.abs(out["slip"][:, :, ~patch]).max() < 1e-12 * moving
    assert np.abs(out["slip_rate"][:, :, ~patch]).max() < 1e-12 * np.abs(out["slip_rate"]).max()
    # and the locked cells do feel the waves: their traction changes
    assert np.ptp(out["traction"][:, 0, ~patch], axis=0).max() > 1e4


def test_variable_steps_converge_like_fixed_steps():
    """Random step sizes (0.1 to 0.3 h / c_s, quasi-dynamic boundary relation): the slip
    at the end of the run is as close to a fine fixed-step solution at the same time
    (0.02 h / c_s) as a fixed-step run of 0.2 h / c_s is (measured 0.38 % against 1.0 %).
    A step of the scheme that mixed two step sizes would not converge (8 %)."""
    wl = workloads.FAULTS["tpv3_tiny8"]
    prm = wl.params()
    h = wl.dx

    def run(dts):
        cfg = StripConfig(wl.n1, wl.n3, h, float(dts[0]), [Layer(RHO, CP, CS)] * 2,
                          Plane(1, MU, CS, CP), window_cap=1, window_mode="static")
        return hybrid.hybrid_rupture(cfg, *prm, len(dts), dts=dts)["slip"][-1]
    dts = np.random.default_rng(14).uniform(0.1, 0.3, 40) * h / CS
    T = dts.sum()
    n_fine, n_coarse = int(round(T / (0.02 * h / CS))), int(round(T / (0.2 * h / CS)))
    ref = run(np.full(n_fine, T / n_fine))
    err = lambda s: np.linalg.norm(s - ref) / np.linalg.norm(ref)  # noqa: E731
    e_var, e_fixed = err(run(dts)), err(run(np.full(n_coarse, T / n_coarse)))
    assert e_var < e_fixed < 0.02, (e_var, e_fixed)


def test_variable_steps_reach_the_plane_wave_slip_rate():
    """k = 0 with the quasi-dynamic boundary relation (pure damping at k = 0) and random
    step sizes inside the elements' stability limit: the slip rate settles on the
    plane-wave value 2 (tau0 - tau_k) c_s / mu, whatever the sequence of steps."""
    n, h = 4, 375.0
    cfg = StripConfig(n, n, h, 0.25 * h / CS, [Layer(RHO, CP, CS)] * 2, Plane(1, MU, CS, CP),
                      window_cap=1, window_mode="static")
    tau0, mus, muk, dc = _uniform(n, 80e6, 0.6, 0.6)
    dts = np.random.default_rng(12).uniform(0.1, 0.3, 600) * h / CS    # c_p dt / h < 0.52
    out = hybrid.hybrid_rupture(cfg, tau0, mus, muk, dc, 600, dts=dts)
    expect = 2 * (80e6 - 0.6 * 120e6) * CS / MU
    assert np.abs(out["slip_rate"][-50:, 0] / expect - 1).max() < 2e-3
    assert out["sliding"][-50:].all()
    # the slip is the time integral of the slip rate over the actual steps
    assert abs(out["slip"][-1, 0, 0, 0] / (expect * dts.sum()) - 1) < 0.05
