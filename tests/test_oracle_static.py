"""Pins of the quasi-dynamic limit of the boundary relation (window mode "static").

The paper names the quasi-dynamic boundary integral relation as the companion
of the dynamic one in a variable time-stepping scheme for earthquake cycles
(Sec. 7): radiation damping of Eq. SBI plus the static elastic response of the
half-space in place of the history integral.  Pins:
  * the static response of one Fourier mode is the Boussinesq-Cerruti surface
    stiffness of a half-space (K11 = K22 = 2 eta^2/(eta^2+1), K12 = -2/(eta^2+1),
    K33 = 1; 1.5, -0.5 and 1 at c_p/c_s = sqrt 3), independent of dt;
  * the dynamic relation with a long window approaches it for a held
    displacement (the kernels' integrals tend to their static limits);
  * a frictionless fault under a sinusoidal load settles on the static slip of
    elasticity (2A/(mu k) antiplane, monotonically; 2(1-nu)A/(mu k) in-plane),
    whatever the sequence of time steps;
  * a uniform fault with variable time steps follows the closed-form slip
    recursion of each step's size.
"""
import math

import numpy as np
import pytest

from oracle import fault
from oracle.sbim import Config, Plane, PlaneOperator


def _held_mode_traction(window_mode, W=1, dt=0.2, steps=1, eta=math.sqrt(3.0)):
    cfg = Config(n1=8, n3=8, dt=dt, planes=[Plane(1, 1.3, 1.0, eta)], window_cap=W,
                 window_mode=window_mode)
    op = PlaneOperator(cfg, 0, (np.array([1]), np.array([2])))   # an oblique mode
    q = float(np.hypot(2 * np.pi / 8, 2 * np.pi * 2 / 8))
    k1, k3 = 2 * np.pi / 8 / q, 2 * np.pi * 2 / 8 / q
    rng = np.random.default_rng(2)
    U = rng.standard_normal(3) + 1j * rng.standard_normal(3)
    Uh = np.repeat(U[None, :, None], steps, axis=0)
    t = op.apply(Uh, np.zeros_like(Uh))[-1, :, 0]
    # rotate to (L, N, T)
    R = np.array([[k1, 0, k3], [0, 1, 0], [-k3, 0, k1]])
    return R @ t, R @ U, 1.3 * q, eta


def test_static_mode_is_boussinesq_cerruti_stiffness():
    for eta in (math.sqrt(3.0), 2.2):
        tr, Ur, muq, eta = _held_mode_traction("static", eta=eta)
        e2 = eta * eta
        K11 = K22 = 2 * e2 / (e2 + 1)
        K12 = -2 / (e2 + 1)
        expect = -muq * np.array([K11 * Ur[0] + 1j * K12 * Ur[1],
                                  K22 * Ur[1] - 1j * K12 * Ur[0],
                                  Ur[2]])
        np.testing.assert_allclose(tr, expect, rtol=1e-12, atol=1e-12 * np.abs(expect).max())
    # independent of the time step
    a = _held_mode_traction("static", dt=0.2)[0]
    b = _held_mode_traction("static", dt=1.7)[0]
    np.testing.assert_allclose(a, b, rtol=1e-14)


def test_dynamic_relation_tends_to_static_for_a_held_displacement():
    stat = _held_mode_traction("static")[0]
    dyn = _held_mode_traction("fixed", W=400, steps=400)[0]   # q c_s t = 140 at the end
    assert np.abs(dyn - stat).max() < 3e-3 * np.abs(stat).max()


def _sinusoid(comp, dts, n1=4):
    cfg = Config(n1=n1, n3=4, dt=0.2, planes=[Plane()], window_cap=1, window_mode="static")
    k = 2 * np.pi / n1
    A = 1e-3
    tau0 = np.zeros((3, n1, 4))
    tau0[1] = -1.0
    tau0[comp] = A * np.cos(k * np.arange(n1))[:, None]
    z = np.zeros((n1, 4))
    out = fault.rupture(cfg, fault.FaultParams(tau0, z, z, z + 1.0), len(dts), dts=dts)
    D = out["slip"][:, 0 if comp == 0 else 1, :, 0]
    return (D * np.cos(k * np.arange(n1))).sum(-1) * 2 / n1, A, k


@pytest.mark.parametrize("comp,factor", [(2, 1.0), (0, 0.75)])
def test_quasi_dynamic_fault_settles_on_static_slip(comp, factor):
    rng = np.random.default_rng(9)
    for dts in ([0.2] * 300, list(rng.uniform(0.05, 0.6, 300))):
        amp, A, k = _sinusoid(comp, dts)
        expect = 2 * factor * A / k
        assert abs(amp[-1] / expect - 1) < 1e-9
        if comp == 2:            # antiplane: one degree of freedom, monotone approach
            assert np.all(np.diff(amp) >= -1e-18)


def test_uniform_fault_with_variable_time_steps():
    """k = 0: delta^{n+1} = delta^n + dt_n (A + B delta^n) while weakening."""
    cfg = Config(n1=4, n3=4, dt=0.2, planes=[Plane()], window_cap=1, window_mode="static")
    tau0 = np.zeros((3, 4, 4))
    tau0[0], tau0[1] = 0.65, -1.0
    full = lambda x: np.full((4, 4), float(x))  # noqa: E731
    rng = np.random.default_rng(4)
    dts = rng.uniform(0.05, 0.3, 25)
    out = fault.rupture(cfg, fault.FaultParams(tau0, full(0.6), full(0.5), full(10.0)), 25, dts=dts)
    A = (0.65 - 0.6) * 2.0
    B = 0.1 / 10.0 * 2.0
    d = 0.0
    for n in range(25):
        d = d + dts[n] * (A + B * d)
        assert abs(out["slip"][n, 0, 0, 0] - d) < 1e-13
    with pytest.raises(ValueError):
        fault.rupture(Config(n1=4, n3=4, planes=[Plane()]), fault.FaultParams(tau0, full(0.6), full(0.5),
                      full(10.0)), 3, dts=[0.1, 0.1, 0.1])
