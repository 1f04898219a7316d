"""Pins of the oracle's full per-step update (transforms, operator, history).

Each pin is fixed by something other than the oracle itself:
  * transforms: numpy.fft.rfft2 / irfft2 (library routines);
  * single oblique Fourier modes of each polarisation, held constant from
    step 0: closed-form physical-space tractions in terms of G_ab(T), with
    G_ab taken from mpmath's inverse Laplace transform of the half-space
    stiffness (independent of the oracle's branch-cut quadrature);
  * k = 0: a uniform velocity radiates plane S and P waves, traction
    -(mu/c_s) v for shear and -(c_p/c_s)(mu/c_s) v for the normal component;
  * the lower half-space is the mirror image x2 -> -x2 of the upper one;
  * isotropy: rotating a mode's wavevector and polarisation rotates its traction;
  * time invariance, linearity, and the transpose identity <A u, g> = <u, A^T g>;
  * dimensional scaling with the paper's TPV3 material constants.
"""
import json
import math
import os

import mpmath as mp
import numpy as np
import pytest

import oracle
from oracle import dft, kernels
from oracle.sbim import Config, Plane, PlaneOperator

HERE = os.path.dirname(os.path.abspath(__file__))


def _G_inverse_laplace(T, eta):
    """G_ab(T), ab = (11, 12, 22, 33), by Talbot inversion of F_ab(s)/s (mpmath)."""
    from tests.test_oracle_kernels import _F_mp
    mp.mp.dps = 25
    e = mp.mpf(eta)
    if T == 0:
        return np.zeros(4)
    return np.array([float(mp.invertlaplace(lambda s: _F_mp(s, e)[ab] / s, T, method="talbot"))
                     for ab in range(4)])


# ---------------------------------------------------------------- transforms

@pytest.mark.parametrize("shape", [(4, 4), (8, 6), (16, 16), (6, 10)])
def test_dft_matches_numpy(shape):
    rng = np.random.default_rng(1)
    u = rng.standard_normal((2,) + shape)
    np.testing.assert_allclose(dft.forward_half(u), np.fft.rfft2(u), atol=1e-12)
    h = shape[1] // 2 + 1
    t = rng.standard_normal((2, shape[0], h)) + 1j * rng.standard_normal((2, shape[0], h))
    # imaginary parts on the i3 = 0 and i3 = n3/2 columns are not Hermitian-consistent on purpose
    np.testing.assert_allclose(dft.inverse_half(t, shape[1]), np.fft.irfft2(t, s=shape), atol=1e-13)


# ---------------------------------------------------------- single-mode pins

def _mode_field(n1, n3, m1, m3, fn):
    x1 = np.arange(n1)[:, None]
    x3 = np.arange(n3)[None, :]
    ph = 2 * np.pi * (m1 * x1 / n1 + m3 * x3 / n3)
    return fn(ph)


@pytest.mark.parametrize("side", [1, -1])
@pytest.mark.parametrize("pol", ["L", "N", "T"])
def test_oblique_mode_step_response(side, pol):
    """u = e cos(k.x) held from step 0 (absolute input, no velocity given).

    With alpha = [(2 - eta) - G12(T)] mu q and T = q c_s dt min(n+1, W):
      e = L:  tau = -s mu q G11 L cos(k.x) + alpha e2 sin(k.x)
      e = N:  tau = -s mu q G22 e2 cos(k.x) - alpha L sin(k.x)
      e = T:  tau = -s mu q G33 That cos(k.x)
    plus, at n = 0 only, the damping of V^0 = u/dt.
    """
    n1, n3, m1, m3 = 16, 16, 2, 1
    mu, cs, cp, dt, W, N = 1.3, 0.8, 0.8 * 1.9, 0.3, 4, 6
    eta = cp / cs
    cfg = Config(n1=n1, n3=n3, dt=dt, window_cap=W, planes=[Plane(side, mu, cs, cp)])
    k = np.array([2 * np.pi * m1 / n1, 2 * np.pi * m3 / n3])
    q = float(np.hypot(*k))
    L = np.array([k[0] / q, 0.0, k[1] / q])
    E2 = np.array([0.0, 1.0, 0.0])
    That = np.array([-k[1] / q, 0.0, k[0] / q])
    e = {"L": L, "N": E2, "T": That}[pol]
    cosf = _mode_field(n1, n3, m1, m3, np.cos)
    sinf = _mode_field(n1, n3, m1, m3, np.sin)
    u = np.einsum("c,ab->cab", e, cosf)
    u_hist = np.broadcast_to(u, (N, 1, 3, n1, n3)).copy()
    tau = oracle.forward(cfg, u_hist)
    damp = np.array([1.0, eta, 1.0])
    for n in range(N):
        T = q * cs * dt * min(n + 1, W)
        G11, G12, G22, G33 = _G_inverse_laplace(T, eta)
        alpha = ((2 - eta) - G12) * mu * q
        if pol == "L":
            exp = -side * mu * q * G11 * np.einsum("c,ab->cab", L, cosf) + alpha * np.einsum("c,ab->cab", E2, sinf)
        elif pol == "N":
            exp = -side * mu * q * G22 * np.einsum("c,ab->cab", E2, cosf) - alpha * np.einsum("c,ab->cab", L, sinf)
        else:
            exp = -side * mu * q * G33 * np.einsum("c,ab->cab", That, cosf)
        if n == 0:
            exp = exp - side * (mu / cs) / dt * np.einsum("c,ab->cab", damp * e, cosf)
        np.testing.assert_allclose(tau[n, 0], exp, atol=1e-12)


@pytest.mark.parametrize("side", [1, -1])
def test_uniform_velocity_pure_damping(side):
    """k = 0: plane S / P waves; eta_22 = c_p / c_s (the paper's eta_22 taken as a typo)."""
    mu, cs, cp, dt = 2.0, 1.5, 2.9, 0.1
    cfg = Config(n1=8, n3=4, dt=dt, window_cap=5, planes=[Plane(side, mu, cs, cp)],
                 input_kind="increment")
    v = np.array([0.7, -1.1, 0.4])
    du = np.broadcast_to((v * dt)[:, None, None], (3, 8, 4))
    du_hist = np.broadcast_to(du, (7, 1, 3, 8, 4)).copy()
    tau = oracle.forward(cfg, du_hist)
    exp = -side * (mu / cs) * np.array([1.0, cp / cs, 1.0]) * v
    np.testing.assert_allclose(tau, np.broadcast_to(exp[:, None, None], tau.shape[2:])[None, None]
                               * np.ones_like(tau), atol=1e-12)


@pytest.mark.parametrize("side", [1, -1])
def test_instantaneous_term_is_a_local_operator(side):
    """The instantaneous part of the boundary relation (the K12 -> eta - 2 limit) is, in
    physical space, the local operator (2 - eta) mu (du2/dx1, -(du1/dx1 + du3/dx3), du2/dx3),
    with the same sign on both sides.  At the first step with the damping velocity zero
    the history weights vanish as dt -> 0 (w_0 = G(q c_s dt) -> 0), so the traction is that
    operator alone.  The derivatives here: spectral differentiation with numpy FFTs of a
    field without Nyquist content."""
    n1, n3, dx1, dx3 = 16, 12, 0.7, 1.3
    mu, cs, cp = 1.3, 1.0, 1.9
    cfg = Config(n1=n1, n3=n3, dx1=dx1, dx3=dx3, dt=1e-10, window_cap=4,
                 planes=[Plane(side, mu, cs, cp)], input_kind="absolute")
    rng = np.random.default_rng(17)
    spec = rng.standard_normal((3, n1, n3 // 2 + 1)) + 1j * rng.standard_normal((3, n1, n3 // 2 + 1))
    spec[:, n1 // 2, :] = 0
    spec[:, :, n3 // 2] = 0
    u = np.fft.irfft2(spec, s=(n1, n3))
    k1 = 2 * np.pi * np.fft.fftfreq(n1, dx1)[:, None]
    k3 = 2 * np.pi * np.fft.rfftfreq(n3, dx3)[None, :]
    d1 = lambda f: np.fft.irfft2(1j * k1 * np.fft.rfft2(f), s=(n1, n3))  # noqa: E731
    d3 = lambda f: np.fft.irfft2(1j * k3 * np.fft.rfft2(f), s=(n1, n3))  # noqa: E731
    exp = (2.0 - cp / cs) * mu * np.stack([d1(u[1]), -(d1(u[0]) + d3(u[2])), d3(u[1])])
    tau = oracle.forward(cfg, u[None, None], np.zeros((1, 1, 3, n1, n3)))[0, 0]
    np.testing.assert_allclose(tau, exp, atol=1e-8 * np.abs(exp).max())
    assert np.abs(exp).max() > 1e-2                      # a non-trivial field


def test_mirror_rule():
    """tau^-(u1, u2, u3) = diag(-1, 1, -1) tau^+(u1, -u2, u3)."""
    rng = np.random.default_rng(3)
    u = rng.standard_normal((5, 1, 3, 8, 8))
    base = dict(n1=8, n3=8, window_cap=4, window_mode="fixed")
    up = oracle.forward(Config(**base, planes=[Plane(1, 1.2, 0.9, 1.7)]), u * np.array([1, -1, 1])[None, None, :, None, None])
    lo = oracle.forward(Config(**base, planes=[Plane(-1, 1.2, 0.9, 1.7)]), u)
    np.testing.assert_allclose(lo, up * np.array([-1, 1, -1])[None, None, :, None, None], atol=1e-12)


def test_isotropy_rotated_mode():
    """Modes (5, 0) and (3, 4) have equal q on a square grid; their responses are rotations."""
    cfg = Config(n1=16, n3=16, window_cap=6)
    op_a = PlaneOperator(cfg, 0, (np.array([5]), np.array([0])))
    op_b = PlaneOperator(cfg, 0, (np.array([3]), np.array([4])))
    rng = np.random.default_rng(4)
    N = 7
    U = rng.standard_normal((N, 3, 1)) + 1j * rng.standard_normal((N, 3, 1))
    V = rng.standard_normal((N, 3, 1)) + 1j * rng.standard_normal((N, 3, 1))
    c, s = 0.6, 0.8
    Rt = np.array([[c, 0, -s], [0, 1, 0], [s, 0, c]])   # (L, N, T) -> lab for khat = (0.6, 0.8)
    ta = op_a.apply(U, V)
    tb = op_b.apply(np.einsum("ab,nbm->nam", Rt, U), np.einsum("ab,nbm->nam", Rt, V))
    np.testing.assert_allclose(tb, np.einsum("ab,nbm->nam", Rt, ta), atol=1e-12)


# ------------------------------------------------------------ invariances

def test_time_shift_and_linearity():
    rng = np.random.default_rng(5)
    cfg = Config(n1=8, n3=8, window_cap=12, planes=[Plane(1), Plane(-1, 1.1, 0.9, 1.8)])
    u = rng.standard_normal((6, 2, 3, 8, 8))
    w = rng.standard_normal((6, 2, 3, 8, 8))
    t_u = oracle.forward(cfg, u)
    t_w = oracle.forward(cfg, w)
    np.testing.assert_allclose(oracle.forward(cfg, 2.5 * u - 0.5 * w), 2.5 * t_u - 0.5 * t_w, atol=1e-11)
    shifted = np.concatenate([np.zeros((3,) + u.shape[1:]), u], axis=0)
    t_s = oracle.forward(cfg, shifted)
    np.testing.assert_allclose(t_s[3:], t_u, atol=1e-12)
    np.testing.assert_allclose(t_s[:3], 0.0, atol=0)


@pytest.mark.parametrize("kind", ["absolute", "increment"])
@pytest.mark.parametrize("with_v", [False, True])
def test_transpose_identity(kind, with_v):
    rng = np.random.default_rng(6)
    cfg = Config(n1=8, n3=6, dx1=0.7, window_cap=5, window_mode="per_mode", eta_w=0.6,
                 input_kind=kind, planes=[Plane(1), Plane(-1, 2.0, 1.3, 2.5)])
    u = rng.standard_normal((9, 2, 3, 8, 6))
    v = rng.standard_normal(u.shape) if with_v else None
    g = rng.standard_normal(u.shape)
    tau = oracle.forward(cfg, u, v)
    du, dv = oracle.adjoint(cfg, g, with_velocity=with_v)
    lhs = np.sum(tau * g)
    rhs = np.sum(du * u) + (np.sum(dv * v) if with_v else 0.0)
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))


def test_per_mode_window_truncates():
    """W(q) = min(cap, ceil(2 pi eta_w / (q c_s dt))): a mode's history ends after W(q) lags."""
    cfg = Config(n1=16, n3=16, window_cap=50, window_mode="per_mode", eta_w=1.0)
    q, _, _ = oracle.mode_geometry(cfg)
    W = oracle.mode_window(q, 1.0, cfg.dt, cfg)
    assert W[0, 0] == 0
    assert W[1, 0] == min(50, math.ceil(2 * math.pi / (2 * math.pi / 16 * 0.2)))
    assert W[8, 8] == math.ceil(2 * math.pi / (math.hypot(math.pi, math.pi) * 0.2))
    # an impulse at step 0 stops acting on mode (i1, i3) after W(q) steps
    op = PlaneOperator(cfg, 0, (np.array([8]), np.array([8])))
    N = int(W[8, 8]) + 3
    U = np.zeros((N, 3, 1), complex)
    U[0] = 1.0
    t = op.apply(U, np.zeros_like(U))
    assert np.abs(t[int(W[8, 8]) - 1]).max() > 1e-6
    assert np.abs(t[int(W[8, 8]):]).max() == 0.0


def test_dimensional_scaling_tpv3_material():
    """Physical units with the paper's TPV3 bulk map exactly onto unit-free variables.

    x -> x/dx, t -> t c_s/dx, u -> u/dx, tau -> tau/mu with mu = rho c_s^2.
    """
    with open(os.path.join(HERE, "golden", "tpv3_material.json")) as f:
        mat = json.load(f)
    rho, cp, cs, dx = mat["rho_kg_m3"], mat["cp_m_s"], mat["cs_m_s"], mat["dx_m"]
    mu = rho * cs * cs
    dt = 0.3 * dx / cp
    rng = np.random.default_rng(7)
    u = rng.standard_normal((5, 1, 3, 8, 8)) * 0.01
    dim = Config(n1=8, n3=8, dx1=dx, dx3=dx, dt=dt, window_cap=4, planes=[Plane(1, mu, cs, cp)])
    nd = Config(n1=8, n3=8, dx1=1.0, dx3=1.0, dt=dt * cs / dx, window_cap=4, planes=[Plane(1, 1.0, 1.0, cp / cs)])
    t_dim = oracle.forward(dim, u)
    t_nd = oracle.forward(nd, u / dx)
    np.testing.assert_allclose(t_dim / mu, t_nd, rtol=1e-11, atol=1e-13 * np.abs(t_nd).max())
    assert abs(cp / cs - math.sqrt(3.0)) < 1e-3          # Poisson ratio 0.25 of the workloads
