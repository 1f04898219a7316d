"""Pins of the oracle's elastodynamic kernels against what the mathematics fixes.

Chain of pins:
  * the closed-form Laplace-domain stiffness equals an independent numerical
    solve of Navier's equations in a half-space (eigenvectors of the 4x4
    first-order system, decaying branch) at several (q, p) with Re p > 0;
  * the branch-cut kernels H_ab(T) and their integrals G_ab(T) equal mpmath's
    numerical inverse Laplace transform (Talbot contour) of that stiffness
    minus its instantaneous part, and of that divided by s;
  * H_ab(0) equals the initial-value theorem limits of the large-s expansion;
  * G_33 equals its Bessel closed form int_0^T J0 - J1(T) (scipy.special);
  * the per-lag weights telescope to G and converge under node doubling.
"""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy import special

from oracle import kernels

ETAS = [math.sqrt(3.0), 2.3]


def int_j0(x):
    """int_0^x J0 by its Struve-function closed form (scipy.special)."""
    x = np.asarray(x, dtype=np.float64)
    return x * special.j0(x) + np.pi * x / 2 * (special.j1(x) * special.struve(0, x)
                                                - special.j0(x) * special.struve(1, x))


def navier_stiffness(q, p, mu, cs, cp):
    """Surface stiffness of x2 > 0 by eigen-decomposition of d/dx2 (u1, u2, s12, s22).

    Returns S (2x2) with (s12, s22) = S (U_L, U_N) and the anti-plane
    stiffness s (s32 = s U_T) for one mode exp(i q x1 + p t).
    """
    rho = mu / cs ** 2
    lam = rho * cp ** 2 - 2 * mu
    M = lam + 2 * mu
    ik = 1j * q
    A = np.zeros((4, 4), dtype=complex)
    A[0, 1] = -ik
    A[0, 2] = 1 / mu
    A[1, 0] = -lam * ik / M
    A[1, 3] = 1 / M
    A[2, 0] = rho * p ** 2 - ik * (M * ik - lam * lam * ik / M)
    A[2, 3] = -ik * lam / M
    A[3, 1] = rho * p ** 2
    A[3, 2] = -ik
    ev, V = np.linalg.eig(A)
    dec = np.where(ev.real < 0)[0]
    assert dec.size == 2
    U = V[:2, dec]
    S = V[2:, dec] @ np.linalg.inv(U)
    a = np.sqrt(q * q + p * p / cs ** 2)
    a = a if a.real > 0 else -a
    return S, -mu * a


@pytest.mark.parametrize("eta", ETAS)
@pytest.mark.parametrize("q,p", [(1.0, 0.3), (2.5, 1.7), (0.2, 5.0), (1.3, 0.4 + 1.3j), (0.7, 2.0 - 3.0j)])
def test_stiffness_matches_navier_solve(eta, q, p):
    mu, cs = 1.7, 0.9
    cp = eta * cs
    S, s33 = navier_stiffness(q, p, mu, cs, cp)
    s = p / (q * cs)
    k11, k22, k12, k33 = kernels.laplace_stiffness(s, eta)
    expect = -mu * q * np.array([[k11, 1j * k12], [-1j * k12, k22]])
    np.testing.assert_allclose(S, expect, rtol=1e-11, atol=1e-11 * abs(mu * q))
    np.testing.assert_allclose(s33, -mu * q * k33, rtol=1e-12)


def _F_mp(s, eta):
    """Closed-form stiffness minus instantaneous parts, continued off the cut [-i eta, i eta].

    (Pinned to the Navier solve above on Re s > 0 through the oracle's numpy
    version, compared here at the same points.)
    """
    e2 = eta * eta
    a_s = s * mp.sqrt(1 + 1 / s ** 2)
    a_p = s * mp.sqrt(1 + e2 / s ** 2) / eta
    d = s ** 2 + e2 + 1
    return ((a_s * (e2 + s ** 2) + e2 * a_p) / d - s,
            (e2 * a_s * a_p - e2 - 2 - 2 * s ** 2) / d - (eta - 2),
            e2 * ((1 + s ** 2) * a_p + a_s) / d - eta * s,
            a_s - s)


@pytest.mark.parametrize("eta", ETAS)
def test_mp_stiffness_agrees_with_numpy_on_right_half_plane(eta):
    for s in [0.3, 1.0, 4.0, 0.5 + 2j, 1.5 - 0.7j]:
        a = [complex(v) for v in _F_mp(mp.mpc(s), mp.mpf(eta))]
        b = kernels.kernel_laplace(s, eta)
        np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("eta", ETAS)
def test_kernels_match_inverse_laplace(eta):
    mp.mp.dps = 25
    e = mp.mpf(eta)
    T = [0.3, 1.7, 4.0]
    H = kernels.kernel_H(T, eta)
    G = kernels.kernel_G(T, eta)
    for t_i, t in enumerate(T):
        for ab in range(4):
            h_ref = mp.invertlaplace(lambda s: _F_mp(s, e)[ab], t, method="talbot")
            g_ref = mp.invertlaplace(lambda s: _F_mp(s, e)[ab] / s, t, method="talbot")
            assert abs(H[ab, t_i] - float(h_ref)) < 1e-13
            assert abs(G[ab, t_i] - float(g_ref)) < 1e-13


@pytest.mark.parametrize("eta", ETAS)
def test_initial_values(eta):
    """H_ab(0) = lim s F_ab(s): eta - 1/2, 0, eta^2 (2 - eta)/2, 1/2; H12'(0) = -eta (eta-1)^2 / 2."""
    H0 = kernels.kernel_H([0.0], eta)[:, 0]
    np.testing.assert_allclose(H0, [eta - 0.5, 0.0, eta ** 2 * (2 - eta) / 2, 0.5], atol=1e-14)
    mp.mp.dps = 40
    big = mp.mpf(10) ** 9
    sF = [float(mp.re(big * f)) for f in _F_mp(big, mp.mpf(eta))]
    np.testing.assert_allclose(sF, H0, atol=1e-8)
    h = 1e-5
    d12 = (kernels.kernel_H([h], eta)[1, 0] - kernels.kernel_H([-h], eta)[1, 0]) / (2 * h)
    assert abs(d12 + eta * (eta - 1) ** 2 / 2) < 1e-8
    mp.mp.dps = 50
    big = mp.mpf(10) ** 12
    assert abs(float(big * big * _F_mp(big, mp.mpf(eta))[1]) + eta * (eta - 1) ** 2 / 2) < 1e-9


@pytest.mark.parametrize("eta", ETAS)
def test_G33_bessel_closed_form(eta):
    T = np.array([0.01, 0.5, 3.0, 17.0, 80.0, 333.3])
    G = kernels.kernel_G(T, eta)[3]
    ref = int_j0(T) - special.j1(T)
    np.testing.assert_allclose(G, ref, rtol=0, atol=2e-14)
    H = kernels.kernel_H(T, eta)[3]
    np.testing.assert_allclose(H, special.j1(T) / T, rtol=0, atol=2e-15)


@pytest.mark.parametrize("q,dt,W", [(2 * math.pi / 64, 0.2, 100), (1.9, 0.2, 300), (4.4, 0.2, 60), (0.003, 0.2, 400)])
def test_weights_telescope_to_G(q, dt, W):
    eta = math.sqrt(3.0)
    w = kernels.lag_weights(q, 1.0, dt, W, eta)
    partial = np.cumsum(w, axis=1)
    T = q * dt * np.arange(1, W + 1)
    G = kernels.kernel_G(T, eta)
    scale = np.abs(G).max() + 1e-300
    np.testing.assert_allclose(partial, G, rtol=0, atol=1e-14 * max(1.0, scale))


def test_weights_G33_bessel_and_node_doubling():
    """w33_j = int_{T_j}^{T_j+1} J1(t)/t dt (mpmath Bessel quadrature), and n -> 2n changes nothing."""
    eta = math.sqrt(3.0)
    q, dt, W = 3.1, 0.2, 500
    w = kernels.lag_weights(q, 1.0, dt, W, eta)
    mp.mp.dps = 30
    for j in [0, 1, 7, 41, 250, 499]:
        a, b = mp.mpf(q * dt * j), mp.mpf(q * dt * (j + 1))
        ref = mp.quad(lambda t: mp.besselj(1, t) / t, mp.linspace(a, b, 4))
        assert abs(w[3, j] - float(ref)) < 1e-16
    Tj = q * dt * np.arange(W + 1)
    np.testing.assert_allclose(w[3], np.diff(int_j0(Tj) - special.j1(Tj)), rtol=0, atol=2e-12)
    n0 = kernels._node_count(q * dt * W, eta)
    w2 = kernels.lag_weights(q, 1.0, dt, W, eta, n=2 * n0)
    np.testing.assert_allclose(w, w2, rtol=0, atol=4e-16)


def test_static_limits():
    """G_ab(T) -> F_ab(0): the static Fourier stiffness of the half-space minus eta - 2."""
    eta = math.sqrt(3.0)
    e2 = eta * eta
    F0 = kernels.kernel_laplace(1e-9, eta)
    static = [2 * e2 / (e2 + 1), -2 / (e2 + 1) - (eta - 2), 2 * e2 / (e2 + 1), 1.0]
    np.testing.assert_allclose(np.real(F0), static, atol=1e-8)
    G = kernels.kernel_G([4000.0], eta)[:, 0]
    np.testing.assert_allclose(G, static, atol=2e-4)
