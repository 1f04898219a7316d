"""Elastodynamic half-space kernels of the spectral boundary integral relation.

Oracle module: test infrastructure only (see ``oracle/__init__.py``).

The paper states the boundary relation (Sec. 2.3, Eq. SBI) and says the nonlocal
term is a spatial Fourier transform plus a time convolution of the displacement
history with elastodynamic kernels, deferring the kernels themselves to the
independent formulation of Breitenfeld & Geubelle.  Those kernels follow from the
momentum balance (Sec. 2.1, Eq. consmoment) and isotropic linear elasticity
(Sec. 2.1, Eq. linelasticity) applied to a half-space; this module writes the
result out in three forms:

* ``laplace_stiffness``: the exact Fourier-Laplace surface stiffness K_ab(s),
  s = p / (q c_s), of the half-space lying on the +x2 side of its boundary;
* ``kernel_H`` / ``kernel_G``: the time kernels H_ab(T), T = q c_s t, i.e. the
  inverse Laplace transforms of K_ab(s) minus their instantaneous parts, and
  their running integrals G_ab(T);
* ``lag_weights``: the per-lag convolution weights
  w_ab,j(q) = G_ab(q c_s (j+1) dt) - G_ab(q c_s j dt).

Wave-speed ratio eta = c_p / c_s.  Index order of the four kernels everywhere:
(11, 12, 22, 33) = (L-L, L-N coupling, N-N, T-T) in the wavevector frame
(L along k, N the plane normal e2, T transverse).
"""
from __future__ import annotations

import numpy as np

KERNEL_NAMES = ("11", "12", "22", "33")


def laplace_stiffness(s, eta):
    """Fourier-Laplace stiffness (K11, K22, K12, K33) of an elastic half-space.

    For one Fourier mode exp(i k x) with |k| = q and Laplace variable p,
    s = p / (q c_s), the surface tractions sigma_i2 of the half-space x2 > 0 are
        tau_L = -mu q [K11 U_L + i K12 U_N]
        tau_N = -mu q [K22 U_N - i K12 U_L]
        tau_T = -mu q  K33 U_T.
    Derived from Eq. consmoment + Eq. linelasticity with decaying P and S
    potentials; valid for Re s > 0, where the principal square roots are the
    decaying branches.
    """
    s = np.asarray(s, dtype=complex)
    e2 = eta * eta
    a_s = np.sqrt(1.0 + s * s)
    a_p = np.sqrt(1.0 + s * s / e2)
    d = s * s + e2 + 1.0
    k11 = (a_s * (e2 + s * s) + e2 * a_p) / d
    k22 = e2 * ((1.0 + s * s) * a_p + a_s) / d
    k12 = (e2 * a_s * a_p - e2 - 2.0 - 2.0 * s * s) / d
    return k11, k22, k12, a_s


def instantaneous_parts(s, eta):
    """Large-s parts of (K11, K22, K12, K33): (s, eta s, eta - 2, s).

    The s-proportional parts are the radiation damping of Eq. SBI (mu/c_s for
    the in-plane and anti-plane shear components, eta mu / c_s for the normal
    one); the constant eta - 2 is the instantaneous L-N coupling.
    """
    s = np.asarray(s, dtype=complex)
    return s, eta * s, (eta - 2.0) + 0.0 * s, s


def kernel_laplace(s, eta):
    """F_ab(s) = K_ab(s) minus its large-s part, order (11, 12, 22, 33).

    F_ab is the Laplace transform (in T) of the time kernel H_ab(T).
    """
    k11, k22, k12, k33 = laplace_stiffness(s, eta)
    i11, i22, i12, i33 = instantaneous_parts(s, eta)
    return k11 - i11, k12 - i12, k22 - i22, k33 - i33


# --------------------------------------------------------------------------
# Branch-cut representation.  Each F_ab is analytic off the cut [-i eta, i eta]
# and decays at infinity, so wrapping the Bromwich contour around the cut gives
#   H_ab(T) = (1/pi) int_0^eta D_ab(y) cos(y T) dy     (ab = 11, 22, 33)
#   H_12(T) = (1/pi) int_0^eta D_12(y) sin(y T) dy
# with D_ab the jump of F_ab across the cut (computed below), and
# A_s = sqrt(1-y^2), A_p = sqrt(1-y^2/eta^2), B_s = sqrt(y^2-1),
# d = eta^2 + 1 - y^2:
#   D_11 = 2[A_s (eta^2-y^2) + eta^2 A_p]/d  (y<1),   2 eta^2 A_p/d        (1<y<eta)
#   D_22 = 2 eta^2[(1-y^2) A_p + A_s]/d      (y<1),   2 eta^2 (1-y^2) A_p/d (1<y<eta)
#   D_12 = 0                                 (y<1),  -2 eta^2 B_s A_p/d     (1<y<eta)
#   D_33 = 2 A_s                             (y<1),   0                     (1<y<eta)
# The square-root end points at y = 1 and y = eta are removed by the
# substitutions y = sin(theta) on [0, 1] and y^2 = 1 + (eta^2-1) sin^2(psi) on
# [1, eta]; after them every integrand is smooth and Gauss-Legendre converges
# geometrically once the oscillation is resolved.
# --------------------------------------------------------------------------

_GL_CACHE = {}


def _gauss_legendre(n):
    """n-point Gauss-Legendre rule on [-1, 1] in extended precision.

    Nodes are Newton-polished roots of P_n (three-term recurrence), started
    from numpy's estimates; weights 2 / ((1 - x^2) P_n'(x)^2).  numpy's own
    weights lose up to 1e-13 absolute at n ~ 1600, which is why the rule is
    recomputed here.
    """
    if n in _GL_CACHE:
        return _GL_CACHE[n]
    x = np.polynomial.legendre.leggauss(n)[0].astype(np.longdouble)

    def legendre_and_derivative(x):
        p0 = np.ones_like(x)
        p1 = x.copy()
        for k in range(2, n + 1):
            p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
        return p1, n * (x * p1 - p0) / (x * x - 1)

    for _ in range(3):
        p, dp = legendre_and_derivative(x)
        x = x - p / dp
    p, dp = legendre_and_derivative(x)
    w = 2 / ((1 - x * x) * dp * dp)
    _GL_CACHE[n] = (x, w)
    return x, w


def _cut_nodes(n, eta):
    """Nodes y and the four weighted densities D_ab(y) dy on [0, eta].

    Returns y (2n,) in extended precision and dens (4, 2n) float64 with
    dens[ab] = D_ab(y) * (dy/dvar) * Gauss weight.
    """
    x, wx = _gauss_legendre(n)
    quarter_pi = np.arctan(np.longdouble(1))  # pi/4 in extended precision
    t = (x + 1) * quarter_pi                  # map [-1, 1] -> [0, pi/2]
    wt = wx * quarter_pi
    eta = np.longdouble(eta)
    e2 = eta * eta

    # piece A: y = sin(t), 0 < y < 1
    ya = np.sin(t)
    a_s = np.cos(t)
    a_pa = np.sqrt(1 - ya * ya / e2)
    da = e2 + 1 - ya * ya
    jac_a = np.cos(t) * wt
    d11a = 2 * (a_s * (e2 - ya * ya) + e2 * a_pa) / da
    d22a = 2 * e2 * ((1 - ya * ya) * a_pa + a_s) / da
    d12a = np.zeros_like(ya)
    d33a = 2 * a_s

    # piece B: y^2 = 1 + (eta^2 - 1) sin^2(t), 1 < y < eta
    sb, cb = np.sin(t), np.cos(t)
    yb = np.sqrt(1 + (e2 - 1) * sb * sb)
    b_s = np.sqrt(e2 - 1) * sb
    a_pb = np.sqrt(e2 - 1) * cb / eta
    db = e2 + 1 - yb * yb
    jac_b = (e2 - 1) * sb * cb / yb * wt
    d11b = 2 * e2 * a_pb / db
    d22b = 2 * e2 * (1 - yb * yb) * a_pb / db
    d12b = -2 * e2 * b_s * a_pb / db
    d33b = np.zeros_like(yb)

    y = np.concatenate([ya, yb])
    dens = np.stack([
        np.concatenate([d11a * jac_a, d11b * jac_b]),
        np.concatenate([d12a * jac_a, d12b * jac_b]),
        np.concatenate([d22a * jac_a, d22b * jac_b]),
        np.concatenate([d33a * jac_a, d33b * jac_b]),
    ]).astype(np.float64)
    return y, dens


def _node_count(t_max, eta):
    """Gauss-Legendre nodes per cut piece for oscillation up to phase t_max.

    d y / d(var) <= max(1, (eta^2 - 1)/2) on both pieces, so the phase y T
    varies at most that fast in the substituted variable over [0, pi/2];
    the count below is about twice what convergence to rounding needs.
    """
    rate = max(1.0, (eta * eta - 1.0) / 2.0)
    return int(np.ceil(1.2 * t_max * rate * np.pi / 4.0 + 48))


def kernel_H(T, eta, n=None):
    """H_ab(T) for an array of T >= 0, shape (4, len(T)), order (11, 12, 22, 33)."""
    T = np.atleast_1d(np.asarray(T, dtype=np.float64))
    if n is None:
        n = _node_count(float(T.max()) if T.size else 0.0, eta)
    y, dens = _cut_nodes(n, eta)
    ph = np.multiply.outer(T.astype(np.longdouble), y)
    c = np.cos(ph).astype(np.float64)
    s = np.sin(ph).astype(np.float64)
    out = np.empty((4, T.size))
    out[0] = c @ dens[0] / np.pi
    out[1] = s @ dens[1] / np.pi
    out[2] = c @ dens[2] / np.pi
    out[3] = c @ dens[3] / np.pi
    return out


def kernel_G(T, eta, n=None):
    """G_ab(T) = int_0^T H_ab, shape (4, len(T)).

    G_ab = (1/pi) int D sin(yT)/y dy for the cosine kernels and
    (1/pi) int D (1 - cos yT)/y dy for ab = 12; 1 - cos(yT) is written as
    2 sin^2(yT/2) to avoid cancellation at small T.
    """
    T = np.atleast_1d(np.asarray(T, dtype=np.float64))
    if n is None:
        n = _node_count(float(T.max()) if T.size else 0.0, eta)
    y, dens = _cut_nodes(n, eta)
    ph = np.multiply.outer(T.astype(np.longdouble), y)
    sn = (np.sin(ph) / y).astype(np.float64)
    vc = (2 * np.sin(ph / 2) ** 2 / y).astype(np.float64)
    out = np.empty((4, T.size))
    out[0] = sn @ dens[0] / np.pi
    out[1] = vc @ dens[1] / np.pi
    out[2] = sn @ dens[2] / np.pi
    out[3] = sn @ dens[3] / np.pi
    return out


def lag_weights(q, cs, dt, W, eta, n=None):
    """Convolution weights w_ab,j(q), j = 0..W-1, shape (4, W).

    The displacement history is taken piecewise constant, U(t_n - t') = U^{n-j}
    for t' in [j dt, (j+1) dt), and the kernel is integrated exactly over each
    interval:  w_ab,j = G_ab(T_{j+1}) - G_ab(T_j),  T_j = q c_s j dt.
    Written without the difference (which would cancel for small q):
      cos kernels:  w_j = (2/pi) int D(y)/y cos(y Tbar_j) sin(y dT/2) dy
      ab = 12:      w_j = (2/pi) int D(y)/y sin(y Tbar_j) sin(y dT/2) dy
    with dT = q c_s dt and Tbar_j = (j + 1/2) dT.  Phases are formed in extended
    precision so that their rounding (relative 1e-19) stays far below the
    float64 result.
    """
    W = int(W)
    if W <= 0 or q == 0.0:
        return np.zeros((4, max(W, 0)))
    dT = float(q) * float(cs) * float(dt)
    if n is None:
        n = _node_count(dT * W, eta)
    y, dens = _cut_nodes(n, eta)
    yl = y
    tbar = (np.arange(W, dtype=np.longdouble) + np.longdouble(0.5)) * np.longdouble(dT)
    ph = np.multiply.outer(tbar, yl)
    c = np.cos(ph).astype(np.float64)
    s = np.sin(ph).astype(np.float64)
    half = (np.sin(yl * np.longdouble(dT) / 2) / yl).astype(np.float64)
    g = dens * half[None, :] * (2.0 / np.pi)
    w = np.empty((4, W))
    w[0] = c @ g[0]
    w[1] = s @ g[1]
    w[2] = c @ g[2]
    w[3] = c @ g[3]
    return w
