"""Hybrid finite-element / spectral-boundary-integral rupture (Sec. 2.4).

Oracle module: test infrastructure only (see ``oracle/__init__.py``).

A thin strip of 8-node hexahedral finite elements (Sec. 2.2, FEM) sits on the
fault; its far boundary S+ is closed by the boundary relation of an elastic
half-space (Sec. 2.3, Eq. SBI), which absorbs the waves that leave the strip.
``hybrid_rupture`` models only the upper half of the strip: the fault plane is a
symmetry plane (Sec. 3.1), so the lower half moves as the mirror image, the slip
is twice the upper side's tangential displacement, the fault normal traction
keeps its background value and no normal constraint is needed.
``hybrid_rupture_two_sided`` models both halves with split fault nodes, each
closed by its own boundary relation (S+ and S-), for different materials
across the fault.

Discretisation (the paper's regular hexahedral mesh with matching SBI grid,
Sec. 2.4 and the closing remarks of Sec. 7):
* cubic elements of side h = dx1 = dx3, N2 element layers between the fault
  (node layer 0) and S+ (node layer N2); periodic in x1 and x3 with the SBI
  plane's n1 x n3 grid; each element layer has its own (rho, lambda, mu);
* element stiffness by 2x2x2 Gauss quadrature of the trilinear shape functions
  with isotropic elasticity (Eq. linelasticity), lumped mass rho h^3 / 8 per
  element corner.

Time step t -> t+1 (Sec. 2.2, explicit central differences in predictor-
corrector form; Sec. 2.4 items 1-7):
1. v_{t+1/2} = v_t + dt/2 a_t;  u_{t+1} = u_t + dt v_{t+1/2};
   v^pred_{t+1} = v_t + dt a_t (Eq. fepred).  The displacement advances with the
   half-step velocity: that is the form under which the stick condition on the
   next half-step slip rate keeps the slip fixed, as the paper argues after
   Eq. freeslip.
2-3. The S+ layer's displacement u_{t+1} and predicted velocity v^pred go to the
   boundary relation of the half-space above S+ (side +1), which returns
   tau^SBI (the stress sigma_2i there).
4. Nodal forces r = -K u_{t+1} + h^2 tau^SBI on the S+ layer (outward normal +e2).
5. Fault nodes (layer 0), tangential components: without fault traction the
   next half-step velocity would be v* = v_{t+1/2} + dt r / M (Eq. freeslip
   for one side of a symmetric fault).  The stress change that stops it is
   M v* / (dt h^2) (Eq. sticktraction with the impedance of two mirrored
   sides), so the stick traction is tau~ = tau0 + M v* / (dt h^2).  Strength
   tau^s = sigma0 mu(delta) with delta = 2 |u_t(t+1)| the slip amplitude and mu
   of Eq. slipweak; tau = tau~ if |tau~| <= tau^s, else tau^s tau~/|tau~|
   (Eq. stickslip).  The fault pushes on the strip with -h^2 (tau - tau0).
6-7. a_{t+1} = (r + fault force) / M (Eq. tintf);  v_{t+1} = v_{t+1/2} + dt/2 a_{t+1}
   (Eq. fecorr).
Slip rate reported: 2 v_{t+1} of the fault nodes' tangential components.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import dft
from .fault import friction_coefficient
from .sbim import Config, Plane, PlaneOperator

# node (a1, a2, a3) of an element, a_i in {0, 1}, has local index a1 + 2 a2 + 4 a3
CORNERS = np.array([[i & 1, (i >> 1) & 1, (i >> 2) & 1] for i in range(8)])


def hex8_stiffness(h, lam, mu):
    """24 x 24 stiffness of a cube of side h (dof order: node-major, then x1, x2, x3).

    K = sum over the 2x2x2 Gauss points of B^T D B det(J) w, with B the strain-
    displacement matrix of the trilinear shape functions and D the isotropic
    elasticity matrix in Voigt order (11, 22, 33, 23, 13, 12).
    """
    g = 1.0 / math.sqrt(3.0)
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[np.arange(3), np.arange(3)] = lam + 2 * mu
    D[3, 3] = D[4, 4] = D[5, 5] = mu
    K = np.zeros((24, 24))
    s = 2 * CORNERS - 1                               # corner signs in reference coords
    for xi in (-g, g):
        for eta in (-g, g):
            for zeta in (-g, g):
                p = np.array([xi, eta, zeta])
                # dN/dxi_k for each corner: s_k/8 * prod_{m != k} (1 + s_m p_m)
                dN = np.empty((8, 3))
                for k in range(3):
                    other = [m for m in range(3) if m != k]
                    dN[:, k] = s[:, k] / 8.0 * (1 + s[:, other[0]] * p[other[0]]) * \
                        (1 + s[:, other[1]] * p[other[1]])
                dNdx = dN * (2.0 / h)                 # x = h (1 + xi) / 2 per axis
                B = np.zeros((6, 24))
                for a in range(8):
                    d1, d2, d3 = dNdx[a]
                    B[0, 3 * a] = d1
                    B[1, 3 * a + 1] = d2
                    B[2, 3 * a + 2] = d3
                    B[3, 3 * a + 1], B[3, 3 * a + 2] = d3, d2
                    B[4, 3 * a], B[4, 3 * a + 2] = d3, d1
                    B[5, 3 * a], B[5, 3 * a + 1] = d2, d1
                K += B.T @ D @ B * (h / 2.0) ** 3
    return K


@dataclass
class Layer:
    rho: float
    cp: float
    cs: float

    @property
    def mu(self):
        return self.rho * self.cs ** 2

    @property
    def lam(self):
        return self.rho * self.cp ** 2 - 2 * self.mu


@dataclass
class StripConfig:
    """n1 x n3 periodic grid of spacing h; layers[j] fills x2 in [j h, (j+1) h]."""
    n1: int
    n3: int
    h: float
    dt: float
    layers: list
    plane: Plane                      # the half-space above S+ (side +1)
    window_cap: int = 100
    window_mode: str = "fixed"
    eta_w: float = 1.0

    @property
    def n2(self):
        return len(self.layers)

    def sbim_config(self):
        return Config(n1=self.n1, n3=self.n3, dx1=self.h, dx3=self.h, dt=self.dt,
                      planes=[self.plane], window_cap=self.window_cap,
                      window_mode=self.window_mode, eta_w=self.eta_w, input_kind="absolute")


class Strip:
    """Element loop over the periodic strip (plain numpy; test sizes only)."""

    def __init__(self, cfg: StripConfig):
        self.cfg = cfg
        n1, n2, n3 = cfg.n1, cfg.n2, cfg.n3
        self.shape = (3, n2 + 1, n1, n3)              # [component][node layer][x1][x3]
        self.K = [hex8_stiffness(cfg.h, L.lam, L.mu) for L in cfg.layers]
        # element (l, i1, i3) -> its 8 node indices in the flattened [layer][x1][x3] grid
        i1, i3 = np.meshgrid(np.arange(n1), np.arange(n3), indexing="ij")
        self.conn = []
        for l in range(n2):
            nodes = [((l + a2) * n1 + (i1 + a1) % n1) * n3 + (i3 + a3) % n3
                     for a1, a2, a3 in CORNERS]
            self.conn.append(np.stack([x.ravel() for x in nodes], axis=1))   # [E, 8]
        nn = (n2 + 1) * n1 * n3
        m = np.zeros(nn)
        for l in range(n2):
            np.add.at(m, self.conn[l].ravel(), cfg.layers[l].rho * cfg.h ** 3 / 8.0)
        self.mass = m.reshape(n2 + 1, n1, n3)

    def internal_force(self, u):
        """K u on every node: u [3, n2+1, n1, n3] -> same shape."""
        nn = u[0].size
        uf = u.reshape(3, nn)
        out = np.zeros((3, nn))
        for l, conn in enumerate(self.conn):
            ue = uf[:, conn].transpose(1, 2, 0).reshape(-1, 24)      # [E, 24] node-major
            fe = ue @ self.K[l].T
            fe = fe.reshape(-1, 8, 3)
            for c in range(3):
                np.add.at(out[c], conn.ravel(), fe[:, :, c].ravel())
        return out.reshape(u.shape)


def _step_sizes(cfg, steps, dts):
    """Per-step time steps: allowed with the quasi-dynamic (static) boundary relation,
    which does not depend on dt (Sec. 7, variable time stepping); each step of the
    explicit scheme then runs with its own size in the predictor, the stick traction and
    the corrector."""
    if dts is None:
        return [cfg.dt] * steps
    if cfg.window_mode != "static":
        raise ValueError("variable time steps need the quasi-dynamic (static) boundary relation")
    if len(dts) < steps:
        raise ValueError("fewer time steps than steps")
    return [float(x) for x in dts]


def hybrid_rupture(cfg: StripConfig, tau0, mu_s, mu_k, d_c, steps, weights_cache=None, dts=None):
    """Run the hybrid scheme; returns float64 histories (``dts``: per-step time steps, for
    the quasi-dynamic boundary relation only):

    traction [N, 3, n1, n3]   fault traction (shear from the friction solve, normal tau0_2)
    sliding [N, n1, n3]       the slip branch of Eq. stickslip was taken (bool)
    slip_rate [N, 2, n1, n3]  2 v_{t+1} of the fault nodes, components (1, 3); at a
                              stuck node this is zero up to round-off
    slip [N, 2, n1, n3]       2 u_{t+1} of the fault nodes
    top_u, top_v [N, 3, n1, n3]  S+ layer displacement u_{t+1} and predicted velocity
    """
    strip = Strip(cfg)
    n1, n3, h = cfg.n1, cfg.n3, cfg.h
    dts = _step_sizes(cfg, steps, dts)
    top = cfg.n2
    scfg = cfg.sbim_config()
    op = PlaneOperator(scfg, 0, None, {} if weights_cache is None else weights_cache)
    hh = n3 // 2 + 1
    A = h * h
    M = strip.mass
    u = np.zeros(strip.shape)
    v = np.zeros(strip.shape)
    a = np.zeros(strip.shape)
    hist = []
    sh = [0, 2]
    out = {k: np.empty((steps,) + s) for k, s in (
        ("traction", (3, n1, n3)), ("slip_rate", (2, n1, n3)), ("slip", (2, n1, n3)),
        ("top_u", (3, n1, n3)), ("top_v", (3, n1, n3)))}
    out["sliding"] = np.zeros((steps, n1, n3), dtype=bool)
    for n in range(steps):
        dt = dts[n]
        v_half = v + 0.5 * dt * a
        u = u + dt * v_half
        v_pred = v + dt * a
        # boundary relation on S+: history of the layer's displacement, predicted velocity
        U = dft.forward_half(u[:, top]).reshape(3, -1)
        hist.append(U)
        if len(hist) > max(op.Wmax, 1):
            hist = hist[-op.Wmax:]
        Vh = dft.forward_half(v_pred[:, top]).reshape(3, -1)
        t_hat = op.apply_last(np.stack(hist), Vh)
        tau_sbi = dft.inverse_half(t_hat.reshape(3, n1, hh), n3)
        r = -strip.internal_force(u)
        r[:, top] += A * tau_sbi
        # fault nodes: forward Lagrange multiplier with slip-weakening strength
        M0 = M[0]
        v_star = v_half[sh, 0] + dt * r[sh, 0] / M0
        stick = tau0[sh] + M0 * v_star / (dt * A)
        mag = np.sqrt(stick[0] * stick[0] + stick[1] * stick[1])
        slip_now = 2.0 * u[sh, 0]
        delta = np.sqrt(slip_now[0] * slip_now[0] + slip_now[1] * slip_now[1])
        strength = np.maximum(-tau0[1], 0.0) * friction_coefficient(delta, mu_s, mu_k, d_c)
        slipping = mag > strength
        scale = np.where(slipping, strength / np.where(slipping, mag, 1.0), 1.0)
        tau_sh = stick * scale
        r[sh, 0] -= A * (tau_sh - tau0[sh])
        a = r / M[None]
        v = v_half + 0.5 * dt * a
        out["sliding"][n] = slipping
        out["traction"][n][sh] = tau_sh
        out["traction"][n][1] = tau0[1]
        out["slip_rate"][n] = 2.0 * v[sh, 0]
        out["slip"][n] = slip_now
        out["top_u"][n] = u[:, top]
        out["top_v"][n] = v_pred[:, top]
    return out


@dataclass
class TwoSidedConfig:
    """The strip on both sides of the fault: ``upper[j]`` fills x2 in [j h, (j+1) h]
    above the fault and ``lower[j]`` fills [-(j+1) h, -j h] below it (both listed from
    the fault outwards); ``plane_up`` (side +1) closes S+, ``plane_down`` (side -1) S-."""
    n1: int
    n3: int
    h: float
    dt: float
    upper: list
    lower: list
    plane_up: Plane
    plane_down: Plane
    window_cap: int = 100
    window_mode: str = "fixed"
    eta_w: float = 1.0

    def sbim_config(self):
        return Config(n1=self.n1, n3=self.n3, dx1=self.h, dx3=self.h, dt=self.dt,
                      planes=[self.plane_up, self.plane_down], window_cap=self.window_cap,
                      window_mode=self.window_mode, eta_w=self.eta_w, input_kind="absolute")


def hybrid_rupture_two_sided(cfg: TwoSidedConfig, tau0, mu_s, mu_k, d_c, steps,
                             weights_cache=None, dts=None):
    """The hybrid scheme with the strip on both sides of a split-node fault.

    Each side is its own block of elements (the fault nodes are split: the upper
    copy belongs to the elements above, the lower copy to those below), closed by
    its own boundary relation at S+ or S-.  Per step, as the one-sided scheme for
    each block, and at the fault (Sec. 2.2, Eqs. freeslip, sticktraction,
    stickslip): the half-step velocities the two copies would reach without fault
    traction, v*+ and v*-, give the traction change that closes their jump,
        dtau~ = (v*+ - v*-) / (dt h^2 (1/M+ + 1/M-))      (all three components),
    the normal component is applied as it is (no opening or interpenetration),
    the shear pair is limited by the strength max(-tau_2, 0) mu(delta), delta the
    slip amplitude |u+ - u-| at t+1, and the copies receive -/+ h^2 (tau - tau0).

    Returns float64 histories: traction [N, 3, n1, n3]; sliding [N, n1, n3];
    slip_rate and slip [N, 2, n1, n3] (upper minus lower copy, components 1, 3, at
    t+1); normal_jump [N, n1, n3] (v2 of the upper minus the lower copy).
    """
    up = Strip(StripConfig(cfg.n1, cfg.n3, cfg.h, cfg.dt, cfg.upper, cfg.plane_up))
    lo = Strip(StripConfig(cfg.n1, cfg.n3, cfg.h, cfg.dt, cfg.lower[::-1], cfg.plane_down))
    n1, n3, h = cfg.n1, cfg.n3, cfg.h
    dts = _step_sizes(cfg, steps, dts)
    top, Lb = len(cfg.upper), len(cfg.lower)
    scfg = cfg.sbim_config()
    cache = {} if weights_cache is None else weights_cache
    ops = [PlaneOperator(scfg, p, None, cache) for p in range(2)]
    hh = n3 // 2 + 1
    A = h * h
    state = {k: [np.zeros(s.shape) for _ in range(3)] for k, s in (("up", up), ("lo", lo))}
    hist = [[], []]
    sh = [0, 2]
    out = {k: np.empty((steps,) + s) for k, s in (
        ("traction", (3, n1, n3)), ("slip_rate", (2, n1, n3)), ("slip", (2, n1, n3)),
        ("normal_jump", (n1, n3)))}
    out["sliding"] = np.zeros((steps, n1, n3), dtype=bool)
    for n in range(steps):
        dt = dts[n]
        pred = {}
        for k in ("up", "lo"):
            u, v, a = state[k]
            v_half = v + 0.5 * dt * a
            u = u + dt * v_half
            pred[k] = (u, v_half, v + dt * a)
        tau_sbi = []
        for p, (k, layer) in enumerate((("up", top), ("lo", 0))):
            u, _, v_pred = pred[k]
            hist[p].append(dft.forward_half(u[:, layer]).reshape(3, -1))
            if len(hist[p]) > max(ops[p].Wmax, 1):
                hist[p] = hist[p][-ops[p].Wmax:]
            Vh = dft.forward_half(v_pred[:, layer]).reshape(3, -1)
            t_hat = ops[p].apply_last(np.stack(hist[p]), Vh)
            tau_sbi.append(dft.inverse_half(t_hat.reshape(3, n1, hh), n3))
        (uu, vhu, _), (ul, vhl, _) = pred["up"], pred["lo"]
        ru = -up.internal_force(uu)
        rl = -lo.internal_force(ul)
        ru[:, top] += A * tau_sbi[0]          # S+: outward normal +e2
        rl[:, 0] -= A * tau_sbi[1]            # S-: outward normal -e2
        Mp, Mm = up.mass[0], lo.mass[Lb]
        vsp = vhu[:, 0] + dt * ru[:, 0] / Mp
        vsm = vhl[:, Lb] + dt * rl[:, Lb] / Mm
        stick = tau0 + (vsp - vsm) / (dt * A * (1.0 / Mp + 1.0 / Mm))
        tau = np.empty_like(stick)
        tau[1] = stick[1]
        mag = np.sqrt(stick[0] * stick[0] + stick[2] * stick[2])
        slip_now = uu[sh, 0] - ul[sh, Lb]
        delta = np.sqrt(slip_now[0] * slip_now[0] + slip_now[1] * slip_now[1])
        strength = np.maximum(-tau[1], 0.0) * friction_coefficient(delta, mu_s, mu_k, d_c)
        slipping = mag > strength
        scale = np.where(slipping, strength / np.where(slipping, mag, 1.0), 1.0)
        tau[sh] = stick[sh] * scale
        ru[:, 0] -= A * (tau - tau0)
        rl[:, Lb] += A * (tau - tau0)
        au = ru / up.mass[None]
        al = rl / lo.mass[None]
        vu = vhu + 0.5 * dt * au
        vl = vhl + 0.5 * dt * al
        state["up"] = [uu, vu, au]
        state["lo"] = [ul, vl, al]
        out["traction"][n] = tau
        out["sliding"][n] = slipping
        out["slip"][n] = slip_now
        out["slip_rate"][n] = vu[sh, 0] - vl[sh, Lb]
        out["normal_jump"][n] = vu[1, 0] - vl[1, Lb]
    return out
