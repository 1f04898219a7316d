"""Frictional fault between the two half-spaces: pure spectral-boundary-integral rupture.

Oracle module: test infrastructure only (see ``oracle/__init__.py``).

The fault is the plane x2 = 0 between an upper half-space (plane side +1) and a
lower one (side -1), each with its own boundary displacement u^+ / u^- and its
own boundary relation (Sec. 2.3, Eq. SBI; two independent half-spaces, as in the
independent formulation the paper defers to).  The interface conditions are the
ones of Sec. 2.2: traction continuity across the fault, the stick and slip
conditions (Eqs. stick and slip) and linear slip-weakening strength (Eq.
slipweak, strength = normal stress x friction coefficient, with the slip delta
of Eq. slipweak the amplitude of the slip vector, Sec. 2.2).  The paper runs this
with its finite elements next to the fault (Sec. 2.4, items 5-7); here the two
half-spaces touch the fault directly, which is the stand-alone boundary-integral
rupture it compares against in Sec. 3.

Explicit step n (u^{+,0} = u^{-,0} = 0, slip D^0 = 0):

1. f^{+-} = tau0 + s^{+-}: background traction plus the traction that each
   half-space's boundary relation gives for its displacement history up to
   u^{+-,n} with the radiation-damping term left out (``sbim.PlaneOperator``
   with zero velocity).
2. Traction balance.  The upper side carries tau = f^+ - Z^+ v^+ and the lower
   side tau = f^- + Z^- v^- (the damping coefficients of Eq. SBI,
   Z_i = eta_ii mu / c_s with eta_22 = c_p / c_s; the lower side's sign follows
   from the mirror x2 -> -x2).  Both equal the fault traction tau.
   Normal component: no opening (v2^+ = v2^-), hence
       tau_2 = (Z2^- f2^+ + Z2^+ f2^-) / (Z2^+ + Z2^-).
   Shear components (1, 3): the traction that keeps the slip rate zero is
       tau~ = (Z^- f^+ + Z^+ f^-) / (Z^+ + Z^-).
3. Strength tau^s = sigma^n mu(delta^n) with sigma^n = max(-tau_2, 0)
   (compression positive; tension gives zero strength), mu of Eq. slipweak and
   delta^n = |D^n| the amplitude of the slip before this step's update.
4. Stick if |tau~| <= tau^s: tau = tau~, slip rate V = 0.  Otherwise slip:
   tau = tau^s tau~ / |tau~| and V = (tau~ - tau)(1/Z^+ + 1/Z^-), parallel to
   tau~ (so V >= 0 along the traction, as Eq. slip requires).
5. v^+ = (f^+ - tau)/Z^+, v^- = (tau - f^-)/Z^-; u^{+-,n+1} = u^{+-,n} + dt v^{+-};
   slip D^{n+1} = D^n + dt V.

One plane only (side +1): the lower half-space is the mirror image of the upper
one (same material, u^- = (-u1^+, u2^+, -u3^+)), so s^- = (s1^+, -s2^+, s3^+) and
the fault plane is a symmetry plane (Sec. 3.1: the normal stress stays at its
background value).  Two planes: sides (+1, -1) in that order, materials free.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import dft
from .sbim import Config, PlaneOperator


@dataclass
class FaultParams:
    """Per-cell fault properties; arrays on the [n1, n3] grid (tau0: [3, n1, n3]).

    tau0: background traction sigma_2i on the fault (component 2 is the normal
          traction, tension positive); mu_s, mu_k: static and kinetic friction
          coefficients; d_c: slip-weakening distance (Eq. slipweak).
    """
    tau0: np.ndarray
    mu_s: np.ndarray
    mu_k: np.ndarray
    d_c: np.ndarray


def impedances(cfg):
    """(Z^+, Z^-), each [3]: eta_ii mu / c_s of the upper and lower half-space."""
    def z(pl):
        return np.array([pl.mu / pl.cs, (pl.cp / pl.cs) * pl.mu / pl.cs, pl.mu / pl.cs])
    zp = z(cfg.planes[0])
    zm = zp if len(cfg.planes) == 1 else z(cfg.planes[1])
    return zp, zm


def friction_coefficient(delta, mu_s, mu_k, d_c):
    """Eq. slipweak: linear weakening from mu_s to mu_k as the slip grows to d_c."""
    return np.where(delta < d_c, mu_s - (mu_s - mu_k) * delta / d_c, mu_k)


def interface_solve(fp, fm, zp, zm, D, prm):
    """Steps 2-4 on the grid.  fp, fm: [3, n1, n3] traction functionals of the two
    sides (background included); D [2, n1, n3]: slip before the step.  Returns
    (tau [3], V [2] for components (1, 3), v^+ [3], v^- [3])."""
    tau = np.empty_like(fp)
    tau[1] = (zm[1] * fp[1] + zp[1] * fm[1]) / (zp[1] + zm[1])
    sh = [0, 2]
    stick = (zm[0] * fp[sh] + zp[0] * fm[sh]) / (zp[0] + zm[0])      # [2, n1, n3]
    mag = np.sqrt(stick[0] ** 2 + stick[1] ** 2)
    delta = np.sqrt(D[0] * D[0] + D[1] * D[1])
    strength = np.maximum(-tau[1], 0.0) * friction_coefficient(delta, prm.mu_s, prm.mu_k, prm.d_c)
    slipping = mag > strength
    scale = np.where(slipping, strength / np.where(slipping, mag, 1.0), 1.0)
    tau[sh] = stick * scale
    V = (stick - tau[sh]) * (1.0 / zp[0] + 1.0 / zm[0])
    vp = (fp - tau) / zp[:, None, None]
    vm = (tau - fm) / zm[:, None, None]
    return tau, V, vp, vm


MIRROR = np.array([1.0, -1.0, 1.0])      # s^- of the mirrored lower half-space


def rupture(cfg, prm: FaultParams, steps, weights_cache=None, dts=None):
    """Run ``steps`` explicit steps; returns a dict of float64 histories.

    ``dts``: per-step time steps, allowed in the quasi-dynamic limit
    (window_mode "static"), whose boundary relation does not depend on dt.

    traction [N, 3, n1, n3]   fault traction tau^n
    slip_rate [N, 2, n1, n3]  V^n, components (1, 3)
    slip [N, 2, n1, n3]       D^{n+1} (after the step's update)
    v_plus, v_minus [N, 3, n1, n3]  side velocities v^{+-,n}
    """
    if not isinstance(cfg, Config):
        cfg = Config.from_dict(cfg)
    P = len(cfg.planes)
    sides = [pl.side for pl in cfg.planes]
    if sides not in ([1], [1, -1]):
        raise ValueError(f"fault needs planes with sides [+1] or [+1, -1], got {sides}")
    if cfg.input_kind != "absolute":
        raise ValueError("the fault oracle pushes absolute displacements")
    if dts is not None and cfg.window_mode != "static":
        raise ValueError("variable time steps need the quasi-dynamic (static) boundary relation")
    dts = [cfg.dt] * steps if dts is None else [float(x) for x in dts]
    n1, n3 = cfg.n1, cfg.n3
    h = n3 // 2 + 1
    cache = {} if weights_cache is None else weights_cache
    ops = [PlaneOperator(cfg, p, None, cache) for p in range(P)]
    zp, zm = impedances(cfg)
    tau0 = np.asarray(prm.tau0, dtype=np.float64)

    u = np.zeros((P, 3, n1, n3))
    D = np.zeros((2, n1, n3))
    hist = [[] for _ in range(P)]
    out = {k: np.empty((steps,) + s) for k, s in (
        ("traction", (3, n1, n3)), ("slip_rate", (2, n1, n3)), ("slip", (2, n1, n3)),
        ("v_plus", (3, n1, n3)), ("v_minus", (3, n1, n3)))}
    for n in range(steps):
        s = np.empty((P, 3, n1, n3))
        for p in range(P):
            Uh = dft.forward_half(u[p]).reshape(3, -1)
            hist[p].append(Uh)
            keep = max(ops[p].Wmax, 1)
            if len(hist[p]) > keep:
                hist[p] = hist[p][-keep:]
            th = ops[p].apply_last(np.stack(hist[p]), np.zeros_like(Uh))
            s[p] = dft.inverse_half(th.reshape(3, n1, h), n3)
        fp = tau0 + s[0]
        fm = tau0 + (MIRROR[:, None, None] * s[0] if P == 1 else s[1])
        tau, V, vp, vm = interface_solve(fp, fm, zp, zm, D, prm)
        dt = dts[n]
        u[0] += dt * vp
        if P == 2:
            u[1] += dt * vm
        D += dt * V
        out["traction"][n] = tau
        out["slip_rate"][n] = V
        out["slip"][n] = D
        out["v_plus"][n] = vp
        out["v_minus"][n] = vm
    return out
