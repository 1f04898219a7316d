"""Seeded synthetic boundary-displacement workloads.

Shared by the tests (both the oracle side and the GPU side draw inputs from
here) and by ``bench.py``.  It holds no part of the boundary-integral
arithmetic: only random numbers, a spectral shaping of white noise with scipy's
FFT, and the named workload shapes.

The paper's runs are earthquake ruptures on regular boundary grids (Sec. 3-6;
Poisson ratio 0.25, i.e. c_p/c_s = sqrt(3)).  No field data is used: the
workloads below are nondimensional stand-ins with mu = 1, c_s = 1,
c_p = sqrt(3), dx = 1, dt = 0.2.

Random increments: for each plane p and component c a PCG64 stream seeded with
1000*workload + 10*p + c draws white N(0,1) fields in step order; each field is
shaped to spectral amplitude |k|^-2 (k = 0 removed) and normalised to unit RMS.
For the larger workloads a bank of 64 such fields per (plane, component) is
drawn once and step n uses bank[(7 n) mod 64].
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field

import numpy as np

SQRT3 = math.sqrt(3.0)


@dataclass
class Workload:
    ident: int
    name: str
    n1: int
    n3: int
    planes: list                 # list of dicts: side, mu, cs, cp
    window_cap: int
    steps: int
    window_mode: str = "fixed"
    eta_w: float = 1.0
    dt: float = 0.2
    dx1: float = 1.0
    dx3: float = 1.0
    input_kind: str = "increment"
    bank: int = 0                # 0: fresh field every step; else bank size
    pulse: bool = False          # Gaussian ramp pulse on u1
    slip_ramp: float = 0.0       # final uniform slip velocity on u1 (k = 0 mode)
    extra: dict = field(default_factory=dict)

    def config_dict(self):
        return dict(n1=self.n1, n3=self.n3, dx1=self.dx1, dx3=self.dx3, dt=self.dt,
                    planes=[dict(p) for p in self.planes], window_cap=self.window_cap,
                    window_mode=self.window_mode, eta_w=self.eta_w,
                    input_kind=self.input_kind)

    def scaled(self, **kw):
        d = dict(self.__dict__)
        d.update(kw)
        return Workload(**d)


def _plane(side):
    return dict(side=side, mu=1.0, cs=1.0, cp=SQRT3)


ONE = [_plane(+1)]
TWO = [_plane(+1), _plane(-1)]

WORKLOADS = {
    1: Workload(1, "plane64_w100_fp64", 64, 64, ONE, 100, 200),
    2: Workload(2, "two_planes512_w1000", 512, 512, TWO, 1000, 2000, bank=64, pulse=True),
    3: Workload(3, "two_planes2048_permode400", 2048, 2048, TWO, 400, 1000,
                window_mode="per_mode", bank=64),
    4: Workload(4, "plane256_w300_adjoint", 256, 256, ONE, 300, 500),
    5: Workload(5, "two_planes1024_w2000_longrun", 1024, 1024, TWO, 2000, 5000,
                bank=64, slip_ramp=10.0),
}


def shaped_field(rng, n1, n3, dx1=1.0, dx3=1.0):
    """One white field shaped to spectral amplitude |k|^-2, k = 0 removed, unit RMS."""
    import scipy.fft as sfft
    white = rng.standard_normal((n1, n3))
    workers = min(16, os.cpu_count() or 1)
    spec = sfft.rfft2(white, workers=workers)
    k1 = 2 * np.pi * np.fft.fftfreq(n1, d=dx1)
    k3 = 2 * np.pi * np.fft.rfftfreq(n3, d=dx3)
    kk = k1[:, None] ** 2 + k3[None, :] ** 2
    amp = np.zeros_like(kk)
    amp[kk > 0] = 1.0 / kk[kk > 0]
    f = sfft.irfft2(spec * amp, s=(n1, n3), workers=workers)
    rms = np.sqrt(np.mean(f * f))
    return f / rms if rms > 0 else f


class Increments:
    """Deterministic per-step displacement increments du^n [P, 3, n1, n3] float64."""

    def __init__(self, wl: Workload):
        self.wl = wl
        P = len(wl.planes)
        self._rngs = [[np.random.default_rng(1000 * wl.ident + 10 * p + c) for c in range(3)]
                      for p in range(P)]
        self._bank = None
        if wl.bank:
            self._bank = np.empty((wl.bank, P, 3, wl.n1, wl.n3))
            for b in range(wl.bank):
                for p in range(P):
                    for c in range(3):
                        self._bank[b, p, c] = shaped_field(self._rngs[p][c], wl.n1, wl.n3,
                                                           wl.dx1, wl.dx3)
        self._next = 0
        self._cache = {}
        if wl.pulse:
            x1 = np.arange(wl.n1) - wl.n1 / 2
            x3 = np.arange(wl.n3) - wl.n3 / 2
            r2 = x1[:, None] ** 2 + x3[None, :] ** 2
            self._gauss = 10.0 * np.exp(-r2 / (2.0 * 20.0 ** 2))

    def _random(self, n):
        wl = self.wl
        P = len(wl.planes)
        if self._bank is not None:
            return self._bank[(7 * n) % wl.bank].copy()
        # fresh fields: generate sequentially so any n is reproducible
        while self._next <= n:
            f = np.empty((P, 3, wl.n1, wl.n3))
            for p in range(P):
                for c in range(3):
                    f[p, c] = shaped_field(self._rngs[p][c], wl.n1, wl.n3, wl.dx1, wl.dx3)
            self._cache[self._next] = f
            self._next += 1
        return self._cache[n].copy()

    def uniform(self, n):
        """[P, 3] spatially uniform part of du^n (the slip ramp on u1; zero otherwise)."""
        wl = self.wl
        out = np.zeros((len(wl.planes), 3))
        if wl.slip_ramp:
            out[:, 0] = wl.slip_ramp * n / max(wl.steps - 1, 1) * wl.dt
        return out

    def varying(self, n):
        """du^n without its uniform part: the random field plus the pulse ramp."""
        wl = self.wl
        du = self._random(n)
        if wl.pulse:
            ramp = lambda m: min(max(m, 0) / 50.0, 1.0)  # noqa: E731
            du[:, 0] += self._gauss * (ramp(n) - ramp(n - 1))
        return du

    def __call__(self, n):
        return self.varying(n) + self.uniform(n)[:, :, None, None]

    def history(self, steps):
        return np.stack([self(n) for n in range(steps)])


def absolute_history(du_hist):
    """u^n = sum_{i<=n} du^i along axis 0."""
    return np.cumsum(du_hist, axis=0)


def step_sources(wl: Workload):
    """(fields, index, uniform) with du^n = fields[index(n)] + uniform(n)[:, :, None, None].

    ``fields`` are the distinct spatially varying increments of the workload
    (bank entries plus the steps that differ from them), ``uniform(n)`` the
    [P, 3] uniform part.  Lets consumers transform each distinct field once.
    """
    inc = Increments(wl)
    fields = []
    special = {}
    n = 0
    while True:
        d = inc.varying(n)
        if inc._bank is not None and n > 0 and np.array_equal(d, inc._bank[(7 * n) % wl.bank]):
            break
        special[n] = len(fields)
        fields.append(d)
        n += 1
        if inc._bank is None and n >= wl.steps:
            break
    base = len(fields)
    if inc._bank is not None:
        fields.extend(inc._bank)

    def index(m):
        if m in special:
            return special[m]
        return base + (7 * m) % wl.bank
    return fields, index, inc.uniform


# ------------------------------------------------------------------ fault runs
#
# Stand-alone boundary-integral dynamic rupture on the plane between two
# half-spaces, with the setup of the paper's TPV3 benchmark (Sec. 3.1): bulk
# rho = 2670 kg/m^3, c_p = 6000 m/s, c_s = 3464 m/s; friction mu_s = 0.677,
# mu_k = 0.525, d_c = 0.4 m; background shear 70 MPa along x1 and normal stress
# 120 MPa (compressive); nucleation over a centred square patch of side 3 km;
# rupture region 30 km x 15 km (Sec. 3.1 setup figure); dx = 50 m (Sec. 3.2).
# Readings where the paper prints no number: the shear stress in the patch is
# (mu_s + 0.005) sigma0, just above the static strength; outside the rupture
# region the fault is locked (a static coefficient of 1e4); the time step is
# c_s dt / dx = 0.25.  Cell centres sit at x = (i - n/2 + 1/2) dx, so the patch
# and the region are symmetric about the grid centre.

TPV3 = dict(rho=2670.0, cp=6000.0, cs=3464.0, mu_s=0.677, mu_k=0.525, d_c=0.4,
            tau0=70.0e6, sigma0=120.0e6, patch=3000.0, region=(30000.0, 15000.0), dx=50.0)
LOCKED_MU_S = 1.0e4


@dataclass
class FaultWorkload:
    name: str
    n1: int
    n3: int
    dx: float
    steps: int
    beta: float = 0.25                       # c_s dt / dx
    region: tuple = TPV3["region"]           # (L1, L3) of the rupture region, m
    patch: float = TPV3["patch"]             # side of the nucleation patch, m
    lower: dict = None                       # material below the fault (None: mirror image)
    window_cap: int = 0                      # 0: the whole run
    window_mode: str = "fixed"
    eta_w: float = 1.0
    excess: float = 0.005                    # patch stress = (mu_s + excess) sigma0
    tau0_3: float = 0.0                      # background shear along x3, Pa

    def upper(self):
        t = TPV3
        return dict(side=1, mu=t["rho"] * t["cs"] ** 2, cs=t["cs"], cp=t["cp"])

    @property
    def dt(self):
        return self.beta * self.dx / TPV3["cs"]

    def planes(self):
        if self.lower is None:
            return [self.upper()]
        return [self.upper(), dict(side=-1, **self.lower)]

    def config_dict(self):
        return dict(n1=self.n1, n3=self.n3, dx1=self.dx, dx3=self.dx, dt=self.dt,
                    planes=self.planes(), window_cap=self.window_cap or self.steps,
                    window_mode=self.window_mode, eta_w=self.eta_w)

    def coords(self):
        x1 = (np.arange(self.n1) - self.n1 / 2 + 0.5) * self.dx
        x3 = (np.arange(self.n3) - self.n3 / 2 + 0.5) * self.dx
        return np.meshgrid(x1, x3, indexing="ij")

    def masks(self):
        X1, X3 = self.coords()
        h = self.patch / 2
        patch = (np.abs(X1) < h) & (np.abs(X3) < h)
        region = (np.abs(X1) < self.region[0] / 2) & (np.abs(X3) < self.region[1] / 2)
        return patch, region

    def params(self):
        """(tau0 [3, n1, n3], mu_s, mu_k, d_c [n1, n3]) float64."""
        t = TPV3
        patch, region = self.masks()
        tau0 = np.zeros((3, self.n1, self.n3))
        tau0[0] = t["tau0"]
        tau0[0][patch] = (t["mu_s"] + self.excess) * t["sigma0"]
        tau0[1] = -t["sigma0"]
        tau0[2] = self.tau0_3
        mu_s = np.where(region, t["mu_s"], LOCKED_MU_S)
        mu_k = np.full((self.n1, self.n3), t["mu_k"])
        d_c = np.full((self.n1, self.n3), t["d_c"])
        return tau0, mu_s, mu_k, d_c


SLOWER = dict(mu=0.64 * TPV3["rho"] * TPV3["cs"] ** 2, cs=0.8 * TPV3["cs"], cp=0.8 * TPV3["cp"])

FAULTS = {
    # the paper's resolution and setup; the periodic images of the rupture
    # region lie 21 km (x1) and 36 km (x3) beyond its edges
    "tpv3_1024": FaultWorkload("tpv3_1024", 1024, 1024, 50.0, 2000),
    # coarse grids for parity with the oracle
    "tpv3_coarse16": FaultWorkload("tpv3_coarse16", 16, 16, 750.0, 80, region=(9000.0, 9000.0)),
    "tpv3_coarse32": FaultWorkload("tpv3_coarse32", 32, 32, 375.0, 150, region=(9000.0, 9000.0)),
    "tpv3_rect32x16": FaultWorkload("tpv3_rect32x16", 32, 16, 375.0, 120, region=(9000.0, 4500.0),
                                    tau0_3=4.0e6),
    "bimaterial32": FaultWorkload("bimaterial32", 32, 32, 375.0, 120, region=(9000.0, 9000.0),
                                  lower=SLOWER),
    # fewer cells than one 64-wide wavefront per strip row block
    "tpv3_tiny8": FaultWorkload("tpv3_tiny8", 8, 8, 750.0, 40, region=(4500.0, 4500.0),
                                patch=1500.0),
}
