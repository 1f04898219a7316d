"""Per-time-step spectral boundary integral update of the exterior half-spaces.

Oracle module: test infrastructure only (see ``oracle/__init__.py``).

What it computes, per boundary plane and per step n (Sec. 2.3, Eq. SBI, with
the nonlocal term evaluated spectrally as described after Eq. SBI; hybrid step
items 2-3 of Sec. 2.4 give the call order: push u^n, then traction tau^n):

1. U^n = DFT(u^n) on the stored half spectrum (``oracle.dft``).  With
   ``input_kind = "increment"`` the input is du^n and U^n = U^{n-1} + DFT(du^n).
2. V^n = DFT(v^n) when a velocity is supplied, else (U^n - U^{n-1}) / dt with
   U^{-1} = 0 (history before the first step is the reference state, Sec. 2.1
   initial conditions).
3. Per mode, rotate (1, 2, 3) -> (L, N, T): L along k, N = e2, T = e2 x L.
4. C_ab^n = sum_{j=0}^{min(n, W(q)-1)} w_ab,j(q) U_b^{n-j} (``oracle.kernels``).
5. Traction of the half-space on side sigma = +1 (on the +x2 side of its plane)
   or -1, with eta = c_p / c_s:
     tau_L = -sigma (mu/c_s) V_L - sigma mu q C11[U_L] + i(2-eta) mu q U_N - i mu q C12[U_N]
     tau_N = -sigma (eta mu/c_s) V_N - sigma mu q C22[U_N] - i(2-eta) mu q U_L + i mu q C12[U_L]
     tau_T = -sigma (mu/c_s) V_T - sigma mu q C33[U_T]
   The damping terms are Eq. SBI's radiation damping with eta_22 = c_p/c_s;
   the lower half-space follows from the upper one by the mirror x2 -> -x2.
6. Rotate back and invert the transform; add the far-field traction tau_inf.

Each operator is built as explicit 3x3 complex matrices per mode (damping D,
instantaneous I, lag matrices K_j) so that the adjoint can take their
conjugate transposes literally.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import dft
from .kernels import kernel_laplace, lag_weights


@dataclass
class Plane:
    side: int = 1          # +1: half-space on the +x2 side of the plane, -1: below
    mu: float = 1.0
    cs: float = 1.0
    cp: float = math.sqrt(3.0)


@dataclass
class Config:
    n1: int
    n3: int
    dx1: float = 1.0
    dx3: float = 1.0
    dt: float = 0.2
    planes: list = field(default_factory=lambda: [Plane()])
    window_cap: int = 100
    window_mode: str = "fixed"        # "fixed" | "per_mode" | "static"
    eta_w: float = 1.0
    input_kind: str = "absolute"      # "absolute" | "increment"

    @staticmethod
    def from_dict(d):
        d = dict(d)
        d["planes"] = [p if isinstance(p, Plane) else Plane(**p) for p in d.get("planes", [{}])]
        return Config(**d)


def wavenumbers(cfg):
    """k1[i1] (signed, Nyquist at -pi/dx1) and k3[i3] (i3 = 0..n3/2, Nyquist at +pi/dx3)."""
    i1 = np.arange(cfg.n1)
    m1 = np.where(i1 < cfg.n1 // 2, i1, i1 - cfg.n1)
    m3 = np.arange(cfg.n3 // 2 + 1)
    k1 = (2.0 * math.pi * m1) / (cfg.n1 * cfg.dx1)
    k3 = (2.0 * math.pi * m3) / (cfg.n3 * cfg.dx3)
    return k1, k3


def mode_geometry(cfg):
    """q, unit wavevector (kh1, kh3) on the [n1, n3/2+1] half spectrum.

    q = sqrt(k1^2 + k3^2); at q = 0 the unit vector is taken as (1, 0).
    """
    k1, k3 = wavenumbers(cfg)
    K1, K3 = np.meshgrid(k1, k3, indexing="ij")
    q = np.sqrt(K1 * K1 + K3 * K3)
    safe = np.where(q > 0, q, 1.0)
    kh1 = np.where(q > 0, K1 / safe, 1.0)
    kh3 = np.where(q > 0, K3 / safe, 0.0)
    return q, kh1, kh3


def mode_window(q, cs, dt, cfg):
    """History length W(q) per mode: fixed cap, or min(cap, ceil(2 pi eta_w / (q c_s dt))),
    or 1 in the quasi-dynamic limit ("static")."""
    q = np.asarray(q, dtype=np.float64)
    if cfg.window_mode == "fixed":
        w = np.full(q.shape, cfg.window_cap, dtype=np.int64)
    elif cfg.window_mode == "static":
        w = np.ones(q.shape, dtype=np.int64)
    elif cfg.window_mode == "per_mode":
        with np.errstate(divide="ignore"):
            x = (2.0 * math.pi * cfg.eta_w) / (q * cs * dt)
        w = np.minimum(cfg.window_cap, np.ceil(np.where(q > 0, x, 0.0))).astype(np.int64)
    else:
        raise ValueError(cfg.window_mode)
    return np.where(q > 0, w, 0)


def _rotation(kh1, kh3):
    """R[..., a, b]: rows (L, N, T), columns (1, 2, 3); real orthogonal."""
    R = np.zeros(kh1.shape + (3, 3))
    R[..., 0, 0] = kh1
    R[..., 0, 2] = kh3
    R[..., 1, 1] = 1.0
    R[..., 2, 0] = -kh3
    R[..., 2, 2] = kh1
    return R


def _to_lab(R, Mrot):
    """R^T Mrot R for a batch of modes."""
    return np.einsum("...ba,...bc,...cd->...ad", R, Mrot, R)


class PlaneOperator:
    """Per-mode matrices of one plane on a chosen set of half-spectrum bins.

    ``modes``: None for every bin, else (i1, i3) index arrays.
    """

    def __init__(self, cfg, p, modes=None, weights_cache=None):
        pl = cfg.planes[p]
        q, kh1, kh3 = mode_geometry(cfg)
        if modes is not None:
            i1, i3 = modes
            q, kh1, kh3 = q[i1, i3], kh1[i1, i3], kh3[i1, i3]
        self.shape = q.shape
        q = q.reshape(-1)
        kh1 = kh1.reshape(-1)
        kh3 = kh3.reshape(-1)
        eta = pl.cp / pl.cs
        sg = float(pl.side)
        mu, cs = pl.mu, pl.cs
        self.W = mode_window(q, cs, cfg.dt, cfg)
        self.Wmax = int(self.W.max()) if self.W.size else 0
        R = _rotation(kh1, kh3)
        nm = q.size

        D = np.zeros((nm, 3, 3), dtype=complex)
        D[:, 0, 0] = -sg * mu / cs
        D[:, 1, 1] = -sg * eta * mu / cs
        D[:, 2, 2] = -sg * mu / cs
        Irot = np.zeros((nm, 3, 3), dtype=complex)
        Irot[:, 0, 1] = 1j * (2.0 - eta) * mu * q
        Irot[:, 1, 0] = -1j * (2.0 - eta) * mu * q
        self.D = _to_lab(R, D)
        self.I = _to_lab(R, Irot)

        # lag weights per distinct (q, W); shape (4, Wmax, nm), zero past W(q)
        cache = {} if weights_cache is None else weights_cache
        w = np.zeros((4, self.Wmax, nm))
        for idx in range(nm):
            Wq = int(self.W[idx])
            if Wq == 0:
                continue
            if cfg.window_mode == "static":
                # quasi-dynamic limit: the whole kernel acts on the current
                # displacement, w_ab,0 = G_ab(infinity) = F_ab(s = 0)
                key = ("static", eta)
                if key not in cache:
                    cache[key] = np.real(np.array(kernel_laplace(0.0, eta)))[:, None]
            else:
                key = (float(q[idx]), cs, cfg.dt, Wq, eta)
                if key not in cache:
                    cache[key] = lag_weights(q[idx], cs, cfg.dt, Wq, eta)
            w[:, :Wq, idx] = cache[key]
        self.K = np.zeros((self.Wmax, nm, 3, 3), dtype=complex)
        if self.Wmax:
            Krot = np.zeros((self.Wmax, nm, 3, 3), dtype=complex)
            Krot[:, :, 0, 0] = -sg * mu * q * w[0]
            Krot[:, :, 0, 1] = -1j * mu * q * w[1]
            Krot[:, :, 1, 0] = +1j * mu * q * w[1]
            Krot[:, :, 1, 1] = -sg * mu * q * w[2]
            Krot[:, :, 2, 2] = -sg * mu * q * w[3]
            self.K = _to_lab(R[None], Krot)

    def apply(self, U_hist, V_hist):
        """tau_hat^n for all n; U_hist, V_hist: [N, 3, nm] complex -> [N, 3, nm].

        Direct convolution: for every step n the lags j = 0..min(n, Wmax-1)
        are summed explicitly (K_j is zero past each mode's own W(q)).
        """
        N = U_hist.shape[0]
        out = np.einsum("mab,nbm->nam", self.I, U_hist) + np.einsum("mab,nbm->nam", self.D, V_hist)
        for n in range(N):
            L = min(n + 1, self.Wmax)
            if L:
                past = U_hist[n - L + 1:n + 1][::-1]          # U^{n-j}, j = 0..L-1
                out[n] += np.einsum("jmab,jbm->am", self.K[:L], past, optimize=True)
        return out

    def apply_last(self, U_hist, V_last):
        """tau_hat of the last step only: the same direct sum as ``apply`` for n = N-1."""
        N = U_hist.shape[0]
        out = np.einsum("mab,bm->am", self.I, U_hist[-1]) + np.einsum("mab,bm->am", self.D, V_last)
        L = min(N, self.Wmax)
        if L:
            past = U_hist[N - L:][::-1]
            out += np.einsum("jmab,jbm->am", self.K[:L], past, optimize=True)
        return out

    def apply_adjoint(self, G_hist):
        """(lam_U, lam_V): the conjugate-transposed operators run backwards in time.

        lam_U^m = sum_j K_j^H G^{m+j} + I^H G^m,   lam_V^m = D^H G^m.
        """
        N = G_hist.shape[0]
        Ih = np.conj(np.swapaxes(self.I, -1, -2))
        Dh = np.conj(np.swapaxes(self.D, -1, -2))
        Kh = np.conj(np.swapaxes(self.K, -1, -2))
        lam_u = np.einsum("mab,nbm->nam", Ih, G_hist)
        lam_v = np.einsum("mab,nbm->nam", Dh, G_hist)
        for m in range(N):
            L = min(N - m, self.Wmax)
            if L:
                future = G_hist[m:m + L]                      # G^{m+j}, j = 0..L-1
                lam_u[m] += np.einsum("jmab,jbm->am", Kh[:L], future, optimize=True)
        return lam_u, lam_v


def _check(cfg, arr, name):
    P = len(cfg.planes)
    if arr.ndim != 5 or arr.shape[1:] != (P, 3, cfg.n1, cfg.n3):
        raise ValueError(f"{name}: expected [N, {P}, 3, {cfg.n1}, {cfg.n3}], got {arr.shape}")


def spectra(cfg, u_hist, v_hist=None):
    """Displacement and velocity spectra U^n, V^n: [N, P, 3, n1, n3/2+1] complex."""
    u_hist = np.asarray(u_hist, dtype=np.float64)
    _check(cfg, u_hist, "u_hist")
    X = dft.forward_half(u_hist)
    if cfg.input_kind == "increment":
        U = np.cumsum(X, axis=0)
        V = X / cfg.dt
    elif cfg.input_kind == "absolute":
        U = X
        prev = np.concatenate([np.zeros_like(X[:1]), X[:-1]], axis=0)
        V = (X - prev) / cfg.dt
    else:
        raise ValueError(cfg.input_kind)
    if v_hist is not None:
        v_hist = np.asarray(v_hist, dtype=np.float64)
        _check(cfg, v_hist, "v_hist")
        V = dft.forward_half(v_hist)
    return U, V


def _mode_chunks(cfg, chunk):
    """Flat half-spectrum bins split into (i1, i3) index chunks."""
    h = cfg.n3 // 2 + 1
    flat = np.arange(cfg.n1 * h)
    for s in range(0, flat.size, chunk):
        f = flat[s:s + chunk]
        yield f, (f // h, f % h)


def _chunk_size(cfg, chunk):
    """Bound the per-chunk lag-matrix storage (Wcap * chunk * 144 B) to ~0.5 GB."""
    if chunk is not None:
        return chunk
    return int(max(64, min(8192, 5e8 // (144 * max(cfg.window_cap, 1)))))


def forward(cfg, u_hist, v_hist=None, tau_inf_hist=None, chunk=None, weights_cache=None):
    """Tractions tau^n for n = 0..N-1: [N, P, 3, n1, n3] float64."""
    if not isinstance(cfg, Config):
        cfg = Config.from_dict(cfg)
    U, V = spectra(cfg, u_hist, v_hist)
    N, P = U.shape[:2]
    h = cfg.n3 // 2 + 1
    cache = {} if weights_cache is None else weights_cache
    tau_hat = np.empty((N, P, 3, cfg.n1 * h), dtype=complex)
    Uf = U.reshape(N, P, 3, -1)
    Vf = V.reshape(N, P, 3, -1)
    for p in range(P):
        for f, modes in _mode_chunks(cfg, _chunk_size(cfg, chunk)):
            op = PlaneOperator(cfg, p, modes, cache)
            tp = tau_hat[:, p]
            tp[:, :, f] = op.apply(Uf[:, p][:, :, f], Vf[:, p][:, :, f])
    tau = dft.inverse_half(tau_hat.reshape(N, P, 3, cfg.n1, h), cfg.n3)
    if tau_inf_hist is not None:
        tau = tau + np.asarray(tau_inf_hist, dtype=np.float64)
    return tau


def _input_chain(cfg, lam_u, lam_v, with_velocity):
    """Transpose of ``spectra``'s definitions of U^n and V^n (time on axis 0).

    lam_u, lam_v: dL/dU^n and dL/dV^n; returns the spectra of dL/du^n and
    dL/dv^n (None without an explicit velocity).
    """
    if with_velocity:
        dv_hat = lam_v
        du_hat = lam_u
    else:
        dv_hat = None
        if cfg.input_kind == "absolute":
            nxt = np.concatenate([lam_v[1:], np.zeros_like(lam_v[:1])], axis=0)
            du_hat = lam_u + (lam_v - nxt) / cfg.dt
        else:
            du_hat = lam_u.copy()
    if cfg.input_kind == "increment":
        du_hat = np.flip(np.cumsum(np.flip(du_hat, axis=0), axis=0), axis=0)
        if not with_velocity:
            du_hat = du_hat + lam_v / cfg.dt
    return du_hat, dv_hat


def adjoint(cfg, g_hist, with_velocity=False, chunk=None, weights_cache=None):
    """Transpose of ``forward`` applied to g = dL/dtau (tau_inf excluded).

    Returns dL/du (with respect to whatever ``input_kind`` says u is) and,
    when ``with_velocity``, dL/dv for an explicitly supplied velocity.
    """
    if not isinstance(cfg, Config):
        cfg = Config.from_dict(cfg)
    g_hist = np.asarray(g_hist, dtype=np.float64)
    _check(cfg, g_hist, "g_hist")
    G = dft.forward_half(g_hist)
    N, P = G.shape[:2]
    h = cfg.n3 // 2 + 1
    cache = {} if weights_cache is None else weights_cache
    lam_u = np.empty((N, P, 3, cfg.n1 * h), dtype=complex)
    lam_v = np.empty_like(lam_u)
    Gf = G.reshape(N, P, 3, -1)
    for p in range(P):
        for f, modes in _mode_chunks(cfg, _chunk_size(cfg, chunk)):
            op = PlaneOperator(cfg, p, modes, cache)
            lu, lv = op.apply_adjoint(Gf[:, p][:, :, f])
            lup, lvp = lam_u[:, p], lam_v[:, p]
            lup[:, :, f] = lu
            lvp[:, :, f] = lv
    lam_u = lam_u.reshape(N, P, 3, cfg.n1, h)
    lam_v = lam_v.reshape(N, P, 3, cfg.n1, h)
    du_hat, dv_hat = _input_chain(cfg, lam_u, lam_v, with_velocity)
    du = dft.inverse_half(du_hat, cfg.n3)
    dv = dft.inverse_half(dv_hat, cfg.n3) if dv_hat is not None else None
    return du, dv


def mode_response(cfg, p, bins, U_hist, V_hist, weights_cache=None):
    """tau_hat of plane p at selected half-spectrum bins, every step.

    bins: (i1, i3) index arrays; U_hist, V_hist: [N, 3, len(bins)] spectra of
    the displacement and velocity at those bins (as ``spectra`` defines them).
    Returns [N, 3, len(bins)] in the (x1, x2, x3) frame.
    """
    if not isinstance(cfg, Config):
        cfg = Config.from_dict(cfg)
    op = PlaneOperator(cfg, p, bins, weights_cache)
    return op.apply(np.asarray(U_hist, dtype=complex), np.asarray(V_hist, dtype=complex))


def adjoint_response(cfg, p, bins, G_hist, with_velocity=False, weights_cache=None):
    """Spectra of dL/du (and dL/dv) of plane p at selected bins, every step.

    G_hist: [N, 3, len(bins)] spectrum of g = dL/dtau at those bins; the same
    transpose as ``adjoint`` restricted to the bins.
    """
    if not isinstance(cfg, Config):
        cfg = Config.from_dict(cfg)
    op = PlaneOperator(cfg, p, bins, weights_cache)
    lam_u, lam_v = op.apply_adjoint(np.asarray(G_hist, dtype=complex))
    return _input_chain(cfg, lam_u, lam_v, with_velocity)
