"""Thin Python binding of the HIP boundary-integral library (``include/sbim.h``).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch supplies device memory and the current HIP stream.  The
library must be built (``paper_2102_08756_amd.build``); importing this module
without it raises instead of falling back to anything.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# SBIM_LIBRARY selects another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("SBIM_LIBRARY") or os.path.join(_HERE, "_lib", "libsbim.so")

SBIM_OK, SBIM_E_INVALID, SBIM_E_OOM, SBIM_E_STATE, SBIM_E_DEVICE = 0, -1, -2, -3, -4
PRECISIONS = {"fp64": 0, "fp32": 1, "fp32_comp": 2}
WINDOW_MODES = {"fixed": 0, "per_mode": 1, "static": 2}
INPUT_KINDS = {"absolute": 0, "increment": 1}
ERROR_NAMES = {SBIM_E_INVALID: "SBIM_E_INVALID", SBIM_E_OOM: "SBIM_E_OOM",
               SBIM_E_STATE: "SBIM_E_STATE", SBIM_E_DEVICE: "SBIM_E_DEVICE"}

# every symbol the header declares
EXPORTS = (
    "sbim_init", "sbim_push_displacement", "sbim_tractions", "sbim_backward",
    "sbim_backward_reset", "sbim_reset", "sbim_destroy", "sbim_last_error", "sbim_set_stream",
    "sbim_set_dt", "sbim_count_nonfinite", "sbim_count_nonfinite_noalloc", "sbim_traction_spectrum",
    "sbim_get_info", "sbim_state_bytes", "sbim_save_state", "sbim_load_state",
    "sbim_running_state_bytes", "sbim_save_running_state", "sbim_load_running_state", "sbim_step_work",
    "sbim_mode_kernel", "sbim_profile_conv", "sbim_conv_timing",
    "sbim_fault_create", "sbim_fault_step", "sbim_fault_read", "sbim_fault_reset",
    "sbim_fault_destroy", "sbim_strip_create", "sbim_strip_step", "sbim_strip_read",
    "sbim_strip_reset", "sbim_strip_destroy",
)
STRIP_FIELDS = {"traction": (0, 3), "slip_rate": (1, 2), "slip": (2, 2), "sliding": (3, 1),
                "displacement": (4, None), "velocity": (5, None)}
FAULT_FIELDS = {"traction": (0, 3), "slip_rate": (1, 2), "slip": (2, 2), "displacement": (3, 6),
                "velocity": (4, 6)}


class _Plane(ctypes.Structure):
    _fields_ = [("side", ctypes.c_int), ("mu", ctypes.c_double), ("cs", ctypes.c_double),
                ("cp", ctypes.c_double)]


class _Config(ctypes.Structure):
    _fields_ = [("n1", ctypes.c_int), ("n3", ctypes.c_int), ("dx1", ctypes.c_double),
                ("dx3", ctypes.c_double), ("dt", ctypes.c_double), ("nplanes", ctypes.c_int),
                ("plane", _Plane * 2), ("window_cap", ctypes.c_int), ("window_mode", ctypes.c_int),
                ("eta_w", ctypes.c_double), ("precision", ctypes.c_int),
                ("input_kind", ctypes.c_int), ("stream", ctypes.c_void_p)]


class _Info(ctypes.Structure):
    _fields_ = [("modes_per_plane", ctypes.c_longlong), ("kernel_classes", ctypes.c_longlong),
                ("ring_bytes", ctypes.c_longlong), ("table_bytes", ctypes.c_longlong),
                ("state_bytes", ctypes.c_longlong), ("step", ctypes.c_longlong),
                ("backward_step", ctypes.c_longlong), ("material_groups", ctypes.c_int),
                ("sweep_depth", ctypes.c_int), ("sweep_matrix_cores", ctypes.c_int),
                ("sweep_lag_chunks", ctypes.c_int), ("sweep_quads", ctypes.c_int)]


class _FaultParams(ctypes.Structure):
    _fields_ = [("tau0", ctypes.c_void_p), ("mu_s", ctypes.c_void_p), ("mu_k", ctypes.c_void_p),
                ("d_c", ctypes.c_void_p)]


class _StripConfig(ctypes.Structure):
    _fields_ = [("layers", ctypes.c_int), ("rho", ctypes.POINTER(ctypes.c_double)),
                ("cp", ctypes.POINTER(ctypes.c_double)), ("cs", ctypes.POINTER(ctypes.c_double)),
                ("layers_below", ctypes.c_int), ("rho_below", ctypes.POINTER(ctypes.c_double)),
                ("cp_below", ctypes.POINTER(ctypes.c_double)),
                ("cs_below", ctypes.POINTER(ctypes.c_double))]


_lib = None


def load_library(path=LIB_PATH):
    """Load the built library and declare its C signatures (fails loudly when absent)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build the HIP library first "
                           "(python -c 'import __graft_entry__ as g; g.build()')")
    L = ctypes.CDLL(path)
    vp, i, ll, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_longlong, ctypes.c_double
    sig = {
        "sbim_init": (i, [ctypes.POINTER(_Config), ctypes.POINTER(vp)]),
        "sbim_push_displacement": (i, [vp, vp, vp]),
        "sbim_tractions": (i, [vp, vp, vp]),
        "sbim_backward": (i, [vp, vp, vp, vp]),
        "sbim_backward_reset": (i, [vp]),
        "sbim_reset": (i, [vp]),
        "sbim_destroy": (i, [vp]),
        "sbim_last_error": (ctypes.c_char_p, [vp]),
        "sbim_set_stream": (i, [vp, vp]),
        "sbim_set_dt": (i, [vp, d]),
        "sbim_get_info": (i, [vp, ctypes.POINTER(_Info)]),
        "sbim_count_nonfinite": (i, [vp, vp, ctypes.POINTER(ll)]),
        "sbim_count_nonfinite_noalloc": (i, [vp, vp, vp]),
        "sbim_traction_spectrum": (i, [vp, vp]),
        "sbim_state_bytes": (ll, [vp]),
        "sbim_running_state_bytes": (ll, [vp]),
        "sbim_save_running_state": (i, [vp, vp]),
        "sbim_load_running_state": (i, [vp, vp]),
        "sbim_save_state": (i, [vp, vp]),
        "sbim_load_state": (i, [vp, vp]),
        "sbim_step_work": (i, [vp, ll, ctypes.POINTER(d), ctypes.POINTER(d)]),
        "sbim_mode_kernel": (i, [vp, i, i, i, ctypes.POINTER(d), i]),
        "sbim_profile_conv": (i, [vp, i]),
        "sbim_conv_timing": (i, [vp, ctypes.POINTER(d), ctypes.POINTER(ll)]),
        "sbim_fault_create": (i, [vp, ctypes.POINTER(_FaultParams), ctypes.POINTER(vp)]),
        "sbim_fault_step": (i, [vp, vp, vp]),
        "sbim_fault_read": (i, [vp, i, vp]),
        "sbim_fault_reset": (i, [vp]),
        "sbim_fault_destroy": (i, [vp]),
        "sbim_strip_create": (i, [vp, ctypes.POINTER(_StripConfig), ctypes.POINTER(_FaultParams),
                                  ctypes.POINTER(vp)]),
        "sbim_strip_step": (i, [vp, vp, vp]),
        "sbim_strip_read": (i, [vp, i, vp]),
        "sbim_strip_reset": (i, [vp]),
        "sbim_strip_destroy": (i, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


class SBIMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


@dataclass
class Plane:
    side: int = 1
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
    window_mode: str = "fixed"
    eta_w: float = 1.0
    precision: str = "fp64"
    input_kind: str = "absolute"

    @staticmethod
    def from_dict(d, **overrides):
        d = dict(d)
        d.update(overrides)
        d["planes"] = [p if isinstance(p, Plane) else Plane(**p) for p in d.get("planes", [{}])]
        return Config(**d)

    @property
    def dtype(self):
        return torch.float64 if self.precision == "fp64" else torch.float32


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class SBIM:
    """One library handle: the exterior half-spaces of one or two boundary planes."""

    def __init__(self, cfg: Config, device=None):
        self.cfg = cfg
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self._L = load_library()
        c = _Config()
        c.n1, c.n3, c.dx1, c.dx3, c.dt = cfg.n1, cfg.n3, cfg.dx1, cfg.dx3, cfg.dt
        c.nplanes = len(cfg.planes)
        if not 1 <= c.nplanes <= 2:
            raise ValueError("one or two planes")
        for k, p in enumerate(cfg.planes):
            c.plane[k] = _Plane(int(p.side), float(p.mu), float(p.cs), float(p.cp))
        c.window_cap = int(cfg.window_cap)
        c.window_mode = WINDOW_MODES[cfg.window_mode]
        c.eta_w = float(cfg.eta_w)
        c.precision = PRECISIONS[cfg.precision]
        c.input_kind = INPUT_KINDS[cfg.input_kind]
        with torch.cuda.device(self.device):
            self._stream = torch.cuda.current_stream(self.device)
            c.stream = ctypes.c_void_p(self._stream.cuda_stream)
            h = ctypes.c_void_p()
            rc = self._L.sbim_init(ctypes.byref(c), ctypes.byref(h))
        if rc != SBIM_OK:
            raise SBIMError(rc, self._L.sbim_last_error(None).decode())
        self._h = h
        self.dtype = cfg.dtype
        self.P = c.nplanes
        self.shape = (self.P, 3, cfg.n1, cfg.n3)

    # -------------------------------------------------------------- helpers
    def _check(self, rc):
        if rc != SBIM_OK:
            raise SBIMError(rc, self._L.sbim_last_error(self._h).decode())

    def _sync_stream(self):
        s = torch.cuda.current_stream(self.device)
        if s.cuda_stream != self._stream.cuda_stream:
            self._stream = s
            self._check(self._L.sbim_set_stream(self._h, ctypes.c_void_p(s.cuda_stream)))

    def _field(self, t, name, allow_none=False):
        if t is None:
            if allow_none:
                return None
            raise ValueError(f"{name} is required")
        if not isinstance(t, torch.Tensor) or t.device != self.device:
            raise ValueError(f"{name}: expected a tensor on {self.device}")
        if tuple(t.shape) != self.shape or t.dtype != self.dtype or not t.is_contiguous():
            raise ValueError(f"{name}: expected contiguous {self.dtype} {self.shape}, got "
                             f"{t.dtype} {tuple(t.shape)} contiguous={t.is_contiguous()}")
        return t

    def new_field(self):
        return torch.empty(self.shape, dtype=self.dtype, device=self.device)

    # ------------------------------------------------------------- the ABI
    def push(self, u, v=None):
        self._field(u, "u")
        self._field(v, "v", allow_none=True)
        self._sync_stream()
        self._check(self._L.sbim_push_displacement(self._h, _ptr(u), _ptr(v)))

    def tractions(self, tau_inf=None, out=None):
        self._field(tau_inf, "tau_inf", allow_none=True)
        out = self.new_field() if out is None else self._field(out, "out")
        self._sync_stream()
        self._check(self._L.sbim_tractions(self._h, _ptr(tau_inf), _ptr(out)))
        return out

    def step(self, u, v=None, tau_inf=None, out=None):
        self.push(u, v)
        return self.tractions(tau_inf, out)

    def backward(self, g, du=None, dv=None, with_velocity=False):
        """One reverse step: returns dL/du (and dL/dv when ``with_velocity``)."""
        self._field(g, "dL_dtau")
        du = self.new_field() if du is None else self._field(du, "dL_du")
        if with_velocity and dv is None:
            dv = self.new_field()
        self._field(dv, "dL_dv", allow_none=True)
        self._sync_stream()
        self._check(self._L.sbim_backward(self._h, _ptr(g), _ptr(du), _ptr(dv)))
        return (du, dv) if with_velocity else du

    def count_nonfinite(self, field):
        """Infinities and NaNs in a [P][3][n1][n3] field of the handle's dtype (library
        kernel; synchronises)."""
        self._field(field, "field")
        n = ctypes.c_longlong(0)
        self._sync_stream()
        self._check(self._L.sbim_count_nonfinite(self._h, _ptr(field), ctypes.byref(n)))
        return n.value

    def count_nonfinite_noalloc(self, field, out):
        """The same count written to ``out`` (a one-element int64 tensor on the handle's
        device) without any device allocation; asynchronous on the current stream."""
        self._field(field, "field")
        if (not isinstance(out, torch.Tensor) or out.device != self.device
                or out.dtype != torch.int64 or out.numel() < 1):
            raise ValueError(f"out: expected an int64 tensor of at least one element on {self.device}")
        self._sync_stream()
        self._check(self._L.sbim_count_nonfinite_noalloc(self._h, _ptr(field), _ptr(out)))
        return out

    def traction_spectrum(self, out=None):
        """Traction spectrum of the last push: complex [P, 3, n3/2+1, n1] (complex64 for the
        float32 forms), before tau_inf and the inverse transform."""
        ct = torch.complex128 if self.dtype == torch.float64 else torch.complex64
        shape = (self.P, 3, self.cfg.n3 // 2 + 1, self.cfg.n1)
        if out is None:
            out = torch.empty(shape, dtype=ct, device=self.device)
        if tuple(out.shape) != shape or out.dtype != ct or not out.is_contiguous() or out.device != self.device:
            raise ValueError(f"out: expected contiguous {ct} {shape} on {self.device}")
        self._sync_stream()
        self._check(self._L.sbim_traction_spectrum(self._h, _ptr(out)))
        return out

    def set_dt(self, dt):
        """Time step of the following pushes (quasi-dynamic handles only)."""
        self._check(self._L.sbim_set_dt(self._h, float(dt)))

    def backward_reset(self):
        self._sync_stream()
        self._check(self._L.sbim_backward_reset(self._h))

    def reset(self):
        self._sync_stream()
        self._check(self._L.sbim_reset(self._h))

    def info(self):
        i = _Info()
        self._check(self._L.sbim_get_info(self._h, ctypes.byref(i)))
        return {k: getattr(i, k) for k, _ in _Info._fields_}

    def state_bytes(self):
        return int(self._L.sbim_state_bytes(self._h))

    def save_state(self, buf=None):
        if buf is None:
            buf = torch.empty(self.state_bytes(), dtype=torch.uint8, device=self.device)
        if buf.numel() < self.state_bytes() or buf.device != self.device:
            raise ValueError("snapshot buffer too small or on the wrong device")
        self._sync_stream()
        self._check(self._L.sbim_save_state(self._h, _ptr(buf)))
        return buf

    def load_state(self, buf):
        if buf.numel() < self.state_bytes() or buf.device != self.device:
            raise ValueError("snapshot buffer too small or on the wrong device")
        self._sync_stream()
        self._check(self._L.sbim_load_state(self._h, _ptr(buf)))

    def running_state_bytes(self):
        return int(self._L.sbim_running_state_bytes(self._h))

    def save_running_state(self, buf=None):
        """Light snapshot: the float64 running state and the step counter only."""
        if buf is None:
            buf = torch.empty(self.running_state_bytes(), dtype=torch.uint8, device=self.device)
        if buf.numel() < self.running_state_bytes() or buf.device != self.device:
            raise ValueError("snapshot buffer too small or on the wrong device")
        self._sync_stream()
        self._check(self._L.sbim_save_running_state(self._h, _ptr(buf)))
        return buf

    def load_running_state(self, buf):
        """Restore a light snapshot; the history ring and pending sums start empty, so the
        next W_cap + sweep_depth + 2 pushes rebuild what the tractions need."""
        if buf.numel() < self.running_state_bytes() or buf.device != self.device:
            raise ValueError("snapshot buffer too small or on the wrong device")
        self._sync_stream()
        self._check(self._L.sbim_load_running_state(self._h, _ptr(buf)))

    def replay_steps(self):
        """Pushes that rebuild the history after load_running_state: W_cap + sweep_depth + 2."""
        return int(self.cfg.window_cap) + int(self.info()["sweep_depth"]) + 2

    def step_work(self, n):
        a, b = ctypes.c_double(), ctypes.c_double()
        self._check(self._L.sbim_step_work(self._h, int(n), ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def mode_kernel(self, p, i1, i3, max_lags):
        import numpy as np
        buf = (ctypes.c_double * (4 * max(max_lags, 1)))()
        rc = self._L.sbim_mode_kernel(self._h, p, i1, i3, buf, max_lags)
        if rc < 0:
            self._check(rc)
        w = np.frombuffer(buf, dtype=np.float64).reshape(4, max(max_lags, 1))[:, :min(rc, max_lags)]
        return rc, w.copy()

    def profile_conv(self, enable=True, every=1):
        """Time every ``every``-th step launch with HIP events (all of them by default);
        ``enable=False`` turns the timing off."""
        self._check(self._L.sbim_profile_conv(self._h, int(every) if enable else 0))

    def conv_timing(self):
        ms, n = ctypes.c_double(), ctypes.c_longlong()
        self._check(self._L.sbim_conv_timing(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def close(self):
        if getattr(self, "_h", None):
            self._L.sbim_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ fault

class Fault:
    """Frictional fault between plane 0 (above, side +1) and plane 1 (below,
    side -1) of ``sbim``, or plane 0's mirror image when it has one plane.

    tau0 [3, n1, n3], mu_s, mu_k, d_c [n1, n3]: float64 tensors on the handle's
    device (copied).  Each ``step`` is one explicit step of the library's
    interface solve (``sbim_fault_step``); fields are float64 [rows, n1, n3].
    """

    def __init__(self, sbim: SBIM, tau0, mu_s, mu_k, d_c):
        self.sbim = sbim
        n1, n3 = sbim.cfg.n1, sbim.cfg.n3
        shapes = {"tau0": (3, n1, n3), "mu_s": (n1, n3), "mu_k": (n1, n3), "d_c": (n1, n3)}
        args = {"tau0": tau0, "mu_s": mu_s, "mu_k": mu_k, "d_c": d_c}
        for k, t in args.items():
            if (not isinstance(t, torch.Tensor) or t.device != sbim.device or t.dtype != torch.float64
                    or tuple(t.shape) != shapes[k] or not t.is_contiguous()):
                raise ValueError(f"{k}: expected a contiguous float64 {shapes[k]} tensor on {sbim.device}")
        self.cells = (n1, n3)
        p = _FaultParams(*(ctypes.c_void_p(args[k].data_ptr()) for k in ("tau0", "mu_s", "mu_k", "d_c")))
        sbim._sync_stream()
        f = ctypes.c_void_p()
        sbim._check(sbim._L.sbim_fault_create(sbim._h, ctypes.byref(p), ctypes.byref(f)))
        self._f = f

    def _out(self, t, rows, name):
        if t is None:
            return None
        shape = (rows,) + self.cells
        if (not isinstance(t, torch.Tensor) or t.device != self.sbim.device or t.dtype != torch.float64
                or tuple(t.shape) != shape or not t.is_contiguous()):
            raise ValueError(f"{name}: expected a contiguous float64 {shape} tensor")
        return t

    def step(self, tau=None, slip_rate=None):
        self._out(tau, 3, "tau")
        self._out(slip_rate, 2, "slip_rate")
        self.sbim._sync_stream()
        self.sbim._check(self.sbim._L.sbim_fault_step(self._f, _ptr(tau), _ptr(slip_rate)))

    def read(self, name):
        fid, rows = FAULT_FIELDS[name]
        out = torch.empty((rows,) + self.cells, dtype=torch.float64, device=self.sbim.device)
        self.sbim._sync_stream()
        self.sbim._check(self.sbim._L.sbim_fault_read(self._f, fid, _ptr(out)))
        return out

    def run(self, steps):
        """``steps`` steps; returns the traction [N, 3, n1, n3] and slip-rate
        [N, 2, n1, n3] histories (device)."""
        tau = torch.empty((steps, 3) + self.cells, dtype=torch.float64, device=self.sbim.device)
        rate = torch.empty((steps, 2) + self.cells, dtype=torch.float64, device=self.sbim.device)
        for n in range(steps):
            self.step(tau[n], rate[n])
        return tau, rate

    def reset(self):
        self.sbim._sync_stream()
        self.sbim._check(self.sbim._L.sbim_fault_reset(self._f))

    def close(self):
        if getattr(self, "_f", None):
            self.sbim._L.sbim_fault_destroy(self._f)
            self._f = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Strip(Fault):
    """Hybrid scheme: a finite-element strip of ``layers`` (list of (rho, c_p, c_s),
    fault side first) on the fault, closed at S+ by the single plane of ``sbim``
    (``sbim_strip_*``).  With ``layers_below`` (same form, fault side first) the
    strip is two-sided: a split-node fault between two blocks, closed at S+ and
    S- by the two planes (sides +1, -1) of ``sbim``.  Fault parameters as for
    ``Fault``."""

    def __init__(self, sbim: SBIM, layers, tau0, mu_s, mu_k, d_c, layers_below=None):
        self.sbim = sbim
        n1, n3 = sbim.cfg.n1, sbim.cfg.n3
        self.cells = (n1, n3)
        below = list(layers_below or [])
        self.n2 = len(layers) + (len(below) + 1 if below else 0)   # top storage node layer
        args = {"tau0": tau0, "mu_s": mu_s, "mu_k": mu_k, "d_c": d_c}
        shapes = {"tau0": (3, n1, n3), "mu_s": (n1, n3), "mu_k": (n1, n3), "d_c": (n1, n3)}
        for k, t in args.items():
            if (not isinstance(t, torch.Tensor) or t.device != sbim.device or t.dtype != torch.float64
                    or tuple(t.shape) != shapes[k] or not t.is_contiguous()):
                raise ValueError(f"{k}: expected a contiguous float64 {shapes[k]} tensor on {sbim.device}")
        def host(rows):
            return [ctypes.cast((ctypes.c_double * max(len(rows), 1))(*[float(L[i]) for L in rows]),
                                ctypes.POINTER(ctypes.c_double)) for i in range(3)]
        self._host = (host(layers), host(below))          # kept alive until the call returns
        nul = ctypes.POINTER(ctypes.c_double)()
        sc = _StripConfig(len(layers), *self._host[0], len(below),
                          *(self._host[1] if below else (nul, nul, nul)))
        p = _FaultParams(*(ctypes.c_void_p(args[k].data_ptr()) for k in ("tau0", "mu_s", "mu_k", "d_c")))
        sbim._sync_stream()
        f = ctypes.c_void_p()
        sbim._check(sbim._L.sbim_strip_create(sbim._h, ctypes.byref(sc), ctypes.byref(p), ctypes.byref(f)))
        self._f = f

    def step(self, tau=None, slip_rate=None):
        self._out(tau, 3, "tau")
        self._out(slip_rate, 2, "slip_rate")
        self.sbim._sync_stream()
        self.sbim._check(self.sbim._L.sbim_strip_step(self._f, _ptr(tau), _ptr(slip_rate)))

    def read(self, name):
        fid, rows = STRIP_FIELDS[name]
        shape = (rows,) + self.cells if rows else (3, self.n2 + 1) + self.cells
        out = torch.empty(shape, dtype=torch.float64, device=self.sbim.device)
        self.sbim._sync_stream()
        self.sbim._check(self.sbim._L.sbim_strip_read(self._f, fid, _ptr(out)))
        return out

    def reset(self):
        self.sbim._sync_stream()
        self.sbim._check(self.sbim._L.sbim_strip_reset(self._f))

    def close(self):
        if getattr(self, "_f", None):
            self.sbim._L.sbim_strip_destroy(self._f)
            self._f = None


# ------------------------------------------------------------------ autograd

class SBIMRun(torch.autograd.Function):
    """tau_hist = SBIMRun.apply(sbim, u_hist[, v_hist]) over N steps from a reset handle.

    The backward runs the library's transpose (``sbim_backward``) over
    n = N-1 .. 0; the operator is linear, so nothing of the forward is kept.
    """

    @staticmethod
    def forward(ctx, sbim: SBIM, u_hist, v_hist=None):
        sbim.reset()
        N = u_hist.shape[0]
        out = torch.empty((N,) + sbim.shape, dtype=sbim.dtype, device=sbim.device)
        for n in range(N):
            sbim.push(u_hist[n].contiguous(), None if v_hist is None else v_hist[n].contiguous())
            sbim.tractions(out=out[n])
        ctx.sbim = sbim
        ctx.with_v = v_hist is not None
        return out

    @staticmethod
    def backward(ctx, g_hist):
        sbim = ctx.sbim
        sbim.backward_reset()
        N = g_hist.shape[0]
        du = torch.empty_like(g_hist)
        dv = torch.empty_like(g_hist) if ctx.with_v else None
        g_hist = g_hist.contiguous()
        for n in range(N - 1, -1, -1):
            sbim.backward(g_hist[n], du=du[n], dv=dv[n] if dv is not None else None,
                          with_velocity=ctx.with_v)
        return None, du, dv


class _CheckpointedLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sbim, every, loss_fn, u_hist, v_hist):
        sbim.reset()
        N = u_hist.shape[0]
        R = sbim.replay_steps()
        nseg = (N + every - 1) // every
        # segment [a, a + every) is recomputed from the running state of step max(0, a - R)
        starts = sorted({max(0, seg * every - R) for seg in range(nseg)})
        snaps = {}
        total = torch.zeros((), dtype=sbim.dtype, device=sbim.device)
        tau = sbim.new_field()
        for n in range(N):
            if n in starts:
                snaps[n] = sbim.save_running_state()
            sbim.push(u_hist[n].contiguous(), None if v_hist is None else v_hist[n].contiguous())
            sbim.tractions(out=tau)
            total = total + loss_fn(tau, n).detach()
        ctx.sbim, ctx.every, ctx.loss_fn, ctx.snaps, ctx.R = sbim, every, loss_fn, snaps, R
        ctx.save_for_backward(u_hist, v_hist if v_hist is not None else torch.empty(0))
        ctx.with_v = v_hist is not None
        return total

    @staticmethod
    def backward(ctx, gout):
        sbim, every, loss_fn, R = ctx.sbim, ctx.every, ctx.loss_fn, ctx.R
        u_hist, v_hist = ctx.saved_tensors
        v_hist = v_hist if ctx.with_v else None
        N = u_hist.shape[0]
        du = torch.empty_like(u_hist)
        dv = torch.empty_like(u_hist) if ctx.with_v else None

        def push(n):
            sbim.push(u_hist[n].contiguous(), None if v_hist is None else v_hist[n].contiguous())
        sbim.backward_reset()
        for seg in range((N - 1) // every, -1, -1):
            a, b = seg * every, min(N, (seg + 1) * every)
            n0 = max(0, a - R)
            sbim.load_running_state(ctx.snaps[n0])
            for n in range(n0, a):               # rebuild the history the segment reads
                push(n)
            taus = []
            for n in range(a, b):                # recompute this segment's tractions
                push(n)
                taus.append(sbim.tractions())
            for n in range(b - 1, a - 1, -1):
                t = taus[n - a].detach().requires_grad_(True)
                with torch.enable_grad():
                    (g,) = torch.autograd.grad(loss_fn(t, n), t)
                g = (g * gout).contiguous()
                sbim.backward(g, du=du[n], dv=dv[n] if dv is not None else None,
                              with_velocity=ctx.with_v)
        return None, None, None, du, dv


def checkpointed_loss(sbim: SBIM, u_hist, loss_fn, every=50, v_hist=None):
    """L = sum_n loss_fn(tau^n, n) without keeping tau^n.

    The forward keeps, per segment of ``every`` steps starting at step a, a light
    snapshot of the running state of step max(0, a - R), R = W_cap + sweep_depth + 2
    (``SBIM.replay_steps``): the float64 displacement spectrum and the step counter,
    ``running_state_bytes()`` each.  The backward restores it, pushes steps
    a - R .. a - 1 again to rebuild the history the truncated convolution reads, then
    recomputes the segment's tractions (bit for bit the forward's) and runs the
    library's transpose over them in reverse.  Memory: N / every snapshots of the
    running state instead of N traction fields (SBIMRun); cost: up to R + every
    pushes per segment in the backward, so ``every`` >= W_cap keeps the recomputation
    within twice the forward.  The handle's forward state is left at the end of the
    first segment afterwards."""
    return _CheckpointedLoss.apply(sbim, int(every), loss_fn, u_hist, v_hist)
