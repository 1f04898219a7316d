"""Naive discrete Fourier transforms on one boundary plane.

Oracle module: test infrastructure only (see ``oracle/__init__.py``).

Convention (the paper fixes none; the reading is recorded with the design):
  forward   U(i1, i3) = sum_x u(x1, x3) exp(-2 pi i (i1 x1 / n1 + i3 x3 / n3))
            for the stored half spectrum i1 = 0..n1-1, i3 = 0..n3/2;
  inverse   t(x) = (1/(n1 n3)) sum_{i1, i3} c(i3) Re[T(i1, i3) exp(+2 pi i (...))]
            with c = 1 on the columns i3 = 0 and i3 = n3/2, c = 2 elsewhere.
The inverse is the real part of the full inverse DFT of the Hermitian
extension of the stored half; it equals numpy's irfft2 for any input.
Both are written as explicit sums (separable: one matrix of exponentials per
axis, each exponent reduced modulo n exactly in integers).
"""
from __future__ import annotations

import numpy as np


def _phase(idx_a, idx_b, n, sign):
    """E[a, b] = exp(sign * 2 pi i ((a b) mod n) / n)."""
    prod = np.multiply.outer(np.asarray(idx_a, dtype=np.int64),
                             np.asarray(idx_b, dtype=np.int64)) % n
    return np.exp(sign * 2j * np.pi * prod / n)


def forward_half(u):
    """Half-spectrum DFT of real fields u[..., n1, n3] -> [..., n1, n3//2 + 1]."""
    u = np.asarray(u, dtype=np.float64)
    n1, n3 = u.shape[-2], u.shape[-1]
    h = n3 // 2 + 1
    e3 = _phase(np.arange(n3), np.arange(h), n3, -1.0)     # [x3, i3]
    e1 = _phase(np.arange(n1), np.arange(n1), n1, -1.0)     # [i1, x1]
    a = u @ e3                                               # [..., x1, i3]
    return np.einsum("ax,...xk->...ak", e1, a)


def inverse_half(t_hat, n3):
    """Real field from a stored half spectrum, per the weighted real-part rule."""
    t_hat = np.asarray(t_hat, dtype=np.complex128)
    n1, h = t_hat.shape[-2], t_hat.shape[-1]
    assert h == n3 // 2 + 1
    c = np.full(h, 2.0)
    c[0] = 1.0
    c[n3 // 2] = 1.0
    e1 = _phase(np.arange(n1), np.arange(n1), n1, +1.0)     # [x1, i1]
    e3 = _phase(np.arange(h), np.arange(n3), n3, +1.0)      # [i3, x3]
    a = np.einsum("xa,...ak->...xk", e1, t_hat)              # [..., x1, i3]
    full = (a * c) @ e3                                      # [..., x1, x3]
    return full.real / (n1 * n3)


def forward_half_fft(u):
    """The same half-spectrum transform as ``forward_half`` with numpy's FFT as the
    step (a library primitive), for grids where explicit sums are too slow.
    Pinned against ``forward_half`` by the tests."""
    return np.fft.rfft2(np.asarray(u, dtype=np.float64))
