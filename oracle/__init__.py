"""CPU float64 oracle of the spectral boundary integral (SBIM) traction update.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this package;
the product library never does, and it shares no code, constants or helpers
with it.  Everything here is plain and slow on purpose: naive DFTs written as
explicit sums, the history convolution as a direct loop over lags, and the
elastodynamic kernels by a quadrature of their branch-cut integrals.

Modules
  kernels  half-space stiffness, time kernels H_ab, integrated kernels G_ab and
           the per-lag convolution weights (Sec. 2.3, Eq. SBI and the kernels
           it defers to; derived from Eqs. consmoment and linelasticity)
  dft      naive forward / inverse transforms on the stored half spectrum
  sbim     the per-step traction update and its exact transpose (adjoint)
  fault    a frictional fault between two half-spaces: stand-alone rupture
           (Sec. 2.2 friction and stick-slip, Eq. SBI on each side)
  hybrid   the hybrid scheme: a strip of hexahedral finite elements on the
           fault, closed at S+ by the boundary relation (Secs. 2.2-2.4)

Every function is pinned by ``tests/test_oracle_*.py`` against closed forms,
library routines (numpy.fft, scipy.special, mpmath inverse Laplace) and
invariants; see each test for the pin it provides.
"""
from . import dft, kernels, sbim  # noqa: F401
from .sbim import (Config, Plane, forward, adjoint, spectra, mode_geometry,  # noqa: F401
                   mode_window, mode_response, adjoint_response)
