"""The seeded workload generators: determinism and the step-source decomposition."""
import numpy as np

import workloads


def test_increments_deterministic_and_unit_rms():
    wl = workloads.WORKLOADS[1].scaled(n1=32, n3=16, steps=5)
    a = workloads.Increments(wl).history(5)
    b = workloads.Increments(wl).history(5)
    assert np.array_equal(a, b)
    rms = np.sqrt(np.mean(a ** 2, axis=(-1, -2)))
    np.testing.assert_allclose(rms, 1.0, rtol=1e-12)
    # spectral amplitude ~ |k|^-2 with the mean removed
    spec = np.abs(np.fft.rfft2(a[0, 0, 0]))
    assert spec[0, 0] < 1e-9


def test_step_sources_reproduce_increments():
    for ident, kw in [(2, dict(n1=16, n3=16, bank=4, steps=80)),
                      (5, dict(n1=16, n3=16, bank=4, steps=20)),
                      (4, dict(n1=8, n3=8, steps=6))]:
        wl = workloads.WORKLOADS[ident].scaled(**kw)
        fields, index, uniform = workloads.step_sources(wl)
        inc = workloads.Increments(wl)
        for n in range(wl.steps):
            np.testing.assert_array_equal(fields[index(n)] + uniform(n)[:, :, None, None], inc(n))
