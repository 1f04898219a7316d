"""Helpers of the full-size GPU tests (sampled Fourier bins): bin choice, input spectra
at the bins, the oracle's traction spectra there.  Not a test module."""
import numpy as np

import oracle
import workloads


def pick_bins(n1, n3, count, seed):
    """DC, the Nyquist row, the Nyquist column (i3 = n3/2, Hermitian-folded), the
    highest-|k| corner (n1/2, n3/2), and ``count`` - 4 random interior bins."""
    rng = np.random.default_rng(seed)
    k = count - 4
    i1 = rng.integers(0, n1, k)
    i3 = rng.integers(1, n3 // 2, k)
    i1 = np.concatenate([[0, n1 // 2, int(rng.integers(0, n1)), n1 // 2], i1])
    i3 = np.concatenate([[0, 1, n3 // 2, n3 // 2], i3])
    return i1, i3


def input_spectra(wl, bins, steps, round32=False):
    """X^n at the bins, n < steps: the DFT of each step's increment field (float64, or the
    float32 rounding of it that the float32 forms receive), the uniform slip at DC."""
    fields, index, uniform = workloads.step_sources(wl)
    i1, i3 = bins
    conv = (lambda f: np.float32(f).astype(np.float64)) if round32 else (lambda f: f)
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=8) as ex:   # the FFTs release the GIL
        X = np.stack(list(ex.map(lambda f: oracle.dft.forward_half_fft(conv(f))[..., i1, i3],
                                 fields)))          # [nf, P, 3, B]
    X = X[[index(n) for n in range(steps)]]
    if wl.slip_ramp:
        assert not round32, "the rounded inputs of a slip ramp differ at every step"
        dc = (i1 == 0) & (i3 == 0)
        X[:, :, :, dc] += (np.stack([uniform(n) for n in range(steps)]) * (wl.n1 * wl.n3))[..., None]
    return X


def oracle_bins(wl, bins, X, weights_cache, history32=False):
    """The oracle's traction spectra at the bins from the input spectra X (increment
    input): [steps, P, 3, B].  ``history32``: the history (the rotated displacement
    spectrum) and the damping velocity rounded to float32 per step, as the float32
    forms store them."""
    cfg = oracle.Config.from_dict(wl.config_dict())
    assert cfg.input_kind == "increment"
    U = np.cumsum(X, axis=0)
    V = X / cfg.dt
    if history32:
        _, kh1, kh3 = oracle.sbim.mode_geometry(cfg)
        c, s = kh1[bins], kh3[bins]

        def round_rotated(Y):
            L = c * Y[:, :, 0] + s * Y[:, :, 2]
            T = -s * Y[:, :, 0] + c * Y[:, :, 2]
            L = L.astype(np.complex64).astype(complex)
            T = T.astype(np.complex64).astype(complex)
            N = Y[:, :, 1].astype(np.complex64).astype(complex)
            return np.stack([c * L - s * T, N, s * L + c * T], axis=2)
        U, V = round_rotated(U), round_rotated(V)
    out = np.empty_like(U)
    for p in range(len(cfg.planes)):
        out[:, p] = oracle.mode_response(cfg, p, bins, U[:, p], V[:, p], weights_cache)
    return out


def _one_thread():
    """Worker initializer: one BLAS/OpenMP thread per worker process (the pool is the
    parallelism; nested thread pools oversubscribe the cores)."""
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)


def _pool(workers):
    import multiprocessing as mp
    import os
    from concurrent.futures import ProcessPoolExecutor
    n = max(1, min(workers, os.cpu_count() or 1, 16))
    return ProcessPoolExecutor(max_workers=n, mp_context=mp.get_context("spawn"),
                               initializer=_one_thread)


def _weights_job(key):
    q, cs, dt, W, eta = key
    return key, oracle.kernels.lag_weights(q, cs, dt, W, eta)


def prefill_weights(wl, bins, cache, workers=16):
    """Fill ``cache`` with the oracle's kernel weights of every (plane material, bin) of
    the workload, the missing ones computed in parallel worker processes (the same
    quadrature PlaneOperator would run, keyed the same way)."""
    import math
    cfg = oracle.Config.from_dict(wl.config_dict())
    q, _, _ = oracle.sbim.mode_geometry(cfg)
    qb = q[bins]
    keys = set()
    for pl in cfg.planes:
        eta = pl.cp / pl.cs
        W = oracle.sbim.mode_window(qb, pl.cs, cfg.dt, cfg)
        for qq, ww in zip(qb, W):
            if ww > 0 and cfg.window_mode != "static":
                keys.add((float(qq), pl.cs, cfg.dt, int(ww), eta))
    todo = sorted(k for k in keys if k not in cache)
    if not todo:
        return cache
    with _pool(workers) as ex:
        for i, (key, w) in enumerate(ex.map(_weights_job, todo)):
            cache[key] = w
            if (i + 1) % 8 == 0 or i + 1 == len(todo):
                print(f"[oracle] kernel weights {i + 1}/{len(todo)}", flush=True)
    assert math.isfinite(sum(float(v.sum()) for v in cache.values()))
    return cache


def _apply_job(args):
    cfg_d, p, bins, U, V, cache = args
    return oracle.mode_response(cfg_d, p, bins, U, V, cache)


def oracle_bins_parallel(wl, bins, X, weights_cache, history32=False, workers=16, chunk=4):
    """``oracle_bins`` with the bins split over worker processes (each bin's convolution
    is independent); the weights must be in the cache already (prefill_weights)."""
    cfg_d = wl.config_dict()
    cfg = oracle.Config.from_dict(cfg_d)
    U = np.cumsum(X, axis=0)
    V = X / cfg.dt
    if history32:
        _, kh1, kh3 = oracle.sbim.mode_geometry(cfg)
        c, s = kh1[bins], kh3[bins]

        def round_rotated(Y):
            L = c * Y[:, :, 0] + s * Y[:, :, 2]
            T = -s * Y[:, :, 0] + c * Y[:, :, 2]
            L = L.astype(np.complex64).astype(complex)
            T = T.astype(np.complex64).astype(complex)
            N = Y[:, :, 1].astype(np.complex64).astype(complex)
            return np.stack([c * L - s * T, N, s * L + c * T], axis=2)
        U, V = round_rotated(U), round_rotated(V)
    B = len(bins[0])
    jobs, where = [], []
    for p in range(len(cfg.planes)):
        for b0 in range(0, B, chunk):
            sl = slice(b0, min(B, b0 + chunk))
            jobs.append((cfg_d, p, (bins[0][sl], bins[1][sl]), U[:, p, :, sl], V[:, p, :, sl],
                         weights_cache))
            where.append((p, sl))
    out = np.empty_like(U)
    with _pool(workers) as ex:
        for i, ((p, sl), r) in enumerate(zip(where, ex.map(_apply_job, jobs))):
            out[:, p, :, sl] = r
            if (i + 1) % 8 == 0 or i + 1 == len(jobs):
                print(f"[oracle] bin groups {i + 1}/{len(jobs)}", flush=True)
    return out
