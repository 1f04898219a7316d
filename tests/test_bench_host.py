"""CPU checks of bench.py's host logic: the kernel-source hash that ties the recorded
HBM-traffic counters to the kernels, the reading of those counters, and the one-GPU
guard of the command line."""
import json
import os
import shutil
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _copy_sources(tmp_path):
    src = os.path.join(ROOT, "paper_2102_08756_amd", "csrc")
    dst = tmp_path / "paper_2102_08756_amd" / "csrc"
    shutil.copytree(src, dst)
    return dst


def test_kernel_hash_ignores_comments_but_not_code(tmp_path, monkeypatch):
    base = bench.kernel_source_hash()
    dst = _copy_sources(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.kernel_source_hash() == base
    k = dst / "kernels.hip"
    k.write_text(k.read_text() + "\n// a comment only\n\n")
    assert bench.kernel_source_hash() == base
    k.write_text(k.read_text() + "\nconstexpr int kUnused = 1;\n")
    assert bench.kernel_source_hash() != base


def test_traffic_is_read_only_for_the_recorded_kernels(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    h = bench.kernel_source_hash()
    line = ("two_planes512_w1000 fp32_comp steady 6.4e+08 312500.0 52000.0 1000\n"
            "two_planes512_w1000 fp32_comp job 5.1e+08 250000.0 52000.0 2000\n")
    (prof / "step_kernel_traffic.txt").write_text(f"# header\nkernel_source_hash={h}\n{line}")
    monkeypatch.setattr(bench, "PROFILES", str(prof))
    assert bench.read_traffic("two_planes512_w1000", "fp32_comp") == 6.4e8
    assert bench.read_traffic("two_planes512_w1000", "fp32_comp", "job") == 5.1e8
    assert bench.read_traffic("two_planes512_w1000", "fp64") is None
    (prof / "step_kernel_traffic.txt").write_text(f"kernel_source_hash=0000000000000000\n{line}")
    assert bench.read_traffic("two_planes512_w1000", "fp32_comp") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_timed_steps_start_at_a_full_window():
    import workloads
    wl = workloads.WORKLOADS[2]
    # the driver's short run times the last steps of the 2000-step job
    assert bench.steady_window(wl, 20) == 1980
    # the default times every step after the 1000-lag window has filled
    k = bench.default_timed_steps(wl)
    assert k == 1000 and bench.steady_window(wl, k) == 1000
    # more timed steps than the job has at a full window: start as soon as it is full
    assert bench.steady_window(wl, 1500) == wl.window_cap - 1
    for n0 in (bench.steady_window(wl, s) for s in (1, 20, 1000, 1500, 5000)):
        assert min(wl.window_cap, n0 + 1) == wl.window_cap


def test_bracketed_launches_meet_every_sweep_phase():
    """bench.py times the step launch of every TIMING_EVERY-th timed step; the stride is
    prime to every sweep depth the library picks, so over one default run the bracketed
    steps meet each phase (n + 1) mod D of the sweep, and their count is what
    sbim_conv_timing returns for that run."""
    import math
    every = bench.TIMING_EVERY
    for depth in (1, 2, 4, 6, 8, 12, 16, 32):
        assert math.gcd(every, depth) == 1
        phases = {(n + 1) % depth for n in bench.bracketed_steps(1000, 1000, every)}
        assert phases == set(range(depth))
    assert len(bench.bracketed_steps(1980, 20, every)) == 3
    assert list(bench.bracketed_steps(1000, 15, every)) == [1000, 1007, 1014]


def test_host_cpu_reports_cores_and_model():
    h = bench.host_cpu()
    assert h["nproc"] >= 1 and h["logical_cpus"] >= h["nproc"]
    assert "model" in h
