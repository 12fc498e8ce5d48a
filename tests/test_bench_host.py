"""Host-side logic of the benchmark (no GPU): the single-GPU guard, the
rocprofv3 summaries, and the byte accounting of the roofline."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_summaries_of_trace_and_counter_files(tmp_path, capsys):
    B = _bench()
    kt = tmp_path / "kt_kernel_trace.csv"
    kt.write_text("Kernel_Name,Start_Timestamp,End_Timestamp\n"
                  "k_a,100,1100\nk_a,2000,5000\nk_b,0,500\n")
    pc = tmp_path / "pc_counter_collection.csv"
    pc.write_text("Kernel_Name,Counter_Name,Counter_Value\n"
                  "k_a,FETCH_SIZE,10\nk_a,FETCH_SIZE,30\nk_b,WRITE_SIZE,7\n")
    B.summarize([str(kt), str(pc)])
    out = capsys.readouterr().out
    # k_a: two launches of 1 us and 3 us
    line = [l for l in out.splitlines() if l.endswith("k_a") and "calls" in l][0]
    assert "calls=     2" in line and "mean_us=     2.000" in line
    line = [l for l in out.splitlines() if "FETCH_SIZE" in l][0]
    assert "dispatches=     2" in line and "mean=          20.0" in line


def test_kernel_occupancy_of_a_trace_window():
    B = _bench()
    ns = 1_000_000  # 1 ms
    rows = [dict(Start_Timestamp=a * ns, End_Timestamp=b * ns)
            for a, b in ((0, 4), (5, 7), (6, 8), (9, 10))]
    # last 5 ms = [5, 10]: kernels cover [5, 8] and [9, 10], overlaps counted once
    n, busy, frac = B.busy_window(rows, 5.0)
    assert (n, busy, frac) == (3, 4.0, 0.8)
    # a window reaching back into the first kernel clips it: [3, 10] holds 1 + 3 + 1 ms
    n, busy, frac = B.busy_window(rows, 7.0)
    assert n == 4 and busy == 5.0 and abs(frac - 5.0 / 7.0) < 1e-12


def test_algorithmic_bytes_and_profile_lookup():
    B = _bench()
    sl = B.sl
    # plain spin update: s r/w, own r, 14 indices; cached: 14 J instead of r
    assert B.SPIN_BYTES[sl.SL_FP64] == 128 and B.SPIN_BYTES_JC[sl.SL_FP64] == 216
    assert B.FORCE_BYTES[sl.SL_FP64] == 384
    assert B.JCACHE_BYTES[sl.SL_FP64] == 192
    # a summary of another launch shape or of older sources is never used
    assert B.counter_traffic("k_spin_phase", sl.SL_FP64, "lanes=3,jcache=0") is None
    assert B.counter_traffic("no_such_kernel", sl.SL_FP64, "lanes=1") is None


def test_committed_counter_summaries_match_the_sources():
    # the summaries under profiles/ were taken on the current kernel sources
    # (same SHA-256) for the shape the autotuner picks at 432 000 atoms, so
    # the benchmark reports their traffic instead of null
    B = _bench()
    sl = B.sl
    t = B.counter_traffic("k_spin_phase", sl.SL_FP64, "lanes=1,jcache=0")
    tc = B.counter_traffic("k_spin_phase", sl.SL_FP64, "lanes=1,jcache=1")
    f = B.counter_traffic("k_force", sl.SL_FP64, "lanes=1")
    assert t is not None and tc is not None and f is not None
    alg_spin = B.SPIN_BYTES[sl.SL_FP64] * 108000
    alg_force = B.FORCE_BYTES[sl.SL_FP64] * 432000
    assert alg_spin < t < 5 * alg_spin and alg_force < f < 5 * alg_force


def test_whole_step_byte_conventions():
    # the unfused count of one FP64 atom-step: four spin sweeps of 128 B, a
    # force pass writing F (304 B), kick + drift (120 B), final kick (72 B)
    B = _bench()
    sl = B.sl
    assert B.STEP_BYTES_UNFUSED[sl.SL_FP64] == 1008
    assert B.STEP_BYTES[sl.SL_FP64] == 4 * 128 + 384 == 896


def test_drift_slope_and_standard_error():
    # a known slope under correlated noise: the estimate is within a few
    # standard errors, and the error grows with the correlation time
    import numpy as np
    B = _bench()
    rng = np.random.default_rng(3)
    t = np.linspace(0.0, 10.0, 4000)
    white = rng.standard_normal(t.size)
    slow = np.convolve(rng.standard_normal(t.size + 99), np.ones(100) / 10.0, mode="valid")
    for noise in (white, slow):
        y = 2.5e-3 * t + 1e-2 * noise
        s, se, g = B.slope_with_error(t, y)
        assert abs(s - 2.5e-3) < 4 * se
    _, se_w, g_w = B.slope_with_error(t, 2.5e-3 * t + 1e-2 * white)
    _, se_s, g_s = B.slope_with_error(t, 2.5e-3 * t + 1e-2 * slow)
    assert g_w < 3 and g_s > 20 and se_s > 3 * se_w
