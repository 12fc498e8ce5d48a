"""Autotuner: picks launch shapes on a scratch copy without advancing the
system, and the tuned system still matches the oracle (1e-10 over the
run). The JSON-lines cache returns the stored choice without re-timing."""
import os

import numpy as np
import pytest

from paper_1801_10233_amd import workloads as W
from tests.common import make_gpu, make_oracle

pytestmark = pytest.mark.gpu


def test_autotune_leaves_state_and_keeps_parity(tmp_path, monkeypatch):
    monkeypatch.setenv("SL_TUNE_CACHE", str(tmp_path / "tune.jsonl"))
    w = W.coupled_nve(n=6)
    g = make_gpu(w)
    g.step(10, w.dt)
    before = g.get_state()
    t = g.autotune(5, w.dt)
    after = g.get_state()
    for a, b in zip(before, after):
        assert np.array_equal(a, b)
    assert t["spin_lanes"] in (1, 2, 4, 8) and t["force_lanes"] in (1, 2)
    assert g.tuning()["spin_lanes"] == t["spin_lanes"]
    g.step(90, w.dt)
    o = make_oracle(w)
    o.step(100, w.dt)
    ro, vo, so = o.get_state()
    rg, vg, sg = g.get_state()
    assert np.abs(rg - ro).max() / w.box[0] < 1e-10
    assert np.abs(sg - so).max() < 1e-10
    # a second system of the same shape takes the cached choice
    g2 = make_gpu(w)
    t2 = g2.autotune(5, w.dt)
    assert t2 == t
    with open(tmp_path / "tune.jsonl") as fh:
        assert len(fh.readlines()) == 1


def test_batch_autotune_leaves_state_and_keeps_parity(monkeypatch):
    monkeypatch.delenv("SL_TUNE_CACHE", raising=False)
    from paper_1801_10233_amd import spinlat as sl
    ws = W.batched_replicas(R=3, seed=31, n_lo=5, n_hi=7)
    b = sl.Batch(ws, precision=sl.SL_FP64)
    b.step(10, 1e-4)
    before = [b.get_state(r) for r in range(len(ws))]
    ch = b.autotune(4, 1e-4)
    assert ch["mode"] in (0, 1) and ch["lanes"] in (1, 2, 4)
    assert b.mode() == ch["mode"]
    for r in range(len(ws)):
        for x, y in zip(before[r], b.get_state(r)):
            assert np.array_equal(x, y)
    b.step(40, 1e-4)
    for r, w in enumerate(ws):
        o = make_oracle(w)
        o.step(50, 1e-4)
        ro, vo, so = o.get_state()
        rg, vg, sg = b.get_state(r)
        assert np.abs(rg - ro).max() / w.box[0] < 1e-10
        assert np.abs(sg - so).max() < 1e-10


def test_fp32_autotune_runs(monkeypatch):
    monkeypatch.delenv("SL_TUNE_CACHE", raising=False)
    from paper_1801_10233_amd import spinlat as sl
    w = W.coupled_nve(n=6)
    g = make_gpu(w, precision=sl.SL_FP32)
    g.step(5, w.dt)
    before = g.get_state()
    t = g.autotune(3, w.dt)
    assert t["spin_lanes"] in (1, 2, 4, 8)
    for a, b in zip(before, g.get_state()):
        assert np.array_equal(a, b)
    ws = W.batched_replicas(R=2, seed=3, n_lo=5, n_hi=6)
    b = sl.Batch(ws, precision=sl.SL_FP32)
    b.step(3, 1e-4)
    assert b.autotune(3, 1e-4)["mode"] in (0, 1)
