"""Batched replicas vs the CPU oracle, per replica, in both execution modes
(one persistent launch; one launch per colour phase over all replicas).

Replicas of uneven size, temperature and field, each with its own Philox
replica index; FP64 bar as for a single system (1e-10 over the run),
including replicas that rebuild their lists inside the run."""
import numpy as np
import pytest

from paper_1801_10233_amd import workloads as W
from tests.common import make_oracle, parity

pytestmark = pytest.mark.gpu


def _small_replicas(R=4, seed=77, hot=False):
    ws = W.batched_replicas(R=R, seed=seed, n_lo=5, n_hi=7)
    if hot:
        for w in ws:
            w.pot = dict(w.pot, temperature=1500.0)
            w.v = W.maxwell_velocities(w.mass, 1500.0, 1000 + w.replica)
    return ws


MODES = [0, 1]   # SL_BATCH_PERSISTENT, SL_BATCH_PHASED


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("lanes", [1, 2, 4])
def test_batch_matches_oracle_per_replica(lanes, mode):
    from paper_1801_10233_amd import spinlat as sl
    ws = _small_replicas()
    b = sl.Batch(ws, precision=sl.SL_FP64)
    b.set_lanes(lanes)
    b.set_mode(mode)
    b.step(60, 1e-4)
    for r, w in enumerate(ws):
        o = make_oracle(w)
        o.step(60, 1e-4)
        ro, vo, so = o.get_state()
        rg, vg, sg = b.get_state(r)
        dr = np.abs(rg - ro).max() / w.box[0]
        ds = np.abs(sg - so).max()
        dv = np.abs(vg - vo).max() / np.abs(vo).max()
        print("replica", r, "N", w.N, "T", w.pot["temperature"], dr, ds, dv, flush=True)
        assert dr < 1e-10 and ds < 1e-10 and dv < 1e-10


@pytest.mark.parametrize("modes", [(0, 0), (1, 1), (0, 1), (1, 0)])
def test_batch_through_rebuilds_and_calls(modes):
    # two calls, possibly switching the execution mode between them
    from paper_1801_10233_amd import spinlat as sl
    ws = _small_replicas(R=3, seed=5, hot=True)
    b = sl.Batch(ws, precision=sl.SL_FP64)
    for chunk, mode in zip((45, 80), modes):
        b.set_mode(mode)
        b.step(chunk, 2e-4)
    st = b.stats()
    print("batch stats", st, flush=True)
    tot = 0
    for r, w in enumerate(ws):
        o = make_oracle(w)
        o.step(45, 2e-4)
        o.step(80, 2e-4)
        tot += o.num_rebuilds - 1            # the first build is not a rebuild
        ro, vo, so = o.get_state()
        rg, vg, sg = b.get_state(r)
        assert np.abs(rg - ro).max() / w.box[0] < 1e-10
        assert np.abs(sg - so).max() < 1e-9
        assert np.abs(vg - vo).max() < 1e-9 * np.abs(vo).max()
    assert tot >= 3 and st["rebuilds"] == tot


@pytest.mark.parametrize("mode", MODES)
def test_batch_fp32_energies_close_to_oracle(mode):
    from paper_1801_10233_amd import spinlat as sl
    ws = _small_replicas(R=3, seed=9)
    b = sl.Batch(ws, precision=sl.SL_FP32)
    b.set_mode(mode)
    b.step(50, 1e-4)
    for r, w in enumerate(ws):
        o = make_oracle(w)
        o.step(50, 1e-4)
        eg, eo = b.energy(r)["total"], o.energy()["total"]
        assert abs(eg - eo) / w.N < 1e-5


def test_batch_modes_agree():
    # same per-atom device code and lanes; the compiler may still contract
    # multiply-adds differently in the two kernels, so agreement is to
    # rounding, far inside the oracle bar
    from paper_1801_10233_amd import spinlat as sl
    ws = _small_replicas(R=5, seed=21, hot=True)
    out = []
    for mode in MODES:
        b = sl.Batch(ws, precision=sl.SL_FP64)
        b.set_mode(mode)
        b.step(70, 2e-4)
        out.append([b.get_state(r) for r in range(len(ws))])
        print("mode", mode, b.stats(), flush=True)
        b.close()
    for a, c in zip(*out):
        for x, y in zip(a, c):
            assert np.abs(x - y).max() <= 1e-12 * max(1.0, np.abs(x).max())
