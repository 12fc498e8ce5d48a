"""HIP path vs CPU oracle at the workloads' own sizes, and across calls
that change the step length.

- coupled_nve at its full size (bcc 20^3 cells, 16 000 atoms): 200 steps of
  0.1 fs in two calls, with a list rebuild inside, FP64 bar (1e-10 on
  positions, spins, velocities; same rebuild count and colouring; energies
  and M).
- batched replicas at their real sizes: three replicas of the 64-replica
  workload (24^3 cells = 27 648 atoms at 959 K, 23^3 cells with nine
  colours, 8^3 cells) in both execution modes, 30 steps, every replica
  against its own oracle run.
- a call that raises |dt|: the rebuild decision before its first step takes
  the larger step length (same rebuild steps as the oracle).
"""
import numpy as np
import pytest

from paper_1801_10233_amd import workloads as W
from tests.common import make_gpu, make_oracle, parity

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


def test_coupled_nve_full_size_200_steps_with_rebuild():
    w = W.coupled_nve(n=20)
    o = make_oracle(w)
    g = make_gpu(w, thermo_every=50)
    for chunk in (100, 100):
        o.step(chunk, w.dt)
        g.step(chunk, w.dt)
    p = parity(w, o, g)
    _print("16000 atoms, 200 steps", p, "rebuilds", o.num_rebuilds, g.stats())
    assert p["ok"], p
    assert o.num_rebuilds >= 2                  # the first build and at least one rebuild
    assert g.stats()["rebuilds"] == o.num_rebuilds
    assert np.array_equal(g.coloring()[0], o.coloring()[0])
    eo, eg = o.energy(), g.energy()
    for k in eo:
        assert eg[k] == pytest.approx(eo[k], rel=1e-11, abs=1e-10), k
    Mo, Mg = o.magnetization(), g.magnetization()
    assert np.abs(Mg - Mo).max() <= 1e-10 * w.N


C4_PICK = (11, 46, 56)   # n = 24 (959 K), n = 23 (K = 9), n = 8


@pytest.fixture(scope="module")
def c4_oracle_states():
    ws = W.batched_replicas()
    picked = [ws[k] for k in C4_PICK]
    out = []
    for w in picked:
        o = make_oracle(w)
        o.step(30, w.dt)
        out.append((o.get_state(), o.energy(), o.magnetization(), o.num_rebuilds))
    return picked, out


@pytest.mark.parametrize("mode", [0, 1])   # SL_BATCH_PERSISTENT, SL_BATCH_PHASED
def test_batch_replicas_at_full_size(mode, c4_oracle_states):
    from paper_1801_10233_amd import spinlat as sl
    ws, ref = c4_oracle_states
    assert ws[0].N == 27648
    b = sl.Batch(ws, precision=sl.SL_FP64)
    b.set_mode(mode)
    b.step(30, ws[0].dt)
    tot = 0
    for r, (w, ((ro, vo, so), eo, Mo, nb)) in enumerate(zip(ws, ref)):
        rg, vg, sg = b.get_state(r)
        dr = np.abs(rg - ro).max() / w.box[0]
        ds = np.abs(sg - so).max()
        dv = np.abs(vg - vo).max() / np.abs(vo).max()
        _print("mode", mode, "replica", C4_PICK[r], "N", w.N, dr, ds, dv)
        assert dr < 1e-10 and ds < 1e-10 and dv < 1e-10
        eg = b.energy(r)
        for k in eo:
            assert eg[k] == pytest.approx(eo[k], rel=1e-11, abs=1e-10), k
        Mg = sg.sum(axis=0)
        assert np.abs(Mg - Mo).max() <= 1e-10 * w.N
        tot += nb - 1
    assert b.stats()["rebuilds"] == tot
    b.close()


def _free_flight(speed=10.0, replica=0):
    r, box = W.bcc_lattice(4)
    N = r.shape[0]
    v = np.zeros((N, 3))
    v[0] = (speed, 0.0, 0.0)
    w = W.coupled_nve(n=4)
    w.r, w.v, w.mass = r, v, np.full(N, W.FE_MASS)
    w.pot = W._pot(**dict(W.EXCHANGE_BJ, ex_alpha=0.0))
    w.replica = replica
    return w


def test_larger_dt_in_the_next_call_rebuilds_like_the_oracle():
    # one atom at 10 A/ps among atoms at rest, no forces: 5 steps of 1 fs,
    # then 12 fs steps (0.12 A each); the decision before the first 12 fs
    # step must take 12 fs, so every one of them starts from a fresh list
    w = _free_flight()
    o = make_oracle(w)
    g = make_gpu(w)
    for dt, n in ((1e-3, 5), (1.2e-2, 6)):
        o.step(n, dt)
        g.step(n, dt)
        assert g.stats()["rebuilds"] == o.num_rebuilds
    assert o.num_rebuilds == 7
    p = parity(w, o, g)
    assert p["ok"], p


@pytest.mark.parametrize("mode", [0, 1])
def test_batch_larger_dt_in_the_next_call(mode):
    from paper_1801_10233_amd import spinlat as sl
    ws = [_free_flight(10.0, 0), _free_flight(4.0, 1)]
    b = sl.Batch(ws, precision=sl.SL_FP64)
    b.set_mode(mode)
    os_ = [make_oracle(w) for w in ws]
    for dt, n in ((1e-3, 5), (1.2e-2, 6)):
        for o in os_:
            o.step(n, dt)
        b.step(n, dt)
    for r, (w, o) in enumerate(zip(ws, os_)):
        rg, _, _ = b.get_state(r)
        ro, _, _ = o.get_state()
        assert np.abs(rg - ro).max() / w.box[0] < 1e-12
    _print("batch dt change: rebuilds", b.stats(), [o.num_rebuilds for o in os_])
    assert b.stats()["rebuilds"] == sum(o.num_rebuilds - 1 for o in os_)
