"""Lattice bath (Sec. 4.2, Eq. p_advance_T) and the temperature observables
(Eqs. lattice_temperature, spin_temperature) on the GPU against the oracle.

The bath noise comes from the same counter-based Philox stream on both
sides, so trajectories agree to roundoff (FP64 bar: 1e-10 over 100 steps),
with and without the spin bath, for one system and for batched replicas.
The relaxation runs check the physics the paper reports qualitatively: a
spin bath alone heats a lattice at rest through the magneto-mechanical
force, and an isolated run conserves the total energy while it is
repartitioned between the lattice and the spins."""
import numpy as np
import pytest

from paper_1801_10233_amd import workloads as W
from tests.common import make_gpu, make_oracle, parity

pytestmark = pytest.mark.gpu


def _with_lattice_bath(w, gamma=300.0, T=600.0):
    w.pot = dict(w.pot, lat_gamma=gamma, lat_temperature=T)
    return w


@pytest.mark.parametrize("maker", ["coupled", "langevin"])
def test_lattice_bath_parity(maker):
    w = W.coupled_nve(n=6) if maker == "coupled" else W.large_langevin(n=7)
    w = _with_lattice_bath(w)
    if maker == "coupled":
        w.seed = 4242
    o = make_oracle(w)
    g = make_gpu(w)
    for chunk in (30, 70):
        o.step(chunk, w.dt)
        g.step(chunk, w.dt)
    p = parity(w, o, g)
    print("lattice bath parity", maker, p, flush=True)
    assert p["ok"], p
    assert g.stats()["rebuilds"] == o.num_rebuilds
    # the bath moved the velocities away from the NVE trajectory
    nve = make_oracle(W.coupled_nve(n=6) if maker == "coupled" else W.large_langevin(n=7))
    nve.step(100, w.dt)
    assert np.abs(nve.get_state()[1] - o.get_state()[1]).max() > 1e-3


def test_lattice_bath_negative_dt_and_zero_gamma():
    # zero friction is the plain step; a negative dt damps with |dt|
    w = W.coupled_nve(n=6)
    w.pot = dict(w.pot, lat_gamma=0.0, lat_temperature=900.0)
    o, g = make_oracle(w), make_gpu(w)
    o.step(40, w.dt); g.step(40, w.dt)
    assert parity(w, o, g)["ok"]
    w = _with_lattice_bath(W.coupled_nve(n=6))
    o, g = make_oracle(w), make_gpu(w)
    o.step(20, w.dt); g.step(20, w.dt)
    o.step(20, -w.dt); g.step(20, -w.dt)
    p = parity(w, o, g)
    assert p["ok"], p


def test_temperatures_match_oracle():
    from paper_1801_10233_amd import spinlat as sl
    w = W.large_langevin(n=7)
    w.pot = dict(w.pot, B=(0.3, -0.2, 1.0))
    o = make_oracle(w)
    g = make_gpu(w)
    o.step(20, w.dt); g.step(20, w.dt)
    TLo, TSo = o.temperatures()
    TLg, TSg = g.temperatures()
    print("temperatures", TLo, TLg, TSo, TSg, flush=True)
    assert TLg == pytest.approx(TLo, rel=1e-10)
    assert TSg == pytest.approx(TSo, rel=1e-9)
    # FP32 form: same state, FP32 spins and exchange sums
    f = make_gpu(w, precision=sl.SL_FP32)
    r, v, s = o.get_state()
    f.set_state(r, v, s, w.mass)
    TLf, TSf = f.temperatures()
    assert TLf == pytest.approx(TLo, rel=1e-12)
    assert TSf == pytest.approx(TSo, rel=1e-4)


@pytest.mark.parametrize("mode", [0, 1])
def test_batch_lattice_bath_matches_oracle(mode):
    from paper_1801_10233_amd import spinlat as sl
    ws = W.batched_replicas(R=3, seed=31, n_lo=5, n_hi=7)
    for k, w in enumerate(ws):
        _with_lattice_bath(w, gamma=100.0 * (k + 1), T=200.0 + 300.0 * k)
    b = sl.Batch(ws, precision=sl.SL_FP64)
    b.set_mode(mode)
    b.step(25, 1e-4)
    b.step(35, 1e-4)
    for r, w in enumerate(ws):
        o = make_oracle(w)
        o.step(60, 1e-4)
        ro, vo, so = o.get_state()
        rg, vg, sg = b.get_state(r)
        dr = np.abs(rg - ro).max() / w.box[0]
        ds = np.abs(sg - so).max()
        dv = np.abs(vg - vo).max() / np.abs(vo).max()
        print("replica", r, dr, ds, dv, flush=True)
        assert dr < 1e-10 and ds < 1e-10 and dv < 1e-10
        TLo, TSo = o.temperatures()
        TLg, TSg = b.temperatures(r)
        assert TLg == pytest.approx(TLo, rel=1e-9)
        assert TSg == pytest.approx(TSo, rel=1e-8)


def test_spin_bath_heats_lattice_at_rest():
    # first relaxation run of Sec. 4.2 (scaled down): the spin bath holds
    # T_S near its target; the lattice, at rest at first, is heated only by
    # the magneto-mechanical force
    w = W.two_thermostat(n=8, bath="spin", lam=0.5)
    g = make_gpu(w)
    TL0, _ = g.temperatures()
    assert TL0 == 0.0
    TL, TS = [], []
    for _ in range(10):
        g.step(1000, w.dt)
        a, b = g.temperatures()
        TL.append(a); TS.append(b)
    print("spin bath run T_L", np.round(TL, 2), "T_S", np.round(TS, 1), flush=True)
    assert TL[-1] > 1.0 and TL[-1] > 2.0 * TL[0]
    assert abs(np.mean(TS[-5:]) / 300.0 - 1.0) < 0.3


def test_isolated_run_repartitions_energy():
    # NVE run from paramagnetic spins (Sec. 4.2): the total energy stays
    # constant while the magnetic energy flows into the lattice
    w = W.energy_repartition(n=8)
    g = make_gpu(w)
    e0 = g.energy()
    mag0 = e0["exchange"] + e0["zeeman"] + e0["aniso"]
    es = []
    for _ in range(10):
        g.step(500, w.dt)
        es.append(g.energy())
    mag = np.array([e["exchange"] + e["zeeman"] + e["aniso"] for e in es])
    lat = np.array([e["kin"] + e["pair"] for e in es])
    tot = np.array([e["total"] for e in es])
    print("repartition mag", np.round(mag - mag0, 4), "lat", np.round(lat - (e0["kin"] + e0["pair"]), 4),
          flush=True)
    N = w.N
    assert np.abs(tot - e0["total"]).max() / N < 1e-6
    assert mag[-1] < mag0 - 1e-4 * N          # spins gave energy away ...
    assert lat[-1] > e0["kin"] + e0["pair"] + 1e-4 * N   # ... to the lattice


def test_lattice_bath_holds_target_and_collinear_spins_stay_cold():
    # second relaxation run of Sec. 4.2 (scaled down): the lattice bath
    # brings T_L to its target after the equipartition drop. Isotropic
    # exchange exerts no torque on a collinear state, so without a
    # spin-orbit term the aligned spins cannot take energy from the lattice
    # and T_S stays exactly zero (every s_i x omega_i vanishes).
    w = W.two_thermostat(n=8, bath="lattice", lat_gamma=300.0)
    g = make_gpu(w)
    TL, TS = [], []
    for _ in range(10):
        g.step(1000, w.dt)
        a, b = g.temperatures()
        TL.append(a); TS.append(b)
    print("lattice bath run T_L", np.round(TL, 1), "T_S", TS, flush=True)
    assert abs(np.mean(TL[-5:]) / 300.0 - 1.0) < 0.1
    assert max(abs(t) for t in TS) == 0.0
