"""Split force (tuning `overlap`): the spin-independent pair terms of a
step's closing force computed on a second stream while the spins update,
the spin-dependent terms added by the closing launch. Same physics as the
fused launch, so the FP64 bar against the oracle is unchanged (1e-10 over
100 steps), with every term the split touches: Morse, exchange derivative,
anisotropy and both baths, the Neel and DMI terms, the embedded-atom terms,
the sectored order, list rebuilds, sampled energies and 1 or 2 force lanes."""
import numpy as np
import pytest

from paper_1801_10233_amd import workloads as W
from tests.common import make_gpu, make_oracle, parity

pytestmark = pytest.mark.gpu


def _split(g, force_lanes=1):
    t = g.tuning()
    g.set_tuning(t["spin_lanes"], force_lanes, 0, t["jcache"], 1)
    assert g.tuning()["overlap"] == 1
    return g


def _run_both(w, steps=100, **kw):
    o = make_oracle(w)
    g = _split(make_gpu(w, **kw))
    o.step(steps, w.dt)
    g.step(steps, w.dt)
    return o, g


@pytest.mark.parametrize("force_lanes", [1, 2])
def test_split_coupled_parity_through_rebuilds(force_lanes):
    from paper_1801_10233_amd import spinlat as sl
    w = W.coupled_nve(n=8)
    w.v = w.v * 6.0
    o = make_oracle(w)
    g = _split(make_gpu(w), force_lanes)
    g.set_profiling(True)
    o.step(100, w.dt)
    g.step(100, w.dt)
    launches = g.profile(sl.PROF_PAIR)[0]
    g.set_profiling(False)
    p = parity(w, o, g)
    print("split coupled", force_lanes, p, g.stats(), flush=True)
    assert launches == 100                     # one pair pass per step, native
    assert g.stats()["rebuilds"] >= 2
    assert p["ok"], p


def test_split_langevin_anisotropy_and_lattice_bath():
    w = W.large_langevin(n=7)
    w.pot = dict(w.pot, lat_gamma=300.0, lat_temperature=600.0)
    o, g = _run_both(w)
    p = parity(w, o, g)
    print("split langevin + lattice bath", p, flush=True)
    assert p["ok"], p


def test_split_spin_orbit_terms():
    w = W.soc_coupled(n=6)
    o, g = _run_both(w)
    p = parity(w, o, g)
    print("split soc", p, flush=True)
    assert p["ok"], p


def test_split_eam_with_spin_orbit_and_baths():
    w = W.eam_coupled(n=6, lam=0.05)
    w.pot = dict(w.pot, **W.NEEL_BJ, **W.DMI_BJ, lat_gamma=150.0, lat_temperature=400.0,
                 aniso_K=1e-4)
    o, g = _run_both(w)
    p = parity(w, o, g)
    print("split eam + soc + baths", p, flush=True)
    assert p["ok"], p


def test_split_sectored_order():
    from oracle import oracle as O
    from paper_1801_10233_amd import spinlat as sl
    w = W.large_langevin(n=6)
    o = O.Oracle(w.r, w.v, w.s, w.mass, w.box, w.pot, frozen=w.frozen, skin=w.skin,
                 seed=w.seed, replica=w.replica, ordering=O.SECT, sect_grid=(2, 2, 2))
    g = _split(make_gpu(w))
    g.set_ordering(sl.SL_ORDER_SECTORS, (2, 2, 2))
    o.step(60, w.dt)
    g.step(60, w.dt)
    p = parity(w, o, g)
    print("split sectors", p, flush=True)
    assert p["ok"], p


def test_split_sampled_energies_match_fused():
    w = W.coupled_nve(n=6)
    a = make_gpu(w, thermo_every=10)
    b = _split(make_gpu(w, thermo_every=10))
    a.step(100, w.dt)
    b.step(100, w.dt)
    sa, Ea, Ma = a.thermo()
    sb, Eb, Mb = b.thermo()
    assert np.array_equal(sa, sb) and len(sa) == 10
    scale = np.abs(Ea).max()
    assert np.abs(Eb - Ea).max() <= 1e-12 * scale
    assert np.abs(Mb - Ma).max() <= 1e-10
    o = make_oracle(w)
    o.step(100, w.dt)
    assert b.energy()["total"] == pytest.approx(o.energy()["total"], rel=1e-10)


def test_split_rejects_bad_value_and_keeps_learned_forms_fused():
    from paper_1801_10233_amd import spinlat as sl
    g = make_gpu(W.coupled_nve(n=5))
    with pytest.raises(sl.SpinLatError) as e:
        g.set_tuning(2, 1, 0, -1, 2)
    assert e.value.code == sl.SL_E_ARG
    g.set_tuning(2, 4, 0, -1, 1)               # 4 force lanes: the fused launch runs
    g.set_profiling(True)
    g.step(5, 1e-4)
    assert g.profile(sl.PROF_PAIR)[0] == 0
    g.set_profiling(False)
