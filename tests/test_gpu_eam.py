"""Embedded-atom mechanical potential (Finnis-Sinclair iron, standing in for
the paper's tabulated EAM, Sec. 2) on the GPU against the oracle: the
two-pass force (densities, then the gather) in every combination with the
other terms, launch shapes, batched replicas and the FP32 form."""
import numpy as np
import pytest

from paper_1801_10233_amd import workloads as W
from tests.common import make_gpu, make_oracle, parity

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [6, 7])
def test_eam_coupled_parity(n):
    w = W.eam_coupled(n=n, T=600.0)
    o, g = make_oracle(w), make_gpu(w)
    e0 = o.energy()
    for k, v in g.energy().items():
        assert v == pytest.approx(e0[k], rel=1e-11, abs=1e-11), k
    for chunk in (50, 50):
        o.step(chunk, 2e-4)
        g.step(chunk, 2e-4)
    p = parity(w, o, g)
    print("eam parity", n, p, "rebuilds", o.num_rebuilds, flush=True)
    assert p["ok"], p
    assert g.stats()["rebuilds"] == o.num_rebuilds
    assert np.array_equal(g.coloring()[0], o.coloring()[0])
    eo, eg = o.energy(), g.energy()
    for k in eo:
        assert eg[k] == pytest.approx(eo[k], rel=1e-11, abs=1e-11), k


def test_eam_with_soc_and_baths_parity():
    w = W.eam_coupled(n=6, lam=0.05)
    w.pot = dict(w.pot, **W.NEEL_BJ, **W.DMI_BJ, lat_gamma=150.0, lat_temperature=400.0,
                 aniso_K=1e-4)
    o, g = make_oracle(w), make_gpu(w)
    o.step(100, w.dt)
    g.step(100, w.dt)
    p = parity(w, o, g)
    print("eam + soc + baths parity", p, flush=True)
    assert p["ok"], p


@pytest.mark.parametrize("force_lanes", [1, 2, 4, 8])
def test_eam_launch_shapes_and_fields(force_lanes):
    w = W.eam_coupled(n=6)
    o, g = make_oracle(w), make_gpu(w)
    g.set_tuning(2, force_lanes, -1, 0)
    o.step(30, w.dt); g.step(30, w.dt)
    assert parity(w, o, g)["ok"]
    Fo = o.forces()
    Fg, _ = g.fields()
    assert np.abs(Fg - Fo).max() < 1e-10 * np.abs(Fo).max()


def test_eam_nve_energy_conservation():
    w = W.eam_coupled(n=8, T=300.0)
    g = make_gpu(w)
    e0 = g.energy()["total"]
    dev = 0.0
    for _ in range(10):
        g.step(200, w.dt)
        dev = max(dev, abs(g.energy()["total"] - e0))
    print("eam NVE max |dE|/N", dev / w.N, flush=True)
    assert dev / w.N < 1e-6


def test_eam_fp32_form_close():
    from paper_1801_10233_amd import spinlat as sl
    w = W.eam_coupled(n=6)
    o, g = make_oracle(w), make_gpu(w, precision=sl.SL_FP32)
    o.step(50, w.dt); g.step(50, w.dt)
    _, vo, so = o.get_state()
    _, vg, sg = g.get_state()
    assert np.abs(sg - so).max() < 1e-4
    assert np.abs(vg - vo).max() < 1e-4 * np.abs(vo).max()
    assert abs(g.energy()["total"] - o.energy()["total"]) / w.N < 1e-6


@pytest.mark.parametrize("mode", [0, 1])
def test_eam_batch_matches_oracle(mode):
    from paper_1801_10233_amd import spinlat as sl
    ws = W.batched_replicas(R=3, seed=51, n_lo=5, n_hi=7)
    for k, w in enumerate(ws):
        if k != 2:                                  # one Morse replica stays
            w.pot = dict(w.pot, morse_on=0, **W.FS_FE)
    b = sl.Batch(ws, precision=sl.SL_FP64)
    b.set_mode(mode)
    b.step(30, 1e-4)
    b.step(30, 1e-4)
    for r, w in enumerate(ws):
        o = make_oracle(w)
        o.step(60, 1e-4)
        ro, vo, so = o.get_state()
        rg, vg, sg = b.get_state(r)
        dr = np.abs(rg - ro).max() / w.box[0]
        ds = np.abs(sg - so).max()
        dv = np.abs(vg - vo).max() / np.abs(vo).max()
        print("eam replica", r, dr, ds, dv, flush=True)
        assert dr < 1e-10 and ds < 1e-10 and dv < 1e-10
        eo, eg = o.energy(), b.energy(r)
        assert eg["total"] == pytest.approx(eo["total"], rel=1e-11)


def test_eam_argument_errors():
    from paper_1801_10233_amd import spinlat as sl
    w = W.eam_coupled(n=5)
    g = make_gpu(w)
    for bad in (dict(eam_d=0.0), dict(eam_c=-1.0), dict(eam_A=-1.0)):
        with pytest.raises(sl.SpinLatError):
            g.set_potential(dict(w.pot, **bad))
    f = make_gpu(w, precision=sl.SL_FP32)
    m = sl.Mlp()
    m.set_weights(np.zeros(sl.SL_MLP_NPARAM, dtype=np.float32) + 0.01)
    with pytest.raises(sl.SpinLatError):
        f.set_mlp(m)
