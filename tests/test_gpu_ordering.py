"""The paper's own spin orderings on the GPU (Sec. 5.1): sectors of a grid
of subdomains (Eq. spin_ST_sectoring) and the serial order (Eq.
spin_ST_decomposition), against the same orderings of the oracle to the
FP64 bar, and the sector ordering against the colour ordering at a larger
size (the ordering-equivalence study)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1801_10233_amd import workloads as W
from tests.common import make_gpu, parity

pytestmark = pytest.mark.gpu


def _oracle(w, ordering, grid=(1, 1, 1)):
    return O.Oracle(w.r, w.v, w.s, w.mass, w.box, w.pot, frozen=w.frozen, skin=w.skin,
                    seed=w.seed, replica=w.replica, ordering=ordering, sect_grid=grid)


@pytest.mark.parametrize("grid", [(1, 1, 1), (2, 2, 2), (2, 1, 2)])
def test_sectors_match_oracle_coupled(grid):
    from paper_1801_10233_amd import spinlat as sl
    w = W.large_langevin(n=6)                     # spin bath on: same noise per update
    o = _oracle(w, O.SECT, grid)
    g = make_gpu(w)
    g.set_ordering(sl.SL_ORDER_SECTORS, grid)
    for chunk in (40, 60):
        o.step(chunk, w.dt)
        g.step(chunk, w.dt)
    p = parity(w, o, g)
    print("sectors", grid, p, flush=True)
    assert p["ok"], p
    assert g.stats()["rebuilds"] == o.num_rebuilds


def test_sectors_hot_rebuilds_and_frozen_exact():
    from paper_1801_10233_amd import spinlat as sl
    w = W.coupled_nve(n=6, T=1500.0)
    o = _oracle(w, O.SECT, (2, 2, 2))
    g = make_gpu(w)
    g.set_ordering(sl.SL_ORDER_SECTORS, (2, 2, 2))
    o.step(150, 2e-4); g.step(150, 2e-4)
    assert o.num_rebuilds >= 2 and g.stats()["rebuilds"] == o.num_rebuilds
    assert parity(w, o, g, tol_s=1e-9, rtol_v=1e-9)["ok"]
    f = W.spin_frozen(6)
    g = make_gpu(f)
    g.set_ordering(sl.SL_ORDER_SECTORS, (1, 1, 1))
    e0 = g.energy()["total"]
    g.step(100, 1e-4)
    g.step(10, 2e-2)
    assert abs(g.energy()["total"] / e0 - 1) < 1e-12
    o = _oracle(f, O.SECT)
    o.step(100, 1e-4); o.step(10, 2e-2)
    assert parity(f, o, g)["ok"]


def test_serial_order_matches_oracle():
    from paper_1801_10233_amd import spinlat as sl
    w = W.large_langevin(n=5)
    o = _oracle(w, O.SEQ)
    g = make_gpu(w)
    g.set_ordering(sl.SL_ORDER_SERIAL)
    o.step(30, w.dt); g.step(30, w.dt)
    p = parity(w, o, g)
    print("serial", p, flush=True)
    assert p["ok"], p


def test_ordering_arguments_and_switching():
    from paper_1801_10233_amd import spinlat as sl
    w = W.coupled_nve(n=6)
    g = make_gpu(w)
    with pytest.raises(sl.SpinLatError):
        g.set_ordering(sl.SL_ORDER_SECTORS, (3, 1, 1))     # 2.87 A sectors < 3.8 A
    with pytest.raises(sl.SpinLatError):
        g.set_ordering(7)
    # switching between orderings mid-run keeps each segment exact
    o = _oracle(w, O.COLOUR)
    g.step(20, w.dt); o.step(20, w.dt)
    g.set_ordering(sl.SL_ORDER_SECTORS, (2, 2, 2)); o.set_ordering(O.SECT, (2, 2, 2))
    g.step(20, w.dt); o.step(20, w.dt)
    g.set_ordering(sl.SL_ORDER_COLOUR); o.set_ordering(O.COLOUR)
    g.step(20, w.dt); o.step(20, w.dt)
    assert parity(w, o, g)["ok"]


def test_sector_and_colour_orderings_equivalent_at_scale():
    # E4 analogue: 16000 atoms, 4x4x4 subdomains (7.2 A sectors); energy and
    # |M| statistics of the two orderings agree
    from paper_1801_10233_amd import spinlat as sl
    w = W.coupled_nve(n=20)
    out = {}
    for name, ordering in (("colour", sl.SL_ORDER_COLOUR), ("sectors", sl.SL_ORDER_SECTORS)):
        g = make_gpu(w)
        g.set_ordering(ordering, (4, 4, 4))
        e0 = g.energy()["total"]
        es, ms = [], []
        for _ in range(10):
            g.step(100, w.dt)
            es.append(g.energy()["total"] - e0)
            ms.append(np.linalg.norm(g.magnetization()) / w.N)
        out[name] = (np.array(es) / w.N, np.array(ms), g.get_state()[2])
    (ec, mc, sc), (es_, ms_, ss) = out["colour"], out["sectors"]
    print("E4 colour dE/N", np.abs(ec).max(), "sectors dE/N", np.abs(es_).max(),
          "max |M| diff", np.abs(mc - ms_).max(), flush=True)
    assert np.abs(ec).max() < 1e-6 and np.abs(es_).max() < 1e-6
    assert np.abs(mc - ms_).max() < 2e-3
    assert np.abs(sc - ss).max() > 1e-12          # genuinely different orders
