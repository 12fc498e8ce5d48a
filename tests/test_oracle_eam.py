"""Pins of the oracle's embedded-atom mechanical potential (Finnis-Sinclair
form, standing in for the paper's tabulated EAM; Sec. 2).

The Finnis-Sinclair iron parameters were fitted to the bcc lattice
constant 2.8665 A and the cohesive energy 4.28 eV: the oracle's perfect
crystal must reproduce both (the energy minimum over the lattice constant
and its depth). The many-body force is pinned by finite differences of the
energy (which catch a missing F'(rho_j) term or a wrong sign), and the
dynamics by momentum conservation, energy conservation with O(dt^2)
deviations and time reversibility."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1801_10233_amd import workloads as W

EAM = dict(W._pot(**W.FS_FE))


def _crystal_energy(a, n=5):
    r, box = W.bcc_lattice(n, a)
    N = r.shape[0]
    s = np.tile([0.0, 0.0, 1.0], (N, 1))
    o = O.Oracle(r, np.zeros((N, 3)), s, np.full(N, W.FE_MASS), box, EAM, frozen=False, skin=0.3)
    return o.energy()["pair"] / N


def test_fs_iron_cohesive_energy_and_lattice_constant():
    e0 = _crystal_energy(W.BCC_A)
    assert e0 == pytest.approx(-4.28, abs=2e-3)
    grid = W.BCC_A + np.linspace(-0.01, 0.01, 21)
    es = np.array([_crystal_energy(a) for a in grid])
    c2, c1, _ = np.polyfit(grid - W.BCC_A, es, 2)
    a_min = W.BCC_A - c1 / (2 * c2)
    assert abs(a_min - W.BCC_A) < 2e-3, a_min
    assert c2 > 0


def test_eam_force_and_omega_are_energy_gradients():
    r, box = W.bcc_lattice(4)
    N = r.shape[0]
    r = r + W.thermal_displacements(N, 0.12, 31)
    s = W.random_unit_spins(N, 32)
    p = dict(W._pot(**W.EXCHANGE_BJ, **W.FS_FE, B=(0.3, -0.2, 1.0)))
    o = O.Oracle(r, np.zeros((N, 3)), s, np.full(N, W.FE_MASS), box, p, frozen=False, skin=0.3)
    o.build()
    F = o.forces()
    h = 1e-5
    rng = np.random.default_rng(6)
    for i in rng.choice(N, 8, replace=False):
        for a in range(3):
            rp = r.copy(); rp[i, a] += h
            rm = r.copy(); rm[i, a] -= h
            o.set_state(r=rp); o.build(); Ep = o.energy()["total"]
            o.set_state(r=rm); o.build(); Em = o.energy()["total"]
            # the crystal's energy is ~550 eV, so the difference quotient
            # carries ~1e-8 eV/A of rounding at h = 1e-5
            assert -(Ep - Em) / (2 * h) == pytest.approx(F[i, a], rel=1e-6, abs=5e-8)
    o.set_state(r=r)


def test_eam_dynamics_conserves_momentum_and_energy_to_second_order():
    w = W.eam_coupled(n=4, T=600.0)
    P0 = (w.mass[:, None] * w.v).sum(0)
    devs = []
    for dt in (4e-4, 2e-4):
        o = O.Oracle(w.r, w.v, w.s, w.mass, w.box, w.pot, frozen=False, skin=w.skin)
        e0 = o.energy()["total"]
        nst = int(round(0.04 / dt))
        dev = 0.0
        for _ in range(8):
            o.step(nst // 8, dt)
            dev = max(dev, abs(o.energy()["total"] - e0))
        devs.append(dev)
        _, v, _ = o.get_state()
        assert np.abs((w.mass[:, None] * v).sum(0) - P0).max() < 1e-10 * np.abs(w.mass[:, None] * w.v).sum()
    assert 3.0 < devs[0] / devs[1] < 5.0, devs


def test_eam_reversibility():
    w = W.eam_coupled(n=4)
    o = O.Oracle(w.r, w.v, w.s, w.mass, w.box, w.pot, frozen=False, skin=w.skin)
    o.build()
    o.step(40, 1e-4)
    r0, v0, s0 = o.get_state()
    o.step(40, 1e-4)
    o.step(40, -1e-4)
    r1, v1, s1 = o.get_state()
    assert np.abs(r1 - r0).max() < 1e-10 * w.box[0]
    assert np.abs(s1 - s0).max() < 1e-10
