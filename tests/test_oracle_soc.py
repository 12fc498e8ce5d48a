"""Pins of the oracle's spin-orbit pair terms (appendix A): the Neel
pseudo-dipolar anisotropy and the Dzyaloshinskii-Moriya interaction.

Each check reaches the oracle by a route other than its own code: dimer
energies evaluated by hand from the definitions (with the radial function
taken equal to the exchange J(r), pinned elsewhere), lattice sums over the
bcc shells enumerated here, finite differences of the energy, the exact
energy conservation of the colour sweep on a frozen lattice and momentum
conservation. A wrong sign, a dropped 1/3, a transposed cross product or a
pair counted twice fails one of them."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1801_10233_amd import workloads as W

BASE = dict(morse_on=0, morse_D=0.0, morse_alpha=0.0, morse_r0=0.0, morse_rc=0.0,
            morse_shift=1, ex_alpha=0.0, ex_gamma=0.2, ex_delta=1.2, ex_rc=3.5,
            zeeman_g=2.0, B=(0.0, 0.0, 0.0), aniso_K=0.0, aniso_n=(0.0, 0.0, 1.0),
            lam=0.0, temperature=0.0)
EXF = dict(W.EXCHANGE_BJ)


def _jr(r):
    """Exchange J(r) of the reference parameters (one value)."""
    return float(O.J(dict(BASE, **EXF), float(r))[0][0])


def _same_radial(which):
    """Neel or DMI radial function set equal to the exchange J(r)."""
    p = dict(BASE)
    if which == "neel":
        p.update(neel_alpha=EXF["ex_alpha"], neel_gamma=EXF["ex_gamma"],
                 neel_delta=EXF["ex_delta"], neel_rc=EXF["ex_rc"])
    else:
        p.update(dmi_alpha=EXF["ex_alpha"], dmi_gamma=EXF["ex_gamma"],
                 dmi_delta=EXF["ex_delta"], dmi_rc=EXF["ex_rc"], dmi_n=(0.0, 0.0, 1.0))
    return p


def _dimer(p, si, sj, r=2.6):
    pos = np.array([[5.0, 5.0, 5.0], [5.0 + r, 5.0, 5.0]])
    s = np.array([si, sj], dtype=float)
    o = O.Oracle(pos, np.zeros((2, 3)), s, [1.0, 1.0], [20.0, 20.0, 20.0], p, frozen=True)
    return o


def test_neel_dimer_closed_form():
    p = _same_radial("neel")
    g1 = _jr(2.6)
    x, y, z = (1, 0, 0), (0, 1, 0), (0, 0, 1)
    # E = -g1 [(e.s_i)(e.s_j) - s_i.s_j/3] with e along x
    for si, sj, want in [(x, x, -2.0 / 3.0), (y, y, 1.0 / 3.0), (z, z, 1.0 / 3.0),
                         (x, y, 0.0), ((-1, 0, 0), x, 2.0 / 3.0)]:
        o = _dimer(p, si, sj)
        en, ed = o.soc_energy()
        assert en == pytest.approx(want * g1, rel=1e-13, abs=1e-16), (si, sj)
        assert ed == 0.0
        assert o.energy()["exchange"] == pytest.approx(want * g1, rel=1e-13, abs=1e-16)


def test_dmi_dimer_closed_form():
    p = _same_radial("dmi")
    d = _jr(2.6)
    x, y, z = (1, 0, 0), (0, 1, 0), (0, 0, 1)
    # j sits at +x of i: e_ij = x, D_ij = d (z x x) = d y; E = D.(s_i x s_j)
    for si, sj, want in [(z, x, 1.0), (x, z, -1.0), (x, x, 0.0), (y, z, 0.0),
                         (x, y, 0.0)]:
        o = _dimer(p, si, sj)
        en, ed = o.soc_energy()
        assert en == 0.0
        assert ed == pytest.approx(want * d, rel=1e-13, abs=1e-16), (si, sj)


def _shells(a, c, rc):
    """Neighbour vectors of a body-centred tetragonal lattice (a, a, c)
    within rc, enumerated directly."""
    out = []
    for i in range(-3, 4):
        for j in range(-3, 4):
            for k in range(-3, 4):
                for b in (0.0, 0.5):
                    v = np.array([(i + b) * a, (j + b) * a, (k + b) * c])
                    rr = np.linalg.norm(v)
                    if 1e-9 < rr < rc:
                        out.append(v)
    return np.array(out)


@pytest.mark.parametrize("c_over_a", [1.0, 1.03])
def test_neel_uniform_state_lattice_sum(c_over_a):
    # cubic symmetry: every bcc shell has sum_j (e_j.s)^2 = n_shell/3, so the
    # Neel energy of a uniform state vanishes in any direction; a tetragonal
    # strain gives a uniaxial energy, compared with the lattice sum
    n, a = 6, W.BCC_A
    r, box = W.bcc_lattice(n)
    r = r * np.array([1.0, 1.0, c_over_a])
    box = box * np.array([1.0, 1.0, c_over_a])
    N = r.shape[0]
    p = _same_radial("neel")
    vecs = _shells(a, a * c_over_a, EXF["ex_rc"])
    g1 = np.array([_jr(np.linalg.norm(v)) for v in vecs])
    E = np.array([v / np.linalg.norm(v) for v in vecs])
    rng = np.random.default_rng(4)
    for _ in range(3):
        sdir = rng.standard_normal(3); sdir /= np.linalg.norm(sdir)
        s = np.tile(sdir, (N, 1))
        o = O.Oracle(r, np.zeros((N, 3)), s, np.ones(N), box, p, frozen=True)
        en, _ = o.soc_energy()
        want = -0.5 * N * np.sum(g1 * ((E @ sdir) ** 2 - 1.0 / 3.0))
        scale = 0.5 * N * np.abs(g1).sum()
        assert abs(en - want) < 1e-12 * scale, (en, want)
        if c_over_a == 1.0:
            assert abs(en) < 1e-12 * scale


def test_dmi_spiral_lattice_sum():
    # cycloid s(x) = (cos qx, 0, sin qx) along x (rotation plane holding the
    # DMI axis z): E_DMI per atom is half the shell sum of
    # d(r) (z x e).(s(0) x s(x_j)), enumerated here; the two senses of
    # rotation differ in sign (DMI selects a chirality)
    n = 6
    r, box = W.bcc_lattice(n)
    N = r.shape[0]
    p = _same_radial("dmi")
    vecs = _shells(W.BCC_A, W.BCC_A, EXF["ex_rc"])
    dr = np.array([_jr(np.linalg.norm(v)) for v in vecs])
    res = []
    for m in (1, -1):
        q = 2 * math.pi * m / box[0]
        s = np.stack([np.cos(q * r[:, 0]), np.zeros(N), np.sin(q * r[:, 0])], axis=1)
        o = O.Oracle(r, np.zeros((N, 3)), s, np.ones(N), box, p, frozen=True)
        _, ed = o.soc_energy()
        s0 = np.array([1.0, 0.0, 0.0])
        want = 0.0
        for v, d in zip(vecs, dr):
            e = v / np.linalg.norm(v)
            sj = np.array([math.cos(q * v[0]), 0.0, math.sin(q * v[0])])
            want += d * np.dot(np.cross([0.0, 0.0, 1.0], e), np.cross(s0, sj))
        want *= 0.5 * N
        assert ed == pytest.approx(want, rel=1e-11, abs=1e-14)
        res.append(ed)
    assert res[0] == pytest.approx(-res[1], rel=1e-11)
    assert abs(res[0]) > 1e-6


def test_soc_force_and_omega_are_energy_gradients():
    r, box = W.bcc_lattice(4)
    N = r.shape[0]
    r = r + W.thermal_displacements(N, 0.12, 21)
    s = W.random_unit_spins(N, 22)
    p = dict(BASE, **W.EXCHANGE_BJ, **W.MORSE_BJ, **W.NEEL_BJ, **W.DMI_BJ,
             B=(0.3, -0.2, 1.0), aniso_K=1e-3, aniso_n=(0.0, 0.6, 0.8))
    p["dmi_n"] = (0.6, 0.0, 0.8)
    m = np.full(N, W.FE_MASS)
    o = O.Oracle(r, np.zeros((N, 3)), s, m, box, p, frozen=False, skin=0.3)
    o.build()
    F = o.forces()
    w = o.omega()
    h = 1e-5
    rng = np.random.default_rng(5)
    for i in rng.choice(N, 6, replace=False):
        for a in range(3):
            rp = r.copy(); rp[i, a] += h
            rm = r.copy(); rm[i, a] -= h
            o.set_state(r=rp); o.build(); Ep = o.energy()["total"]
            o.set_state(r=rm); o.build(); Em = o.energy()["total"]
            assert -(Ep - Em) / (2 * h) == pytest.approx(F[i, a], rel=1e-7, abs=1e-8)
            sp = s.copy(); sp[i, a] += h
            sm = s.copy(); sm[i, a] -= h
            o.set_state(r=r, s=sp); o.build()
            e = o.energy(); Ep = e["exchange"] + e["zeeman"] + e["aniso"]
            o.set_state(s=sm); o.build()
            e = o.energy(); Em = e["exchange"] + e["zeeman"] + e["aniso"]
            o.set_state(s=s)
            assert -(Ep - Em) / (2 * h) / O.HBAR == pytest.approx(w[i, a], rel=1e-7, abs=1e-6)


def test_soc_exact_energy_frozen_and_momentum_coupled():
    # the Neel and DMI fields on s_i do not depend on s_i, so each colour
    # update keeps the energy exactly (frozen lattice, any dt)
    w = W.soc_coupled(n=6, frozen=True)
    o = O.Oracle(w.r, w.v, w.s, w.mass, w.box, w.pot, frozen=True)
    e0 = o.energy()["total"]
    o.step(200, 1e-4)
    o.step(10, 3e-2)
    assert abs((o.energy()["total"] - e0) / e0) < 1e-12
    # coupled: total momentum conserved (pair forces antisymmetric)
    w = W.soc_coupled(n=5)
    o = O.Oracle(w.r, w.v, w.s, w.mass, w.box, w.pot, frozen=False, skin=w.skin)
    P0 = (w.mass[:, None] * w.v).sum(0)
    o.step(100, 1e-4)
    _, v, _ = o.get_state()
    assert np.abs((w.mass[:, None] * v).sum(0) - P0).max() < 1e-10 * np.abs(w.mass[:, None] * w.v).sum()
    # and the step stays time reversible
    r0, v0, s0 = o.get_state()
    o.step(50, 1e-4)
    o.step(50, -1e-4)
    r1, v1, s1 = o.get_state()
    assert np.abs(s1 - s0).max() < 1e-10
    assert np.abs(r1 - r0).max() < 1e-10 * w.box[0]
