"""Oracle pins of the two smooth forms (off by default) and of the exact
energy loss of the literal form that they remove.

- Uniaxial anisotropy (appendix A) with the whole precession vector taken at
  the spin's value before the update (the literal reading, Sec. 3): the
  Cayley rotation keeps s.omega fixed, so each update changes the energy by
  exactly -K (delta s.n)^2. On a frozen lattice the energy therefore falls
  at every step for K > 0 and rises for K < 0.
- The symmetric split A(h/2) X(h) A(h/2) is time-reversible and keeps the
  frozen-lattice energy to roundoff, converges as dt^2, and equals the
  literal update when K = 0.
- The shifted exchange is continuous with its derivative at the cutoff
  (Eq. BSfunction cuts J with a step): a dimer that flies through R_c keeps
  its energy with it, and jumps by J(R_c) s_i.s_j without it.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1801_10233_amd import workloads as W
from tests.common import make_oracle


def _frozen(K, split, n=6, seed=1001, n_axis=(0.0, 0.6, 0.8)):
    w = W.spin_frozen(n, seed=seed)
    w.pot = dict(w.pot, aniso_K=K, aniso_n=n_axis, aniso_split=split)
    return w


@pytest.mark.parametrize("K", [2e-3, -2e-3])
def test_literal_anisotropy_loses_energy_every_step(K):
    w = _frozen(K, 0)
    o = make_oracle(w)
    E = [o.energy()["total"]]
    for _ in range(30):
        o.step(1, 1e-3)
        E.append(o.energy()["total"])
    d = np.diff(E)
    # strictly monotone, with the sign of -K, every single step
    assert np.all(np.sign(d) == -np.sign(K)), d
    # size: K <(delta s.n)^2> summed over 4 updates of each spin
    assert 1e-14 < np.abs(d).max() / w.N < abs(K) * 1e-3


def test_literal_update_loses_exactly_K_delta_sn_squared():
    # One spin in a field with anisotropy. With omega taken at the spin's
    # value before the update, the rotation keeps s.omega, so
    # mu B.ds + 2K (s0.n) d(s.n) = 0 and the energy -mu B.s - K (s.n)^2
    # changes by exactly -K (d(s.n))^2. A wrong factor in the anisotropy's
    # share of omega, or omega taken after the update, breaks the identity.
    B = (0.2, -0.4, 1.0)
    K = 0.03
    n = np.array([0.0, 0.6, 0.8])
    s0 = np.array([[0.48, 0.6, 0.64]])
    o = O.Oracle(np.zeros((1, 3)), np.zeros((1, 3)), s0, np.ones(1), np.array([20.0] * 3),
                 W._pot(B=B, aniso_K=K, aniso_n=tuple(n)), frozen=True, skin=0.0)
    dt = 4e-3
    s = s0[0].copy()
    E = o.energy()["total"]
    loss = 0.0
    for _ in range(4):                     # one step of a one-class system: 4 updates of dt/4
        w = o.omega()[0]
        s1 = O.cayley(s, w, dt / 4)
        o.set_state(s=s1[None, :])
        E1 = o.energy()["total"]
        d = float(np.dot(s1 - s, n))
        assert d != 0.0
        assert abs((E1 - E) - (-K * d * d)) < 1e-15 * max(1.0, abs(E)), (E1 - E, -K * d * d)
        loss += K * d * d
        s, E = s1, E1
    # the oracle's own step is those four updates
    o.set_state(s=s0)
    E0 = o.energy()["total"]
    o.step(1, dt)
    assert np.abs(o.get_state()[2][0] - s).max() < 1e-15
    assert abs((o.energy()["total"] - E0) + loss) < 1e-15


def test_literal_anisotropy_loss_is_first_order_in_dt():
    # one spin in a field with anisotropy: each update loses K (delta s.n)^2
    # = O(h^2), so over a fixed time the total loss is O(dt): halving dt
    # halves it
    B = (0.0, 0.3, 1.0)
    K = 0.05
    losses = []
    for dt in (4e-3, 2e-3, 1e-3):
        o = O.Oracle(np.zeros((1, 3)), np.zeros((1, 3)), np.array([[0.6, 0.0, 0.8]]),
                     np.ones(1), np.array([20.0, 20.0, 20.0]),
                     W._pot(B=B, aniso_K=K, aniso_n=(0.0, 0.0, 1.0)), frozen=True, skin=0.0)
        e0 = o.energy()["total"]
        o.step(int(round(0.4 / dt)), dt)
        losses.append(e0 - o.energy()["total"])
    losses = np.array(losses)
    assert np.all(losses > 0)
    r = losses[:-1] / losses[1:]
    assert np.all(np.abs(r - 2.0) < 0.1), r


def _energy_series(w, nsteps, dt, every):
    o = make_oracle(w)
    E = [o.energy()["total"]]
    for _ in range(nsteps // every):
        o.step(every, dt)
        E.append(o.energy()["total"])
    return o, np.array(E)


def test_split_anisotropy_keeps_energy_and_is_reversible():
    # a time-reversible second-order scheme: the energy error stays bounded
    # (no trend over a long run) and scales as dt^2; the literal form loses
    # energy at every step instead
    for K in (2e-3, -2e-3):
        w = _frozen(K, 1)
        o, E = _energy_series(w, 600, 1e-3, 10)
        dev = np.abs(E - E[0])
        assert dev[31:].max() < 1.5 * dev[:31].max()          # bounded, no growth
        _, Eh = _energy_series(w, 1200, 5e-4, 20)
        ratio = dev.max() / np.abs(Eh - Eh[0]).max()
        assert 3.0 < ratio < 5.5, ratio                        # dt^2
        _, El = _energy_series(_frozen(K, 0), 600, 1e-3, 10)
        assert abs(El[-1] - El[0]) > 20 * dev.max()
        o.step(600, -1e-3)
        _, _, s = o.get_state()
        assert np.abs(s - w.s).max() < 1e-11
    # the literal form is not reversible with anisotropy
    w = _frozen(2e-3, 0)
    o = make_oracle(w)
    o.step(300, 1e-3)
    o.step(300, -1e-3)
    assert np.abs(o.get_state()[2] - w.s).max() > 1e-6


def test_split_anisotropy_converges_as_dt_squared():
    # the same time span at dt, dt/2, dt/4; differences to the finest run
    # fall by about 4 per halving
    w = _frozen(5e-3, 1, n=4)
    out = []
    for dt in (4e-3, 2e-3, 1e-3, 5e-4):
        o = make_oracle(w)
        o.step(int(round(0.2 / dt)), dt)
        out.append(o.get_state()[2])
    e = [np.abs(out[k] - out[-1]).max() for k in range(3)]
    assert 3.0 < e[0] / e[1] < 5.5 and 3.0 < e[1] / e[2] < 5.5, e


def test_split_anisotropy_without_anisotropy_is_the_literal_update():
    a = make_oracle(_frozen(0.0, 1))
    b = make_oracle(_frozen(0.0, 0))
    a.step(20, 1e-3)
    b.step(20, 1e-3)
    assert np.array_equal(a.get_state()[2], b.get_state()[2])


def test_shifted_exchange_is_continuous_at_the_cutoff():
    p = dict(W.EXCHANGE_BJ, ex_shift=1)
    rc = p["ex_rc"]
    for eps in (1e-3, 1e-5):
        J, dJ = O.J(p, rc - eps)
        assert abs(J) < 2e-3 * eps and abs(dJ) < 1e-2 * eps ** 0.5
    assert O.J(p, rc + 1e-9) == (0.0, 0.0)
    # inside, the shift is J(rc) + (r^2 - rc^2) J'(rc)/(2 rc) of the literal form
    q = dict(W.EXCHANGE_BJ)
    Jc, dJc = O.J(q, rc * (1 - 1e-15))
    for r in (2.4825, 2.8665, 3.2):
        J0, dJ0 = O.J(q, r)
        J1, dJ1 = O.J(p, r)
        assert J1 == pytest.approx(J0 - Jc - (r * r - rc * rc) * dJc / (2 * rc), rel=1e-12,
                                   abs=1e-15)
        assert dJ1 == pytest.approx(dJ0 - r * dJc / rc, rel=1e-12, abs=1e-15)


@pytest.mark.parametrize("shift", [0, 1])
def test_dimer_through_the_exchange_cutoff(shift):
    # two atoms with parallel spins (no precession), exchange only, flying
    # apart through R_c = 3.5 A
    pot = W._pot(**dict(W.EXCHANGE_BJ, ex_shift=shift))
    r = np.array([[0.0, 0.0, 0.0], [3.3, 0.0, 0.0]])
    v = np.array([[-5.0, 0.0, 0.0], [5.0, 0.0, 0.0]])
    s = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, 1.0]])
    o = O.Oracle(r, v, s, np.full(2, W.FE_MASS), np.array([20.0, 20.0, 20.0]), pot,
                 frozen=False, skin=0.3)
    e0 = o.energy()["total"]
    o.step(400, 1e-4)                      # 0.4 A further apart: 3.5 A crossed
    rr, _, _ = o.get_state()
    assert np.linalg.norm(rr[1] - rr[0]) > 3.55
    de = o.energy()["total"] - e0
    Jc = float(O.J(dict(W.EXCHANGE_BJ), 3.5 * (1 - 1e-15))[0][0])
    if shift:
        assert abs(de) < 1e-9
    else:
        # the step of the literal cut: -J s.s inside, 0 outside
        assert de == pytest.approx(Jc, rel=1e-2)


def test_shifted_exchange_forces_and_fields_are_derivatives():
    w = W.coupled_nve(n=4)
    w.r = w.r + W.thermal_displacements(w.N, 0.15, 8)
    w.pot = dict(w.pot, ex_shift=1)
    o = make_oracle(w)
    F = o.forces()
    e0 = o.energy()
    h = 1e-6
    for i, a in ((3, 0), (17, 1), (40, 2)):
        rp = w.r.copy(); rp[i, a] += h
        rm = w.r.copy(); rm[i, a] -= h
        o.set_state(r=rp); ep = o.energy()["total"]
        o.set_state(r=rm); em = o.energy()["total"]
        fd = -(ep - em) / (2 * h)
        assert fd == pytest.approx(F[i, a], rel=1e-6, abs=1e-8)
    o.set_state(r=w.r)
    assert o.energy()["total"] == pytest.approx(e0["total"], rel=1e-14)
