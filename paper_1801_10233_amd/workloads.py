"""Seeded synthetic inputs for the spin-lattice step (bcc iron-like systems).

This module only *generates inputs*: lattice positions, unit spins, Maxwell
velocities and the named parameter presets of the five workloads. It holds
none of the integrator's arithmetic, so the CPU oracle and the HIP path can
both draw their inputs from here without sharing any method code.

Workloads (bcc, a = 2.8665 A, n cells per side, N = 2 n^3 atoms):

* ``spin_frozen``    n=10, N=2000, frozen lattice, Bethe-Slater exchange
  (alpha=0.1 eV, gamma=0.2, delta=1.2 A, cutoff 3.5 A), Zeeman 1 T along z,
  dt = 1e-4 ps.
* ``coupled_nve``    n=20, N=16000, m=55.845 amu, shifted-force Morse
  (D=0.4174 eV, alpha=1.3885 1/A, r0=2.845 A, cutoff 5 A) + the exchange
  above with its radial-derivative force, Maxwell velocities at 300 K.
* ``large_langevin`` n=60, N=432000, the coupled physics plus uniaxial
  anisotropy K=1e-4 eV along z and spin Langevin damping lambda=0.01 at
  300 K (Philox noise); ``large_nve`` is its undamped twin used for drift.
* ``batched``        64 replicas, n in [8, 24], T in [100, 1000] K, Zeeman
  0-5 T along random directions.

Units: A, ps, eV, amu, K, T.
"""
from __future__ import annotations

import dataclasses
import numpy as np

# Physical constants used only to draw Maxwell velocities (input generation).
KB_EV_PER_K = 8.617333262e-5
AMU_A2_PER_PS2_IN_EV = 1.66053906660e-27 * 1e4 / 1.602176634e-19

BCC_A = 2.8665
FE_MASS = 55.845


def bcc_lattice(n: int, a: float = BCC_A):
    """Perfect periodic bcc crystal of n^3 cubic cells.

    Atom id = 2*(i*n*n + j*n + k) + b, with i along z, j along y, k along x
    and b = 0 (corner) / 1 (body centre). Returns (r[N,3] float64, box[3]).
    """
    idx = np.arange(n, dtype=np.float64)
    i, j, k = np.meshgrid(idx, idx, idx, indexing="ij")
    base = np.stack([k.ravel(), j.ravel(), i.ravel()], axis=1)  # (x, y, z)
    r = np.empty((2 * n ** 3, 3), dtype=np.float64)
    r[0::2] = base * a
    r[1::2] = (base + 0.5) * a
    box = np.array([n * a, n * a, n * a], dtype=np.float64)
    return r, box


def random_unit_spins(N: int, seed: int):
    """Spins uniform on the unit sphere: z = 2u1 - 1, phi = 2 pi u2."""
    rng = np.random.default_rng(seed)
    u = rng.random((N, 2))
    z = 2.0 * u[:, 0] - 1.0
    phi = 2.0 * np.pi * u[:, 1]
    rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    s = np.stack([rho * np.cos(phi), rho * np.sin(phi), z], axis=1)
    s /= np.linalg.norm(s, axis=1, keepdims=True)
    return s


def maxwell_velocities(mass, T: float, seed: int):
    """Gaussian velocities (A/ps) at temperature T with zero total momentum,
    rescaled so that the kinetic temperature over 3N-3 degrees of freedom is
    exactly T (T = 0 gives zero velocities)."""
    mass = np.asarray(mass, dtype=np.float64)
    N = mass.shape[0]
    if T <= 0.0 or N < 2:
        return np.zeros((N, 3))
    rng = np.random.default_rng(seed)
    sigma = np.sqrt(KB_EV_PER_K * T / (mass * AMU_A2_PER_PS2_IN_EV))
    v = rng.standard_normal((N, 3)) * sigma[:, None]
    p = (mass[:, None] * v).sum(axis=0)
    v -= p / mass.sum()
    ke = 0.5 * (mass[:, None] * v * v).sum() * AMU_A2_PER_PS2_IN_EV
    t_now = 2.0 * ke / ((3 * N - 3) * KB_EV_PER_K)
    v *= np.sqrt(T / t_now)
    return v


def thermal_displacements(N: int, sigma: float, seed: int):
    """Isotropic Gaussian displacements (A), used to make disordered tests."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((N, 3)) * sigma


# ----------------------------------------------------------------------------
# Parameter presets (numbers only).

EXCHANGE_BJ = dict(ex_alpha=0.1, ex_gamma=0.2, ex_delta=1.2, ex_rc=3.5)
MORSE_BJ = dict(morse_on=1, morse_D=0.4174, morse_alpha=1.3885, morse_r0=2.845,
                morse_rc=5.0, morse_shift=1)
# Embedded-atom stand-in for the paper's tabulated EAM (Sec. 2): the
# Finnis-Sinclair potential for bcc iron (Finnis and Sinclair, Phil. Mag. A
# 50, 45 (1984)), fitted to a = 2.8665 A and a cohesive energy of 4.28 eV.
FS_FE = dict(eam_on=1, eam_A=1.828905, eam_d=3.569745, eam_beta=1.8, eam_c=3.40,
             eam_c0=1.2371147, eam_c1=-0.3592185, eam_c2=-0.0385607)
# Spin-orbit pair terms (appendix A; the paper's Co parameters are not
# available): Neel g1(r) and the DMI magnitude in the Bethe-Slater form,
# a tenth and a twentieth of the exchange scale, DMI vector n x e_ij, n = z.
NEEL_BJ = dict(neel_alpha=0.01, neel_gamma=0.2, neel_delta=1.2, neel_rc=3.5)
DMI_BJ = dict(dmi_alpha=0.005, dmi_gamma=0.0, dmi_delta=1.4, dmi_rc=3.5,
              dmi_n=(0.0, 0.0, 1.0))


@dataclasses.dataclass
class Workload:
    name: str
    n: int
    r: np.ndarray
    v: np.ndarray
    s: np.ndarray
    mass: np.ndarray
    box: np.ndarray
    pot: dict
    frozen: bool
    dt: float
    steps: int
    skin: float
    seed: int          # Philox key for the Langevin noise
    replica: int = 0
    # list-row order grid (A): neighbour displacements in bcc are multiples
    # of a/2, so rounding to that grid gives every row the same slot order
    row_quantum: float = BCC_A / 2

    @property
    def N(self):
        return self.r.shape[0]


def _pot(**kw):
    base = dict(morse_on=0, morse_D=0.0, morse_alpha=0.0, morse_r0=0.0,
                morse_rc=0.0, morse_shift=1, ex_alpha=0.0, ex_gamma=0.0,
                ex_delta=1.0, ex_rc=0.0, zeeman_g=2.0, B=(0.0, 0.0, 0.0),
                aniso_K=0.0, aniso_n=(0.0, 0.0, 1.0), lam=0.0,
                temperature=0.0, lat_gamma=0.0, lat_temperature=0.0,
                neel_alpha=0.0, neel_gamma=0.0, neel_delta=1.0, neel_rc=0.0,
                dmi_alpha=0.0, dmi_gamma=0.0, dmi_delta=1.0, dmi_rc=0.0,
                dmi_n=(0.0, 0.0, 1.0), eam_on=0, eam_A=0.0, eam_d=0.0,
                eam_beta=0.0, eam_c=0.0, eam_c0=0.0, eam_c1=0.0, eam_c2=0.0,
                ex_shift=0, aniso_split=0)
    base.update(kw)
    return base


def spin_frozen(n: int = 10, seed: int = 1001) -> Workload:
    r, box = bcc_lattice(n)
    N = r.shape[0]
    return Workload("spin_frozen", n, r, np.zeros((N, 3)),
                    random_unit_spins(N, seed), np.full(N, FE_MASS), box,
                    _pot(**EXCHANGE_BJ, B=(0.0, 0.0, 1.0)), True, 1e-4, 1000,
                    0.0, 0)


def coupled_nve(n: int = 20, T: float = 300.0, spin_seed: int = 2001,
                vel_seed: int = 2002) -> Workload:
    r, box = bcc_lattice(n)
    N = r.shape[0]
    m = np.full(N, FE_MASS)
    return Workload("coupled_nve", n, r, maxwell_velocities(m, T, vel_seed),
                    random_unit_spins(N, spin_seed), m, box,
                    _pot(**EXCHANGE_BJ, **MORSE_BJ), False, 1e-4, 10000, 0.3,
                    0)


def large_langevin(n: int = 60, nve: bool = False, spin_seed: int = 3001,
                   vel_seed: int = 3002, key: int = 3003) -> Workload:
    r, box = bcc_lattice(n)
    N = r.shape[0]
    m = np.full(N, FE_MASS)
    pot = _pot(**EXCHANGE_BJ, **MORSE_BJ, aniso_K=1e-4, aniso_n=(0.0, 0.0, 1.0),
               lam=0.0 if nve else 0.01, temperature=0.0 if nve else 300.0)
    return Workload("large_nve" if nve else "large_langevin", n, r,
                    maxwell_velocities(m, 300.0, vel_seed),
                    random_unit_spins(N, spin_seed), m, box, pot, False, 1e-4,
                    1000, 0.3, key)


def two_thermostat(n: int = 10, bath: str = "spin", T: float = 300.0,
                   lam: float = 0.01, lat_gamma: float = 50.0,
                   spin_seed: int = 6001, vel_seed: int = 6002,
                   key: int = 6003) -> Workload:
    """Relaxation with one bath (Sec. 4.2): bath="spin" starts a lattice at
    rest (T_L = 0) with random spins under a spin bath at T; bath="lattice"
    starts spins aligned along z (T_S = 0) and Maxwell velocities at T under
    a lattice bath at T (friction lat_gamma, amu/ps)."""
    r, box = bcc_lattice(n)
    N = r.shape[0]
    m = np.full(N, FE_MASS)
    if bath == "spin":
        v = np.zeros((N, 3))
        s = random_unit_spins(N, spin_seed)
        pot = _pot(**EXCHANGE_BJ, **MORSE_BJ, lam=lam, temperature=T)
    else:
        v = maxwell_velocities(m, T, vel_seed)
        s = np.tile([0.0, 0.0, 1.0], (N, 1))
        pot = _pot(**EXCHANGE_BJ, **MORSE_BJ, lat_gamma=lat_gamma,
                   lat_temperature=T)
    return Workload("two_thermostat_" + bath, n, r, v, s, m, box, pot, False,
                    1e-4, 10000, 0.3, key)


def energy_repartition(n: int = 10, T: float = 200.0, spin_seed: int = 7001,
                       vel_seed: int = 7002) -> Workload:
    """NVE run from random (paramagnetic) spins and Maxwell velocities at T
    on the perfect lattice (Sec. 4.2, the energy-repartition run)."""
    r, box = bcc_lattice(n)
    N = r.shape[0]
    m = np.full(N, FE_MASS)
    return Workload("energy_repartition", n, r, maxwell_velocities(m, T, vel_seed),
                    random_unit_spins(N, spin_seed), m, box,
                    _pot(**EXCHANGE_BJ, **MORSE_BJ), False, 1e-4, 10000, 0.3, 0)


def soc_coupled(n: int = 8, T: float = 300.0, frozen: bool = False,
                spin_seed: int = 8001, vel_seed: int = 8002, key: int = 8003,
                lam: float = 0.0) -> Workload:
    """Coupled run with the Neel and DMI pair terms added to the exchange
    (Sec. 2, appendix A): Maxwell velocities at T (zero when frozen), random
    spins, optional spin bath."""
    r, box = bcc_lattice(n)
    N = r.shape[0]
    m = np.full(N, FE_MASS)
    v = np.zeros((N, 3)) if frozen else maxwell_velocities(m, T, vel_seed)
    pot = _pot(**EXCHANGE_BJ, **({} if frozen else MORSE_BJ), **NEEL_BJ, **DMI_BJ,
               B=(0.0, 0.0, 0.5), lam=lam, temperature=T if lam > 0 else 0.0)
    return Workload("soc_frozen" if frozen else "soc_coupled", n, r, v,
                    random_unit_spins(N, spin_seed), m, box, pot, frozen, 1e-4,
                    1000, 0.0 if frozen else 0.3, key)


def eam_coupled(n: int = 20, T: float = 300.0, spin_seed: int = 9001,
                vel_seed: int = 9002, key: int = 9003, lam: float = 0.0) -> Workload:
    """Coupled run with the embedded-atom (Finnis-Sinclair iron) mechanical
    potential in place of Morse, Bethe-Slater exchange, Maxwell velocities
    at T and random spins."""
    r, box = bcc_lattice(n)
    N = r.shape[0]
    m = np.full(N, FE_MASS)
    pot = _pot(**EXCHANGE_BJ, **FS_FE, lam=lam, temperature=T if lam > 0 else 0.0)
    return Workload("eam_coupled", n, r, maxwell_velocities(m, T, vel_seed),
                    random_unit_spins(N, spin_seed), m, box, pot, False, 1e-4,
                    1000, 0.3, key)


def batched_replicas(R: int = 64, seed: int = 4004, n_lo: int = 8,
                     n_hi: int = 24):
    """R independent replicas of uneven size, temperature and field."""
    rng = np.random.default_rng(seed)
    out = []
    for rep in range(R):
        n = int(rng.integers(n_lo, n_hi + 1))
        T = float(rng.uniform(100.0, 1000.0))
        Bmag = float(rng.uniform(0.0, 5.0))
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        r, box = bcc_lattice(n)
        N = r.shape[0]
        m = np.full(N, FE_MASS)
        pot = _pot(**EXCHANGE_BJ, **MORSE_BJ, B=tuple(Bmag * d), aniso_K=1e-4,
                   lam=0.01, temperature=T)
        out.append(Workload(f"replica{rep}", n, r,
                            maxwell_velocities(m, T, seed * 1000 + 2 * rep),
                            random_unit_spins(N, seed * 1000 + 2 * rep + 1),
                            m, box, pot, False, 1e-4, 1000, 0.3,
                            seed, replica=rep))
    return out
