"""ctypes wrapper of the serial FP64 CPU oracle (``liboracle.so``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU baseline leg of the benchmark, never by the product package. The
library is built from ``oracle.c`` with gcc (``build()``), with no
fast-math and no code shared with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")

HBAR = 6.582119569e-4
KB = 8.617333262e-5
MUB = 5.7883818060e-5
MVV2E = 1.0364269652680506e-4

COLOUR, SEQ, SECT, JACOBI = 0, 1, 2, 3
# key tag of the lattice-noise Philox stream (key = seed XOR tag)
LATTICE_KEY_TAG = 0x6C61747469636521


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc -O2 (IEEE semantics, no contraction)."""
    srcs = [os.path.join(HERE, "oracle.c"), os.path.join(HERE, "mlp.c")]
    newest = max(os.path.getmtime(x) for x in srcs)
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < newest:
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared",
                               "-ffp-contract=off", "-fno-fast-math", "-o", tmp,
                               *srcs, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class Pot(C.Structure):
    _fields_ = [("morse_on", C.c_int), ("morse_D", C.c_double),
                ("morse_alpha", C.c_double), ("morse_r0", C.c_double),
                ("morse_rc", C.c_double), ("morse_shift", C.c_int),
                ("ex_alpha", C.c_double), ("ex_gamma", C.c_double),
                ("ex_delta", C.c_double), ("ex_rc", C.c_double),
                ("zeeman_g", C.c_double), ("B", C.c_double * 3),
                ("aniso_K", C.c_double), ("aniso_n", C.c_double * 3),
                ("lam", C.c_double), ("temperature", C.c_double),
                ("lat_gamma", C.c_double), ("lat_temperature", C.c_double),
                ("neel_alpha", C.c_double), ("neel_gamma", C.c_double),
                ("neel_delta", C.c_double), ("neel_rc", C.c_double),
                ("dmi_alpha", C.c_double), ("dmi_gamma", C.c_double),
                ("dmi_delta", C.c_double), ("dmi_rc", C.c_double),
                ("dmi_n", C.c_double * 3), ("eam_on", C.c_int),
                ("eam_A", C.c_double), ("eam_d", C.c_double), ("eam_beta", C.c_double),
                ("eam_c", C.c_double), ("eam_c0", C.c_double), ("eam_c1", C.c_double),
                ("eam_c2", C.c_double), ("ex_shift", C.c_int), ("aniso_split", C.c_int)]


class MlpCfg(C.Structure):
    _fields_ = [("sigma", C.c_double), ("mu_step", C.c_double), ("sJ", C.c_double),
                ("sP", C.c_double), ("ex_rc", C.c_double), ("rc", C.c_double)]


def make_pot(d: dict) -> Pot:
    p = Pot()
    for k, v in d.items():
        if k in ("B", "aniso_n", "dmi_n"):
            setattr(p, k, (C.c_double * 3)(*v))
        else:
            setattr(p, k, v)
    return p


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.c_int, dp, C.c_int, C.c_double, C.c_uint64, C.c_uint32]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_set_state.argtypes = [C.c_void_p, dp, dp, dp, dp]
        L.orc_get_state.argtypes = [C.c_void_p, dp, dp, dp]
        L.orc_set_potential.argtypes = [C.c_void_p, C.POINTER(Pot)]
        L.orc_set_ordering.argtypes = [C.c_void_p, C.c_int, ip]
        L.orc_set_step_counter.argtypes = [C.c_void_p, C.c_int64]
        L.orc_get_step_counter.restype = C.c_int64
        L.orc_get_step_counter.argtypes = [C.c_void_p]
        L.orc_set_neighbor_list.argtypes = [C.c_void_p, ip, ip]
        L.orc_get_neighbor_list.restype = C.c_long
        L.orc_get_neighbor_list.argtypes = [C.c_void_p, ip, ip, ip, C.c_long]
        L.orc_build_now.argtypes = [C.c_void_p]
        L.orc_set_coloring.argtypes = [C.c_void_p, ip]
        L.orc_get_coloring.argtypes = [C.c_void_p, ip]
        L.orc_num_rebuilds.argtypes = [C.c_void_p]
        L.orc_step.argtypes = [C.c_void_p, C.c_int64, C.c_double]
        L.orc_energy.argtypes = [C.c_void_p, dp]
        L.orc_magnetization.argtypes = [C.c_void_p, dp]
        L.orc_temperatures.argtypes = [C.c_void_p, dp, dp]
        L.orc_soc_energy.argtypes = [C.c_void_p, dp, dp]
        L.orc_omega_all.argtypes = [C.c_void_p, dp]
        L.orc_force_all.argtypes = [C.c_void_p, dp]
        L.orc_J.restype = C.c_double
        L.orc_J.argtypes = [C.POINTER(Pot), C.c_double, dp]
        L.orc_V.restype = C.c_double
        L.orc_V.argtypes = [C.POINTER(Pot), C.c_double, dp]
        L.orc_cayley.argtypes = [dp, dp, C.c_double, dp]
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                        C.POINTER(C.c_uint32)]
        L.orc_gauss3.argtypes = [C.c_uint64, C.c_uint32, C.c_int64, C.c_uint32, C.c_int, dp]
        L.mlp_nparam.restype = C.c_int
        L.mlp_eval.argtypes = [C.POINTER(MlpCfg), dp, C.c_double, dp]
        L.mlp_grad_linear.argtypes = [C.POINTER(MlpCfg), dp, C.c_int, dp, dp, dp, dp, dp, dp]
        L.mlp_loss_grad.restype = C.c_double
        L.mlp_loss_grad.argtypes = [C.POINTER(MlpCfg), dp, C.c_int, dp, dp, dp, C.c_int, ip, ip,
                                    C.c_double, dp, dp, dp, dp]
        L.orc_set_mlp.argtypes = [C.c_void_p, C.POINTER(MlpCfg), dp]
        L.orc_brute_pairs.restype = C.c_long
        L.orc_brute_pairs.argtypes = [C.c_int, dp, dp, C.c_double, ip, ip, C.c_long]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


class Oracle:
    """One simulated system held by the C oracle (user atom order)."""

    def __init__(self, r, v, s, mass, box, pot: dict, frozen=False, skin=0.3,
                 seed=0, replica=0, ordering=COLOUR, sect_grid=(1, 1, 1)):
        L = lib()
        r = _f64(r, (-1, 3))
        self.N = r.shape[0]
        self._box = _f64(box, (3,))
        self.h = L.orc_create(self.N, _dp(self._box), int(frozen), float(skin),
                              int(seed), int(replica))
        if not self.h:
            raise RuntimeError("orc_create failed")
        self.frozen = frozen
        self.set_potential(pot)
        self.set_ordering(ordering, sect_grid)
        self.set_state(r, v, s, mass)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().orc_destroy(h)
            self.h = None

    def set_potential(self, pot: dict):
        self._pot = make_pot(pot)
        lib().orc_set_potential(self.h, C.byref(self._pot))

    def set_mlp(self, cfg, params):
        """Use the FP64 learned pair potential for J and V (None: analytic)."""
        if params is None:
            lib().orc_set_mlp(self.h, None, None)
        else:
            self._mp = _f64(params)
            self._mcfg = cfg
            lib().orc_set_mlp(self.h, C.byref(cfg), _dp(self._mp))

    def set_ordering(self, ordering, sect_grid=(1, 1, 1)):
        g = np.ascontiguousarray(sect_grid, dtype=np.int32)
        lib().orc_set_ordering(self.h, int(ordering), _ip(g))

    def set_state(self, r=None, v=None, s=None, mass=None):
        N = self.N
        args = []
        keep = []
        for a, shp in ((r, (N, 3)), (v, (N, 3)), (s, (N, 3)), (mass, (N,))):
            if a is None:
                args.append(None)
            else:
                x = _f64(a, shp)
                keep.append(x)
                args.append(_dp(x))
        lib().orc_set_state(self.h, *args)

    def get_state(self):
        r = np.empty((self.N, 3)); v = np.empty((self.N, 3)); s = np.empty((self.N, 3))
        lib().orc_get_state(self.h, _dp(r), _dp(v), _dp(s))
        return r, v, s

    def set_step_counter(self, k):
        lib().orc_set_step_counter(self.h, int(k))

    @property
    def step_counter(self):
        return lib().orc_get_step_counter(self.h)

    def set_neighbor_list(self, offsets, idx):
        o = np.ascontiguousarray(offsets, dtype=np.int32)
        i = np.ascontiguousarray(idx, dtype=np.int32)
        rc = lib().orc_set_neighbor_list(self.h, _ip(o), _ip(i))
        if rc:
            raise RuntimeError(f"orc_set_neighbor_list: {rc}")

    def build(self):
        rc = lib().orc_build_now(self.h)
        if rc:
            raise RuntimeError(f"orc_build_now: {rc}")

    def neighbor_list(self):
        """Returns (nspin[N], nall[N], rows: list of int arrays)."""
        ns = np.zeros(self.N, dtype=np.int32)
        na = np.zeros(self.N, dtype=np.int32)
        tot = lib().orc_get_neighbor_list(self.h, _ip(ns), _ip(na), None, 0)
        idx = np.zeros(max(tot, 1), dtype=np.int32)
        lib().orc_get_neighbor_list(self.h, _ip(ns), _ip(na), _ip(idx), tot)
        off = np.concatenate([[0], np.cumsum(na)])
        rows = [idx[off[i]:off[i + 1]] for i in range(self.N)]
        return ns, na, rows

    def set_coloring(self, colour):
        c = np.ascontiguousarray(colour, dtype=np.int32)
        if lib().orc_set_coloring(self.h, _ip(c)):
            raise ValueError("bad colouring")

    def coloring(self):
        c = np.zeros(self.N, dtype=np.int32)
        K = lib().orc_get_coloring(self.h, _ip(c))
        return c, K

    @property
    def num_rebuilds(self):
        return lib().orc_num_rebuilds(self.h)

    def step(self, n, dt):
        rc = lib().orc_step(self.h, int(n), float(dt))
        if rc:
            raise RuntimeError(f"orc_step: {rc}")

    def energy(self):
        e = np.zeros(6)
        lib().orc_energy(self.h, _dp(e))
        return dict(kin=e[0], pair=e[1], exchange=e[2], zeeman=e[3], aniso=e[4],
                    total=e[5])

    def magnetization(self):
        M = np.zeros(3)
        lib().orc_magnetization(self.h, _dp(M))
        return M

    def soc_energy(self):
        a = C.c_double(); b = C.c_double()
        lib().orc_soc_energy(self.h, C.byref(a), C.byref(b))
        return a.value, b.value

    def temperatures(self):
        tl = C.c_double(); ts = C.c_double()
        lib().orc_temperatures(self.h, C.byref(tl), C.byref(ts))
        return tl.value, ts.value

    def omega(self):
        w = np.zeros((self.N, 3))
        lib().orc_omega_all(self.h, _dp(w))
        return w

    def forces(self):
        F = np.zeros((self.N, 3))
        lib().orc_force_all(self.h, _dp(F))
        return F


def J(pot: dict, r):
    p = make_pot(pot)
    d = C.c_double()
    out = []
    for x in np.atleast_1d(r):
        val = lib().orc_J(C.byref(p), float(x), C.byref(d))
        out.append((val, d.value))
    a = np.array(out)
    return a[:, 0], a[:, 1]


def V(pot: dict, r):
    p = make_pot(pot)
    d = C.c_double()
    out = []
    for x in np.atleast_1d(r):
        val = lib().orc_V(C.byref(p), float(x), C.byref(d))
        out.append((val, d.value))
    a = np.array(out)
    return a[:, 0], a[:, 1]


def cayley(s, W, h):
    s = _f64(s, (3,)); W = _f64(W, (3,)); o = np.zeros(3)
    lib().orc_cayley(_dp(s), _dp(W), float(h), _dp(o))
    return o


def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(x) & 0xffffffff for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xffffffff for x in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint64)


def gauss3(seed, atom_id, step, replica, sub):
    o = np.zeros(3)
    lib().orc_gauss3(int(seed), int(atom_id), int(step), int(replica), int(sub), _dp(o))
    return o


def brute_pairs(r, box, rcut):
    r = _f64(r, (-1, 3)); box = _f64(box, (3,))
    N = r.shape[0]
    n = lib().orc_brute_pairs(N, _dp(box), _dp(r), float(rcut), None, None, 0)
    pi = np.zeros(max(n, 1), dtype=np.int32); pj = np.zeros(max(n, 1), dtype=np.int32)
    lib().orc_brute_pairs(N, _dp(box), _dp(r), float(rcut), _ip(pi), _ip(pj), n)
    return pi[:n], pj[:n]


# --------------------------------------------------------------------------
# Per-pair MLP (mlp.c): J(r), phi(r) and derivatives; training gradients.
def mlp_cfg(sigma=0.4, mu_step=5.0 / 15.0, sJ=0.01, sP=1.0, ex_rc=3.5, rc=5.0):
    return MlpCfg(sigma, mu_step, sJ, sP, ex_rc, rc)


def mlp_nparam():
    return lib().mlp_nparam()


def mlp_eval(cfg, params, r):
    p = _f64(params)
    out = np.zeros(4)
    res = []
    for x in np.atleast_1d(r):
        lib().mlp_eval(C.byref(cfg), _dp(p), float(x), _dp(out))
        res.append(out.copy())
    return np.array(res)          # columns J, dJ, phi, dphi


def mlp_grad_linear(cfg, params, r, aJ, adJ, aP, adP):
    p = _f64(params)
    r = _f64(r); aJ = _f64(aJ); adJ = _f64(adJ); aP = _f64(aP); adP = _f64(adP)
    g = np.zeros(p.size)
    lib().mlp_grad_linear(C.byref(cfg), _dp(p), r.size, _dp(r), _dp(aJ), _dp(adJ), _dp(aP),
                          _dp(adP), _dp(g))
    return g


def mlp_loss_grad(cfg, params, box, r, s, pi, pj, Eref, Fref, Wref, w=(1.0, 1.0, 1.0),
                  grad=True):
    p = _f64(params); box = _f64(box, (3,)); r = _f64(r, (-1, 3)); s = _f64(s, (-1, 3))
    pi = np.ascontiguousarray(pi, dtype=np.int32); pj = np.ascontiguousarray(pj, dtype=np.int32)
    Fref = _f64(Fref, (-1, 3)); Wref = _f64(Wref, (-1, 3)); wv = _f64(w, (3,))
    g = np.zeros(p.size) if grad else None
    loss = lib().mlp_loss_grad(C.byref(cfg), _dp(p), r.shape[0], _dp(box), _dp(r), _dp(s),
                               pi.size, _ip(pi), _ip(pj), float(Eref), _dp(Fref), _dp(Wref),
                               _dp(wv), _dp(g) if grad else None)
    return loss, g
