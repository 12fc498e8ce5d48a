"""Thin ctypes binding of the C ABI in include/spinlat.h (libspinlat.so).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library. Importing this module does not need a GPU; calling
into the library does. There is no CPU fallback: if the shared library is
missing the first call raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspinlat.so")

SL_OK = 0
SL_E_ARG = -1
SL_E_BOX = -2
SL_E_NONFINITE = -3
SL_E_NBR_OVERFLOW = -4
SL_E_COLOR = -5
SL_E_HIP = -6
SL_E_STATE = -7
SL_E_NOMEM = -8
SL_HOST = 0
SL_DEVICE = 1
SL_FP64 = 0
SL_FP32 = 1
SL_MLP_PAIRWISE = 0
SL_MLP_SPLINE = 1
SL_BATCH_PERSISTENT = 0
SL_BATCH_PHASED = 1
SL_ORDER_COLOUR, SL_ORDER_SECTORS, SL_ORDER_SERIAL = 0, 1, 2

PROF_SPIN, PROF_FORCE, PROF_REBUILD, PROF_TABLE, PROF_PAIR = 0, 1, 2, 3, 4  # kinds of sl_get_profile
PROF_REDUCE = PROF_TABLE

# Every function the header declares (checked by the tests).
EXPORTS = [
    "sl_create", "sl_destroy", "sl_set_state", "sl_get_state", "sl_set_potential",
    "sl_set_neighbor", "sl_set_neighbor_list", "sl_get_neighbor_list",
    "sl_set_coloring", "sl_get_coloring", "sl_set_step", "sl_step",
    "sl_get_energy", "sl_get_magnetization", "sl_get_temperatures", "sl_get_thermo",
    "sl_get_stats",
    "sl_synchronize", "sl_set_tuning", "sl_get_tuning", "sl_autotune", "sl_set_profiling",
    "sl_set_mlp_mode", "sl_set_ordering", "sl_set_row_order",
    "sl_get_profile", "sl_last_error",
    "sl_mlp_create", "sl_mlp_destroy", "sl_mlp_set_weights", "sl_mlp_get_weights",
    "sl_mlp_eval", "sl_mlp_eval_static", "sl_mlp_last_error", "sl_set_mlp", "sl_get_fields",
    "sl_mlp_loss_grad", "sl_mlp_train",
    "sl_batch_create", "sl_batch_destroy", "sl_batch_set_state", "sl_batch_get_state",
    "sl_batch_get_energy", "sl_batch_get_temperatures", "sl_batch_step", "sl_batch_set_lanes", "sl_batch_set_row_order", "sl_batch_get_stats",
    "sl_batch_last_error", "sl_batch_set_mode", "sl_batch_get_mode", "sl_batch_autotune",
]

SL_MLP_NPARAM = 5378
SL_MLP_EVAL_STATIC_MAX = 32768


class sl_params(C.Structure):
    _fields_ = [("n_atoms", C.c_int64), ("box", C.c_double * 3), ("precision", C.c_int),
                ("frozen", C.c_int), ("skin", C.c_double), ("max_nbr", C.c_int),
                ("max_spin_nbr", C.c_int), ("seed", C.c_uint64), ("replica", C.c_uint32),
                ("thermo_every", C.c_int), ("stream", C.c_void_p)]


class sl_potential(C.Structure):
    _fields_ = [("morse_on", C.c_int), ("morse_D", C.c_double), ("morse_alpha", C.c_double),
                ("morse_r0", C.c_double), ("morse_rc", C.c_double), ("morse_shift", C.c_int),
                ("ex_alpha", C.c_double), ("ex_gamma", C.c_double), ("ex_delta", C.c_double),
                ("ex_rc", C.c_double), ("zeeman_g", C.c_double), ("B", C.c_double * 3),
                ("aniso_K", C.c_double), ("aniso_n", C.c_double * 3), ("lam", C.c_double),
                ("temperature", C.c_double), ("lat_gamma", C.c_double),
                ("lat_temperature", C.c_double),
                ("neel_alpha", C.c_double), ("neel_gamma", C.c_double),
                ("neel_delta", C.c_double), ("neel_rc", C.c_double),
                ("dmi_alpha", C.c_double), ("dmi_gamma", C.c_double),
                ("dmi_delta", C.c_double), ("dmi_rc", C.c_double),
                ("dmi_n", C.c_double * 3), ("eam_on", C.c_int),
                ("eam_A", C.c_double), ("eam_d", C.c_double), ("eam_beta", C.c_double),
                ("eam_c", C.c_double), ("eam_c0", C.c_double), ("eam_c1", C.c_double),
                ("eam_c2", C.c_double), ("ex_shift", C.c_int), ("aniso_split", C.c_int)]


class sl_energy(C.Structure):
    _fields_ = [("kin", C.c_double), ("pair", C.c_double), ("exchange", C.c_double),
                ("zeeman", C.c_double), ("aniso", C.c_double), ("total", C.c_double)]


class sl_stats(C.Structure):
    _fields_ = [("step", C.c_int64), ("rebuilds", C.c_int64), ("n_colours", C.c_int),
                ("jp_rounds", C.c_int), ("max_spin_nbr_seen", C.c_int),
                ("max_nbr_seen", C.c_int)]


class sl_tuning(C.Structure):
    _fields_ = [("spin_lanes", C.c_int), ("force_lanes", C.c_int), ("small_class", C.c_int),
                ("jcache", C.c_int), ("overlap", C.c_int)]


class sl_mlp_spec(C.Structure):
    _fields_ = [("sigma", C.c_double), ("mu_step", C.c_double), ("sJ", C.c_double),
                ("sP", C.c_double), ("ex_rc", C.c_double), ("rc", C.c_double),
                ("stream", C.c_void_p)]


class sl_dataset(C.Structure):
    _fields_ = [("n_snapshots", C.c_int), ("n_atoms", C.c_int64), ("box", C.c_double * 3),
                ("r", C.c_void_p), ("s", C.c_void_p), ("E", C.c_void_p), ("F", C.c_void_p),
                ("hw", C.c_void_p)]


class sl_train_opts(C.Structure):
    _fields_ = [("epochs", C.c_int), ("lr", C.c_double), ("beta1", C.c_double),
                ("beta2", C.c_double), ("eps", C.c_double), ("w_E", C.c_double),
                ("w_F", C.c_double), ("w_W", C.c_double), ("seed", C.c_uint64)]


class sl_train_log(C.Structure):
    _fields_ = [("loss_first", C.c_double), ("loss_last", C.c_double), ("updates", C.c_int64)]


class SpinLatError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"spinlat error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libspinlat.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -c 'import __graft_entry__ as g; g.build()'`")
    L = C.CDLL(LIB_PATH)
    vp, dp, ip, i64 = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int), C.c_int64
    sig = {
        "sl_create": ([C.POINTER(sl_params), C.POINTER(C.c_void_p)], C.c_int),
        "sl_destroy": ([vp], C.c_int),
        "sl_set_state": ([vp, vp, vp, vp, vp, C.c_int], C.c_int),
        "sl_get_state": ([vp, vp, vp, vp, C.c_int], C.c_int),
        "sl_set_potential": ([vp, C.POINTER(sl_potential)], C.c_int),
        "sl_set_neighbor": ([vp, C.c_double, C.c_int], C.c_int),
        "sl_set_neighbor_list": ([vp, vp, vp, C.c_int], C.c_int),
        "sl_get_neighbor_list": ([vp, ip, ip, ip, i64], i64),
        "sl_set_coloring": ([vp, vp, C.c_int], C.c_int),
        "sl_get_coloring": ([vp, ip, ip], C.c_int),
        "sl_set_step": ([vp, i64], C.c_int),
        "sl_step": ([vp, i64, C.c_double], C.c_int),
        "sl_get_energy": ([vp, C.POINTER(sl_energy)], C.c_int),
        "sl_get_magnetization": ([vp, dp], C.c_int),
        "sl_get_temperatures": ([vp, dp, dp], C.c_int),
        "sl_get_thermo": ([vp, C.c_int, C.POINTER(C.c_int64), C.POINTER(sl_energy), dp, ip],
                          C.c_int),
        "sl_get_stats": ([vp, C.POINTER(sl_stats)], C.c_int),
        "sl_synchronize": ([vp], C.c_int),
        "sl_set_tuning": ([vp, C.POINTER(sl_tuning)], C.c_int),
        "sl_get_tuning": ([vp, C.POINTER(sl_tuning)], C.c_int),
        "sl_autotune": ([vp, C.c_int, C.c_double, C.POINTER(sl_tuning)], C.c_int),
        "sl_set_mlp_mode": ([vp, C.c_int], C.c_int),
        "sl_set_ordering": ([vp, C.c_int, ip], C.c_int),
        "sl_set_row_order": ([vp, C.c_double], C.c_int),
        "sl_set_profiling": ([vp, C.c_int], C.c_int),
        "sl_get_profile": ([vp, C.c_int, C.POINTER(C.c_int64), dp, dp], C.c_int),
        "sl_last_error": ([vp], C.c_char_p),
        "sl_mlp_create": ([C.POINTER(sl_mlp_spec), C.POINTER(C.c_void_p)], C.c_int),
        "sl_mlp_destroy": ([vp], C.c_int),
        "sl_mlp_set_weights": ([vp, vp, C.c_int, C.c_int], C.c_int),
        "sl_mlp_get_weights": ([vp, vp, C.c_int, C.c_int], C.c_int),
        "sl_mlp_eval": ([vp, vp, C.c_int64, vp, C.c_int], C.c_int),
        "sl_mlp_eval_static": ([vp, vp, C.c_int64, vp, C.c_int], C.c_int),
        "sl_mlp_last_error": ([vp], C.c_char_p),
        "sl_set_mlp": ([vp, vp], C.c_int),
        "sl_get_fields": ([vp, vp, vp, C.c_int], C.c_int),
        "sl_mlp_loss_grad": ([vp, C.POINTER(sl_dataset), C.c_int, dp, dp, vp], C.c_int),
        "sl_mlp_train": ([vp, C.POINTER(sl_dataset), C.POINTER(sl_train_opts),
                          C.POINTER(sl_train_log)], C.c_int),
        "sl_batch_create": ([C.c_int, C.POINTER(sl_params), C.POINTER(sl_potential),
                             C.POINTER(C.c_void_p)], C.c_int),
        "sl_batch_destroy": ([vp], C.c_int),
        "sl_batch_set_state": ([vp, C.c_int, vp, vp, vp, vp, C.c_int], C.c_int),
        "sl_batch_get_state": ([vp, C.c_int, vp, vp, vp, C.c_int], C.c_int),
        "sl_batch_get_energy": ([vp, C.c_int, C.POINTER(sl_energy)], C.c_int),
        "sl_batch_get_temperatures": ([vp, C.c_int, dp, dp], C.c_int),
        "sl_batch_step": ([vp, i64, C.c_double], C.c_int),
        "sl_batch_set_lanes": ([vp, C.c_int], C.c_int),
        "sl_batch_set_row_order": ([vp, C.c_double], C.c_int),
        "sl_batch_get_stats": ([vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), ip], C.c_int),
        "sl_batch_last_error": ([vp], C.c_char_p),
        "sl_batch_set_mode": ([vp, C.c_int], C.c_int),
        "sl_batch_get_mode": ([vp, ip], C.c_int),
        "sl_batch_autotune": ([vp, C.c_int, C.c_double, ip, ip], C.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _ptr(a):
    """Host numpy array or device tensor -> (address, where)."""
    if a is None:
        return None, SL_HOST
    if isinstance(a, np.ndarray):
        return a.ctypes.data, SL_HOST
    # torch tensor (device or host)
    dev = getattr(a, "is_cuda", False)
    return a.data_ptr(), (SL_DEVICE if dev else SL_HOST)


def make_potential(d: dict) -> sl_potential:
    p = sl_potential()
    for k, v in d.items():
        if k in ("B", "aniso_n", "dmi_n"):
            setattr(p, k, (C.c_double * 3)(*v))
        else:
            setattr(p, k, v)
    return p


class System:
    """One system behind an sl_system handle."""

    def __init__(self, n_atoms, box, precision=SL_FP64, frozen=False, skin=0.3,
                 max_nbr=0, max_spin_nbr=0, seed=0, replica=0, thermo_every=0,
                 stream=None):
        L = lib()
        p = sl_params()
        p.n_atoms = int(n_atoms)
        p.box = (C.c_double * 3)(*[float(x) for x in box])
        p.precision = int(precision)
        p.frozen = int(bool(frozen))
        p.skin = float(skin)
        p.max_nbr = int(max_nbr)
        p.max_spin_nbr = int(max_spin_nbr)
        p.seed = int(seed)
        p.replica = int(replica)
        p.thermo_every = int(thermo_every)
        p.stream = stream
        h = C.c_void_p()
        rc = L.sl_create(C.byref(p), C.byref(h))
        if rc != SL_OK:
            raise SpinLatError(rc, L.sl_last_error(None).decode())
        self.h = h
        self.N = int(n_atoms)
        self.precision = precision

    def close(self):
        if getattr(self, "h", None):
            try:
                lib().sl_destroy(self.h)
            except Exception:
                pass
            self.h = None

    __del__ = close

    def _check(self, rc):
        if rc < 0:
            raise SpinLatError(rc, lib().sl_last_error(self.h).decode())
        return rc

    def set_potential(self, pot: dict):
        self._pot = make_potential(pot)
        self._check(lib().sl_set_potential(self.h, C.byref(self._pot)))

    def set_state(self, r=None, v=None, s=None, mass=None):
        conv = []
        where = SL_HOST
        for a, shape in ((r, (self.N, 3)), (v, (self.N, 3)), (s, (self.N, 3)), (mass, (self.N,))):
            if a is None:
                conv.append(None)
            elif isinstance(a, np.ndarray) or not hasattr(a, "data_ptr"):
                conv.append(np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(shape)))
            else:
                conv.append(a.contiguous())
        ptrs = []
        for a in conv:
            p, w = _ptr(a)
            ptrs.append(p)
            if a is not None:
                where = w
        self._check(lib().sl_set_state(self.h, *ptrs, where))

    def get_state(self):
        r = np.empty((self.N, 3)); v = np.empty((self.N, 3)); s = np.empty((self.N, 3))
        self._check(lib().sl_get_state(self.h, r.ctypes.data, v.ctypes.data, s.ctypes.data,
                                       SL_HOST))
        return r, v, s

    def get_state_device(self, r, v, s):
        """Copy into device tensors (float64, N x 3)."""
        self._check(lib().sl_get_state(self.h, r.data_ptr(), v.data_ptr(), s.data_ptr(),
                                       SL_DEVICE))

    def set_neighbor(self, skin, max_nbr=0):
        self._check(lib().sl_set_neighbor(self.h, float(skin), int(max_nbr)))

    def set_neighbor_list(self, offsets, idx):
        o = np.ascontiguousarray(offsets, dtype=np.int32)
        i = np.ascontiguousarray(idx, dtype=np.int32)
        self._check(lib().sl_set_neighbor_list(self.h, o.ctypes.data, i.ctypes.data, SL_HOST))

    def neighbor_list(self):
        ns = np.zeros(self.N, dtype=np.int32)
        na = np.zeros(self.N, dtype=np.int32)
        ip = C.POINTER(C.c_int)
        tot = self._check(lib().sl_get_neighbor_list(self.h, ns.ctypes.data_as(ip),
                                                     na.ctypes.data_as(ip), None, 0))
        idx = np.zeros(max(tot, 1), dtype=np.int32)
        self._check(lib().sl_get_neighbor_list(self.h, ns.ctypes.data_as(ip),
                                               na.ctypes.data_as(ip), idx.ctypes.data_as(ip),
                                               tot))
        off = np.concatenate([[0], np.cumsum(na)])
        return ns, na, [idx[off[i]:off[i + 1]] for i in range(self.N)]

    def set_coloring(self, colour):
        c = np.ascontiguousarray(colour, dtype=np.int32)
        self._check(lib().sl_set_coloring(self.h, c.ctypes.data, SL_HOST))

    def coloring(self):
        c = np.zeros(self.N, dtype=np.int32)
        K = C.c_int()
        self._check(lib().sl_get_coloring(self.h, c.ctypes.data_as(C.POINTER(C.c_int)),
                                          C.byref(K)))
        return c, K.value

    def set_step(self, k):
        self._check(lib().sl_set_step(self.h, int(k)))

    def step(self, n, dt):
        self._check(lib().sl_step(self.h, int(n), float(dt)))

    def energy(self):
        e = sl_energy()
        self._check(lib().sl_get_energy(self.h, C.byref(e)))
        return dict(kin=e.kin, pair=e.pair, exchange=e.exchange, zeeman=e.zeeman,
                    aniso=e.aniso, total=e.total)

    def magnetization(self):
        M = (C.c_double * 3)()
        self._check(lib().sl_get_magnetization(self.h, M))
        return np.array(list(M))

    def temperatures(self):
        """(T_L, T_S) of the current state in K."""
        tl, ts = C.c_double(), C.c_double()
        self._check(lib().sl_get_temperatures(self.h, C.byref(tl), C.byref(ts)))
        return tl.value, ts.value

    def thermo(self, max_samples=1 << 16):
        steps = (C.c_int64 * max_samples)()
        es = (sl_energy * max_samples)()
        M = np.zeros((max_samples, 3))
        cnt = C.c_int()
        self._check(lib().sl_get_thermo(self.h, max_samples, steps, es,
                                        M.ctypes.data_as(C.POINTER(C.c_double)), C.byref(cnt)))
        k = cnt.value
        return (np.array(steps[:k], dtype=np.int64),
                np.array([e.total for e in es[:k]]), M[:k])

    def stats(self):
        s = sl_stats()
        self._check(lib().sl_get_stats(self.h, C.byref(s)))
        return dict(step=s.step, rebuilds=s.rebuilds, n_colours=s.n_colours,
                    jp_rounds=s.jp_rounds, max_spin_nbr_seen=s.max_spin_nbr_seen,
                    max_nbr_seen=s.max_nbr_seen)

    def synchronize(self):
        self._check(lib().sl_synchronize(self.h))

    def set_tuning(self, spin_lanes=0, force_lanes=0, small_class=0, jcache=0, overlap=0):
        t = sl_tuning(int(spin_lanes), int(force_lanes), int(small_class), int(jcache),
                      int(overlap))
        self._check(lib().sl_set_tuning(self.h, C.byref(t)))

    def tuning(self):
        t = sl_tuning()
        self._check(lib().sl_get_tuning(self.h, C.byref(t)))
        return dict(spin_lanes=t.spin_lanes, force_lanes=t.force_lanes,
                    small_class=t.small_class, jcache=t.jcache, overlap=t.overlap)

    def autotune(self, steps, dt):
        """Time launch shapes on a scratch copy and keep the fastest."""
        t = sl_tuning()
        self._check(lib().sl_autotune(self.h, int(steps), float(dt), C.byref(t)))
        return dict(spin_lanes=t.spin_lanes, force_lanes=t.force_lanes,
                    small_class=t.small_class, jcache=t.jcache, overlap=t.overlap)

    def set_ordering(self, ordering, grid=(1, 1, 1)):
        """SL_ORDER_COLOUR, SL_ORDER_SECTORS (with the subdomain grid) or
        SL_ORDER_SERIAL."""
        g = (C.c_int * 3)(*[int(x) for x in grid])
        self._check(lib().sl_set_ordering(self.h, int(ordering), g))

    def set_row_order(self, quantum):
        """Sort each list-row segment by the neighbour displacement rounded
        to a grid of `quantum` A (0: cell-loop order); from the next build."""
        self._check(lib().sl_set_row_order(self.h, float(quantum)))

    def set_mlp_mode(self, mode):
        self._check(lib().sl_set_mlp_mode(self.h, int(mode)))

    def set_mlp(self, mlp):
        self._mlp = mlp
        self._check(lib().sl_set_mlp(self.h, mlp.h if mlp is not None else None))

    def fields(self):
        """(F[N,3], exchange hbar*omega[N,3]) of the current state."""
        F = np.zeros((self.N, 3)); hw = np.zeros((self.N, 3))
        self._check(lib().sl_get_fields(self.h, F.ctypes.data, hw.ctypes.data, SL_HOST))
        return F, hw

    def set_profiling(self, on=True, every=1):
        """Time kernel launches with HIP events (those of every `every`-th step)."""
        self._check(lib().sl_set_profiling(self.h, int(every) if on else 0))

    def profile(self, kind):
        n = C.c_int64(); ms = C.c_double(); w = C.c_double()
        self._check(lib().sl_get_profile(self.h, int(kind), C.byref(n), C.byref(ms),
                                         C.byref(w)))
        return n.value, ms.value, w.value


class Mlp:
    """Per-pair learned potential behind an sl_mlp handle."""

    def __init__(self, sigma=0.0, mu_step=0.0, sJ=0.0, sP=0.0, ex_rc=0.0, rc=0.0, stream=None):
        spec = sl_mlp_spec(sigma, mu_step, sJ, sP, ex_rc, rc, stream)
        h = C.c_void_p()
        rc_ = lib().sl_mlp_create(C.byref(spec), C.byref(h))
        if rc_ != SL_OK:
            raise SpinLatError(rc_, lib().sl_mlp_last_error(None).decode())
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            try:
                lib().sl_mlp_destroy(self.h)
            except Exception:
                pass
            self.h = None

    __del__ = close

    def _check(self, rc):
        if rc < 0:
            raise SpinLatError(rc, lib().sl_mlp_last_error(self.h).decode())
        return rc

    def set_weights(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        self._check(lib().sl_mlp_set_weights(self.h, p.ctypes.data, p.size, SL_HOST))

    def weights(self):
        p = np.zeros(SL_MLP_NPARAM, dtype=np.float32)
        self._check(lib().sl_mlp_get_weights(self.h, p.ctypes.data, p.size, SL_HOST))
        return p

    def eval(self, r):
        r = np.ascontiguousarray(r, dtype=np.float64).ravel()
        out = np.zeros((r.size, 4))
        self._check(lib().sl_mlp_eval(self.h, r.ctypes.data, r.size, out.ctypes.data, SL_HOST))
        return out

    def eval_static(self, r, out=None):
        """sl_mlp_eval_static: host arrays (returns a new [P][4] array), or
        device tensors r (float64, P) and out (float64, P x 4) on the
        handle's stream (asynchronous)."""
        if hasattr(r, "data_ptr"):
            self._check(lib().sl_mlp_eval_static(self.h, r.data_ptr(), r.numel(), out.data_ptr(),
                                                 SL_DEVICE))
            return out
        r = np.ascontiguousarray(r, dtype=np.float64).ravel()
        out = np.zeros((r.size, 4))
        self._check(lib().sl_mlp_eval_static(self.h, r.ctypes.data, r.size, out.ctypes.data,
                                             SL_HOST))
        return out


class Dataset:
    """Snapshots (host arrays kept alive) for sl_mlp_loss_grad / sl_mlp_train."""

    def __init__(self, box, r, s, E, F, hw):
        self.r = np.ascontiguousarray(r, dtype=np.float64)
        self.s = np.ascontiguousarray(s, dtype=np.float64)
        self.E = np.ascontiguousarray(E, dtype=np.float64)
        self.F = np.ascontiguousarray(F, dtype=np.float64)
        self.hw = np.ascontiguousarray(hw, dtype=np.float64)
        S, N = self.r.shape[0], self.r.shape[1]
        self.c = sl_dataset(S, N, (C.c_double * 3)(*box), self.r.ctypes.data, self.s.ctypes.data,
                            self.E.ctypes.data, self.F.ctypes.data, self.hw.ctypes.data)


def mlp_loss_grad(mlp, ds, snapshot, w=(1.0, 1.0, 1.0)):
    wv = (C.c_double * 3)(*w)
    loss = C.c_double()
    g = np.zeros(SL_MLP_NPARAM, dtype=np.float32)
    mlp._check(lib().sl_mlp_loss_grad(mlp.h, C.byref(ds.c), int(snapshot), wv, C.byref(loss),
                                      g.ctypes.data))
    return loss.value, g


def mlp_train(mlp, ds, epochs, lr=1e-3, w=(1.0, 1.0, 1.0), seed=0):
    o = sl_train_opts(int(epochs), float(lr), 0.0, 0.0, 0.0, float(w[0]), float(w[1]),
                      float(w[2]), int(seed))
    log = sl_train_log()
    mlp._check(lib().sl_mlp_train(mlp.h, C.byref(ds.c), C.byref(o), C.byref(log)))
    return dict(loss_first=log.loss_first, loss_last=log.loss_last, updates=log.updates)


class Batch:
    """Batched replicas behind an sl_batch handle (one workload per replica)."""

    def __init__(self, workloads, precision=SL_FP32, max_nbr=0):
        R = len(workloads)
        P = (sl_params * R)()
        Q = (sl_potential * R)()
        for k, w in enumerate(workloads):
            p = P[k]
            p.n_atoms = w.N
            p.box = (C.c_double * 3)(*[float(x) for x in w.box])
            p.precision = int(precision)
            p.frozen = 0
            p.skin = float(w.skin)
            p.max_nbr = int(max_nbr)
            p.seed = int(w.seed)
            p.replica = int(w.replica)
            Q[k] = make_potential(w.pot)
        h = C.c_void_p()
        rc = lib().sl_batch_create(R, P, Q, C.byref(h))
        if rc != SL_OK:
            raise SpinLatError(rc, lib().sl_batch_last_error(None).decode())
        self.h = h
        self.R = R
        self.N = [w.N for w in workloads]
        for k, w in enumerate(workloads):
            self.set_state(k, w.r, w.v, w.s, w.mass)
        q = {float(getattr(w, "row_quantum", 0.0)) for w in workloads}
        if len(q) == 1 and q.pop() > 0.0:
            self.set_row_order(getattr(workloads[0], "row_quantum"))

    def close(self):
        if getattr(self, "h", None):
            try:
                lib().sl_batch_destroy(self.h)
            except Exception:
                pass
            self.h = None

    __del__ = close

    def _check(self, rc):
        if rc < 0:
            raise SpinLatError(rc, lib().sl_batch_last_error(self.h).decode())
        return rc

    def set_state(self, r, x, v, s, mass):
        arrs = [np.ascontiguousarray(np.asarray(a, dtype=np.float64)) for a in (x, v, s, mass)]
        self._check(lib().sl_batch_set_state(self.h, int(r), *[a.ctypes.data for a in arrs],
                                             SL_HOST))

    def get_state(self, r):
        n = self.N[r]
        x = np.empty((n, 3)); v = np.empty((n, 3)); s = np.empty((n, 3))
        self._check(lib().sl_batch_get_state(self.h, int(r), x.ctypes.data, v.ctypes.data,
                                             s.ctypes.data, SL_HOST))
        return x, v, s

    def energy(self, r):
        e = sl_energy()
        self._check(lib().sl_batch_get_energy(self.h, int(r), C.byref(e)))
        return dict(kin=e.kin, pair=e.pair, exchange=e.exchange, zeeman=e.zeeman,
                    aniso=e.aniso, total=e.total)

    def temperatures(self, r):
        """(T_L, T_S) of replica r in K."""
        tl, ts = C.c_double(), C.c_double()
        self._check(lib().sl_batch_get_temperatures(self.h, int(r), C.byref(tl), C.byref(ts)))
        return tl.value, ts.value

    def step(self, n, dt):
        self._check(lib().sl_batch_step(self.h, int(n), float(dt)))

    def set_lanes(self, lanes):
        self._check(lib().sl_batch_set_lanes(self.h, int(lanes)))

    def set_row_order(self, quantum):
        """List-row order grid (A) of every replica; 0 keeps the cell-loop order."""
        self._check(lib().sl_batch_set_row_order(self.h, float(quantum)))

    def set_mode(self, mode):
        self._check(lib().sl_batch_set_mode(self.h, int(mode)))

    def mode(self):
        m = C.c_int()
        self._check(lib().sl_batch_get_mode(self.h, C.byref(m)))
        return m.value

    def autotune(self, steps, dt):
        """Time (mode, lanes) pairs on a scratch copy and keep the fastest."""
        m = C.c_int(); ln = C.c_int()
        self._check(lib().sl_batch_autotune(self.h, int(steps), float(dt), C.byref(m), C.byref(ln)))
        return dict(mode=m.value, lanes=ln.value)

    def stats(self):
        a = C.c_int64(); b = C.c_int64(); c = C.c_int()
        self._check(lib().sl_batch_get_stats(self.h, C.byref(a), C.byref(b), C.byref(c)))
        return dict(launches=a.value, rebuilds=b.value, lanes=c.value)


def system_from_workload(w, precision=SL_FP64, thermo_every=0, **kw):
    """Convenience: create a system, set the potential and the state of a
    workloads.Workload."""
    S = System(w.N, w.box, precision=precision, frozen=w.frozen, skin=w.skin, seed=w.seed,
               replica=w.replica, thermo_every=thermo_every, **kw)
    S.set_potential(w.pot)
    S.set_state(w.r, w.v, w.s, w.mass)
    if getattr(w, "row_quantum", 0.0) > 0.0:
        S.set_row_order(w.row_quantum)
    return S
