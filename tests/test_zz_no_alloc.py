"""sl_mlp_eval_static (no device allocation; staging in a static device
array per GPU) against sl_mlp_eval, which stages through hipMalloc: same
kernels, so the outputs agree bit for bit. Two calls in a row, the second
smaller, through host and device pointers."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _mlp(stream=None):
    from paper_1801_10233_amd import spinlat as sl
    m = sl.Mlp(stream=stream)
    p = np.random.default_rng(41).standard_normal(sl.SL_MLP_NPARAM) * 0.2
    m.set_weights(p.astype(np.float32))
    return m


def test_static_eval_equals_allocating_eval_host():
    from paper_1801_10233_amd import spinlat as sl
    m = _mlp()
    rng = np.random.default_rng(5)
    for P in (sl.SL_MLP_EVAL_STATIC_MAX, 20011, 777):     # full size, then smaller calls
        r = rng.uniform(0.3, 5.5, P)
        r[:4] = (3.5, 5.0, 2.4825, 2.8665)
        want = m.eval(r)
        got = m.eval_static(r)
        print("P", P, "max |diff|", np.abs(got - want).max(), flush=True)
        assert np.array_equal(got, want)


class _Hip:
    """Device buffers for the test through the HIP runtime the library itself
    links (the test allocates; the entry point under test does not)."""

    def __init__(self):
        import ctypes as C
        self.C = C
        self.lib = C.CDLL("libamdhip64.so.7")
        for name in ("hipMalloc", "hipFree", "hipMemcpy", "hipDeviceSynchronize"):
            getattr(self.lib, name).restype = C.c_int
        self.lib.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
        self.lib.hipFree.argtypes = [C.c_void_p]
        self.lib.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]

    def malloc(self, nbytes):
        p = self.C.c_void_p()
        assert self.lib.hipMalloc(self.C.byref(p), nbytes) == 0
        return p.value

    def h2d(self, dst, a):
        assert self.lib.hipMemcpy(dst, a.ctypes.data, a.nbytes, 1) == 0

    def d2h(self, a, src):
        assert self.lib.hipMemcpy(a.ctypes.data, src, a.nbytes, 2) == 0


class _Dev:
    """A device pointer with the binding's tensor-like interface."""

    def __init__(self, ptr, n):
        self.ptr, self.n = ptr, n

    def data_ptr(self):
        return self.ptr

    def numel(self):
        return self.n


def test_static_eval_equals_allocating_eval_device():
    hip = _Hip()
    m = _mlp()
    rng = np.random.default_rng(9)
    for P in (30000, 1000):
        r = rng.uniform(1.0, 5.2, P)
        want = m.eval(r)
        dr, do = hip.malloc(8 * P), hip.malloc(32 * P)
        try:
            hip.h2d(dr, r)
            hip.h2d(do, np.full((P, 4), np.nan))
            m.eval_static(_Dev(dr, P), _Dev(do, 4 * P))   # enqueued on the handle's stream
            assert hip.lib.hipDeviceSynchronize() == 0
            got = np.empty((P, 4))
            hip.d2h(got, do)
        finally:
            hip.lib.hipFree(dr)
            hip.lib.hipFree(do)
        assert np.array_equal(got, want)


def test_static_eval_rejects_sizes_beyond_its_array():
    from paper_1801_10233_amd import spinlat as sl
    m = _mlp()
    with pytest.raises(sl.SpinLatError) as e:
        m.eval_static(np.full(sl.SL_MLP_EVAL_STATIC_MAX + 1, 3.0))
    assert e.value.code == sl.SL_E_ARG
    assert m.eval_static(np.zeros(0)).shape == (0, 4)
    # still usable after the rejected call
    r = np.linspace(2.0, 5.0, 64)
    assert np.array_equal(m.eval_static(r), m.eval(r))
