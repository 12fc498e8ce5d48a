"""Helpers shared by the GPU tests: the same seeded workload is handed to
the CPU oracle and to the HIP library through its C ABI."""
import numpy as np

from oracle import oracle as O


def make_oracle(w, ordering=O.COLOUR):
    return O.Oracle(w.r, w.v, w.s, w.mass, w.box, w.pot, frozen=w.frozen, skin=w.skin,
                    seed=w.seed, replica=w.replica, ordering=ordering)


def make_gpu(w, precision=0, thermo_every=0, **kw):
    from paper_1801_10233_amd import spinlat as sl
    return sl.system_from_workload(w, precision=precision, thermo_every=thermo_every, **kw)


def parity(w, o, g, rtol_r=1e-10, tol_s=1e-10, rtol_v=1e-10):
    """The agreement asked of the FP64 path: unwrapped positions within
    rtol_r * L, spins within tol_s, velocities within rtol_v * max|v|."""
    ro, vo, so = o.get_state()
    rg, vg, sg = g.get_state()
    dr = np.abs(rg - ro).max() / w.box.max()
    ds = np.abs(sg - so).max()
    vmax = max(np.abs(vo).max(), 1e-300)
    dv = np.abs(vg - vo).max() / vmax if np.abs(vo).max() > 0 else np.abs(vg - vo).max()
    return dict(dr=dr, ds=ds, dv=dv, ok=(dr <= rtol_r and ds <= tol_s and dv <= rtol_v))


def row_sets(rows, ns, segment):
    out = set()
    for i, row in enumerate(rows):
        seg = row[:ns[i]] if segment == "spin" else row
        out.update((i, int(j)) for j in seg)
    return out
