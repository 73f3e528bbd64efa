"""Helpers shared by the tests: problem set-up for the oracle from the synthetic workloads."""
import numpy as np

import oracle as O
from paper_1911_00994_amd import workloads as wl


def oracle_geom(o, l=0):
    """Boundary points / normals of every boundary row of the oracle, as per-grid (W, W, 2) arrays;
    wall Dirichlet points use the node itself."""
    N = o.level_n(l)
    W = N + 2
    gr = o.ghost_rows(l)
    cls = o.classes(l)
    B = gr["B"].reshape(3, W, W, 2).copy()
    nB = gr["nB"].reshape(3, W, W, 2).copy()
    for g in range(3):
        x, y = wl.node_coords(N, g)
        m = cls[g] == O.C_WALLD
        B[g][m, 0] = x[m]
        B[g][m, 1] = y[m]
    return dict(B=(B[0], B[1], B[2]), nB=(nB[0], nB[1], nB[2]))


def make_linear_problem(N, shape, alpha, m=None, t=0.3, motion=None, **kw):
    """Oracle with the manufactured linear problem of eq. (spaceprobaug): rhs from the exact fields."""
    o = O.Oracle(N, **kw)
    mo = None if motion is None else motion.as_array()
    phi = O.levelset_analytic(shape.kind, shape.padded(), [0] * 6 if mo is None else mo, t, N)
    st = o.set_levelset(phi, t, mo)
    assert st == O.OK, st
    o.set_alpha(alpha)
    m = m or wl.TaylorGreenMMS()
    fu, fv, g = wl.mms_linear_rhs(m, N, t, alpha)
    bu, bv, bp = wl.boundary_values_from(m, oracle_geom(o), t, t)
    W = N + 2
    o.set_x(np.zeros((W, W)), np.zeros((W, W)), np.zeros((W, W)), 0.0)
    o.set_boundary_values(bu, bv, bp)
    o.set_rhs(fu, fv, g)
    return o, phi, (fu, fv, g, bu, bv, bp)


def active_mask(cls):
    """Points carrying an equation of the system (internal, ghost, wall)."""
    return (cls == O.C_INT) | (cls == O.C_GHOST) | (cls == O.C_GHOSTX) | (cls == O.C_WALLD) | (cls == O.C_WALLG)


_NATIVE = {}


class native_oracle:
    """Context manager: the oracle library built for this host with OpenMP (oracle.build_native) in place of the
    portable single-thread build, for the parity runs at full size (same arithmetic, several threads)."""

    def __enter__(self):
        import tempfile
        if "path" not in _NATIVE:
            d = tempfile.mkdtemp(prefix="oracle_omp_")
            _NATIVE["path"] = O.build_native(d + "/liboracle_omp.so", openmp=True)
        O.lib(_NATIVE["path"])
        return O

    def __exit__(self, *exc):
        O.lib(O.build_oracle())
        return False
