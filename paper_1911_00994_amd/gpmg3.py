"""ctypes binding of the 3-D entry points (include/gpmg3.h) in libgpmg.so: argument marshalling only; every step runs
in the library's kernels, and the binding raises if the library is missing (no CPU fallback)."""
from __future__ import annotations

import ctypes

import numpy as np

from . import gpmg

EXPORTS = ["gp3_default_params", "gp3_setup_grid", "gp3_destroy", "gp3_num_levels", "gp3_last_hip_error",
           "gp3_set_levelset", "gp3_set_levelset_analytic", "gp3_set_alpha", "gp3_set_rhs", "gp3_set_boundary_values",
           "gp3_set_x", "gp3_get_x", "gp3_get_classes", "gp3_get_ghost_rows", "gp3_relax", "gp3_cycle", "gp3_solve",
           "gp3_residual"]


class Gp3Params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int) for n in ("nu1", "nu2", "gamma", "lambda_ghost", "coarsest_n", "march_max", "krylov")] + \
               [(n, ctypes.c_double) for n in ("dtau_dir", "dtau_neu_over_h", "bisect_eps_over_h", "cg_min")]


_lib3 = None


def lib():
    global _lib3
    if _lib3 is not None:
        return _lib3
    L = gpmg.lib()
    vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    sigs = {
        "gp3_default_params": (None, [ctypes.POINTER(Gp3Params)]),
        "gp3_setup_grid": (i, [ctypes.POINTER(vp), i, ctypes.POINTER(Gp3Params), vp]),
        "gp3_destroy": (None, [vp]),
        "gp3_num_levels": (i, [vp]),
        "gp3_last_hip_error": (ctypes.c_char_p, [vp]),
        "gp3_set_levelset": (i, [vp, vp, i]),
        "gp3_set_levelset_analytic": (i, [vp, i, vp]),
        "gp3_set_alpha": (i, [vp, d]),
        "gp3_set_rhs": (i, [vp, vp, vp, vp, vp, i]),
        "gp3_set_boundary_values": (i, [vp, vp, vp, vp, vp, i]),
        "gp3_set_x": (i, [vp, vp, i]),
        "gp3_get_x": (i, [vp, vp, i]),
        "gp3_get_classes": (i, [vp, i, vp]),
        "gp3_get_ghost_rows": (i, [vp, i, vp, vp, vp, vp, vp]),
        "gp3_relax": (i, [vp, i]),
        "gp3_cycle": (i, [vp, vp]),
        "gp3_solve": (i, [vp, d, i, ctypes.POINTER(gpmg.GpStats)]),
        "gp3_residual": (i, [vp, vp, vp]),
    }
    for name, (res, args) in sigs.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib3 = L
    return L


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


class Solver3:
    """One gpmg3 context on the current HIP device."""

    def __init__(self, N, stream=None, **params):
        self.N, self.W = N, N + 2
        p = Gp3Params()
        lib().gp3_default_params(ctypes.byref(p))
        for k, v in params.items():
            setattr(p, k, v)
        self._p = p
        h = ctypes.c_void_p()
        st = lib().gp3_setup_grid(ctypes.byref(h), N, ctypes.byref(p), ctypes.c_void_p(stream or 0))
        if st != gpmg.GP_OK:
            raise gpmg.GpmgError(st, "gp3_setup_grid", lib().gp_strerror(st).decode())
        self._h = h

    def _check(self, st, where):
        if st != gpmg.GP_OK:
            detail = lib().gp_strerror(st).decode()
            if st == gpmg.GP_EHIP:
                detail += " (" + lib().gp3_last_hip_error(self._h).decode() + ")"
            raise gpmg.GpmgError(st, where, detail)
        return st

    def close(self):
        if getattr(self, "_h", None):
            lib().gp3_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except TypeError:
            pass

    @property
    def n(self):
        return 4 * self.W ** 3 + 1

    def num_levels(self):
        return lib().gp3_num_levels(self._h)

    def set_levelset_analytic(self, kind, params, check=True):
        p = _f(np.asarray(list(params) + [0.0] * (6 - len(params))))
        st = lib().gp3_set_levelset_analytic(self._h, kind, _p(p))
        return self._check(st, "gp3_set_levelset_analytic") if check else st

    def set_levelset(self, phi, check=True):
        st = lib().gp3_set_levelset(self._h, _p(_f(phi)), 0)
        return self._check(st, "gp3_set_levelset") if check else st

    def set_alpha(self, a):
        self._check(lib().gp3_set_alpha(self._h, a), "gp3_set_alpha")

    def set_rhs(self, fu=None, fv=None, fw=None, g=None):
        self._check(lib().gp3_set_rhs(self._h, *[_p(_f(a)) for a in (fu, fv, fw, g)], 0), "gp3_set_rhs")

    def set_boundary_values(self, bu=None, bv=None, bw=None, bp=None):
        self._check(lib().gp3_set_boundary_values(self._h, *[_p(_f(a)) for a in (bu, bv, bw, bp)], 0),
                    "gp3_set_boundary_values")

    def set_x(self, x):
        self._check(lib().gp3_set_x(self._h, _p(_f(x)), 0), "gp3_set_x")

    def get_x(self):
        x = np.zeros(self.n)
        self._check(lib().gp3_get_x(self._h, _p(x), 0), "gp3_get_x")
        return x

    def classes(self, level=0):
        W = (self.N >> level) + 2
        c = np.zeros(4 * W ** 3, np.uint8)
        self._check(lib().gp3_get_classes(self._h, level, _p(c)), "gp3_get_classes")
        return c.reshape(4, W, W, W)

    def ghost_rows(self, level=0):
        W = (self.N >> level) + 2
        P = 4 * W ** 3
        B, th, w, dt = np.zeros(3 * P), np.zeros(3 * P), np.zeros(27 * P), np.zeros(P)
        c = np.zeros(27 * P, np.int32)
        self._check(lib().gp3_get_ghost_rows(self._h, level, _p(B), _p(th), _p(w), _p(c), _p(dt)), "gp3_get_ghost_rows")
        return dict(B=B.reshape(P, 3), theta=th.reshape(P, 3), w=w.reshape(P, 27), col=c.reshape(P, 27), dtau=dt)

    def relax(self, steps=1):
        self._check(lib().gp3_relax(self._h, steps), "gp3_relax")

    def cycle(self):
        r = ctypes.c_double()
        self._check(lib().gp3_cycle(self._h, ctypes.byref(r)), "gp3_cycle")
        return r.value

    def solve(self, tol=1e-10, max_cycles=100, check=True):
        s = gpmg.GpStats()
        st = lib().gp3_solve(self._h, tol, max_cycles, ctypes.byref(s))
        if check:
            self._check(st, "gp3_solve")
        return st, s.as_dict()

    def residual(self):
        r = np.zeros(self.n)
        ri = ctypes.c_double()
        self._check(lib().gp3_residual(self._h, _p(r), ctypes.byref(ri)), "gp3_residual")
        return r, ri.value
