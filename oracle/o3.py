"""Python handle on the 3-D oracle (gpmg3_oracle.c): the space problem of one Crank-Nicolson step in three
dimensions around a body given by a level set (the paper's 3-D outlook, Sect. 3 opening paragraph and Sect. 6).

TEST INFRASTRUCTURE ONLY (the same rule as the 2-D oracle: only the tests may load it).

Reading new in 3-D: the fictitious-time step of the pressure normal-derivative rows is 0.6 h instead of the 2-D
0.9 h: the diagonal of such a row reaches 1.5 (|n_x| + |n_y| + |n_z|)/h <= 2.6/h for a normal along a diagonal,
and 0.9 h would put the step beyond the stability bound dtau c_G < 2 of eq. (ghostrelax).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gpmg3_oracle.c")
_LIB = os.path.join(_HERE, "liboracle3.so")

C_INACTIVE, C_INT, C_GHOST, C_WALLD, C_WALLG, C_GHOSTX = 0, 1, 2, 3, 4, 7
OK, E_INVAL, E_GEOM, E_NOCONV, E_DIVERGED = 0, -1, -4, -5, -6
SPHERE, ELLIPSOID = 0, 1


def build_oracle3(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build_oracle3())
        vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        L.o3_create.restype = vp
        L.o3_create.argtypes = [i, vp, vp]
        L.o3_destroy.argtypes = [vp]
        for name, args in [("o3_set_levelset", [vp, vp]), ("o3_set_alpha", [vp, d]), ("o3_solve", [vp, d, i, vp]),
                           ("o3_levelset_analytic", [i, vp, i, vp]), ("o3_get_classes", [vp, i, vp]),
                           ("o3_csr_size", [vp, vp, vp]), ("o3_csr", [vp, vp, vp, vp, vp]),
                           ("o3_res_history", [vp, vp, i]), ("o3_num_levels", [vp]), ("o3_level_n", [vp, i]),
                           ("o3_relax", [vp, i, i]), ("o3_residual", [vp, vp, vp]),
                           ("o3_get_ghost_rows", [vp, i, vp, vp, vp, vp, vp])]:
            f = getattr(L, name)
            f.restype = i
            f.argtypes = args
        for name, args in [("o3_set_boundary_values", [vp, vp, vp, vp, vp]), ("o3_set_rhs", [vp, vp, vp, vp, vp]),
                           ("o3_set_x", [vp, vp]), ("o3_get_x", [vp, vp]), ("o3_get_b", [vp, vp]),
                           ("o3_st27_dirichlet", [vp, vp]), ("o3_st27_neumann", [vp, vp, vp, d, vp])]:
            f = getattr(L, name)
            f.restype = None
            f.argtypes = args
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def st27_dirichlet(th):
    w = np.zeros(27)
    lib().o3_st27_dirichlet(_p(_f(th)), _p(w))
    return w.reshape(3, 3, 3)  # [c, b, a]: point G - (a s_x, b s_y, c s_z) h


def st27_neumann(th, s, n, h):
    w = np.zeros(27)
    lib().o3_st27_neumann(_p(_f(th)), _p(_f(s)), _p(_f(n)), h, _p(w))
    return w.reshape(3, 3, 3)


def levelset_analytic(kind, params, N):
    """phi on the (2N+1)^3 half-step lattice [kz, ky, kx]; params = (R or A_x, A_y, A_z, c_x, c_y, c_z)"""
    phi = np.zeros((2 * N + 1,) * 3)
    p = _f(np.asarray(list(params) + [0.0] * (6 - len(params))))
    assert lib().o3_levelset_analytic(kind, _p(p), N, _p(phi)) == OK
    return phi


def node_coords(N, g):
    """x, y, z arrays [k+1, j+1, i+1] of grid g (0 u, 1 v, 2 w, 3 p)"""
    h = 2.0 / N
    idx = np.arange(-1, N + 1, dtype=np.float64)
    K, J, I = np.meshgrid(idx, idx, idx, indexing="ij")
    o = [(0, .5, .5), (.5, 0, .5), (.5, .5, 0), (.5, .5, .5)][g]
    return -1 + (I + o[0]) * h, -1 + (J + o[1]) * h, -1 + (K + o[2]) * h


class Oracle3:
    def __init__(self, N, nu1=2, nu2=2, gamma=1, lam=2, coarsest_n=4, march_max=8, krylov=8, dtau_dir=0.9,
                 dtau_neu_over_h=0.6, eps_over_h=0.01, cg_min=0.1):
        self.N, self.W = N, N + 2
        ip = np.array([nu1, nu2, gamma, lam, coarsest_n, march_max, krylov], dtype=np.int32)
        dp = np.array([dtau_dir, dtau_neu_over_h, eps_over_h, cg_min])
        self._h = lib().o3_create(N, _p(ip), _p(dp))
        if not self._h:
            raise ValueError("oracle3: invalid parameters")

    def __del__(self):
        if getattr(self, "_h", None):
            lib().o3_destroy(self._h)
            self._h = None

    @property
    def n(self):
        return 4 * self.W ** 3 + 1

    def set_levelset(self, phi):
        return lib().o3_set_levelset(self._h, _p(_f(phi)))

    def set_alpha(self, a):
        return lib().o3_set_alpha(self._h, a)

    def classes(self, l=0):
        W = lib().o3_level_n(self._h, l) + 2
        c = np.zeros(4 * W ** 3, np.uint8)
        assert lib().o3_get_classes(self._h, l, _p(c)) == OK
        return c.reshape(4, W, W, W)

    def ghost_rows(self, l=0):
        W = lib().o3_level_n(self._h, l) + 2
        P = 4 * W ** 3
        B, th, w, dt = np.zeros(3 * P), np.zeros(3 * P), np.zeros(27 * P), np.zeros(P)
        c = np.zeros(27 * P, np.int32)
        assert lib().o3_get_ghost_rows(self._h, l, _p(B), _p(th), _p(w), _p(c), _p(dt)) == OK
        return dict(B=B.reshape(P, 3), theta=th.reshape(P, 3), w=w.reshape(P, 27), col=c.reshape(P, 27), dtau=dt)

    def set_rhs(self, fu=None, fv=None, fw=None, g=None):
        lib().o3_set_rhs(self._h, *[_p(_f(a)) for a in (fu, fv, fw, g)])

    def set_boundary_values(self, bu=None, bv=None, bw=None, bp=None):
        lib().o3_set_boundary_values(self._h, *[_p(_f(a)) for a in (bu, bv, bw, bp)])

    def set_x(self, x):
        lib().o3_set_x(self._h, _p(_f(x)))

    def get_x(self):
        x = np.zeros(self.n)
        lib().o3_get_x(self._h, _p(x))
        return x

    def get_b(self):
        b = np.zeros(self.n)
        lib().o3_get_b(self._h, _p(b))
        return b

    def relax(self, l=0, steps=1):
        return lib().o3_relax(self._h, l, steps)

    def residual(self):
        r = np.zeros(self.n)
        ri = ctypes.c_double()
        assert lib().o3_residual(self._h, _p(r), ctypes.byref(ri)) == OK
        return r, ri.value

    def solve(self, tol=1e-10, max_cycles=100):
        s = np.zeros(4)
        st = lib().o3_solve(self._h, tol, max_cycles, _p(s))
        return st, dict(cycles=int(s[0]), res0=s[1], res=s[2], rho=s[3])

    def res_history(self):
        h = np.zeros(512)
        m = lib().o3_res_history(self._h, _p(h), 512)
        return h[:m]

    def csr(self):
        import scipy.sparse as sp
        n, nnz = ctypes.c_int(), ctypes.c_long()
        assert lib().o3_csr_size(self._h, ctypes.byref(n), ctypes.byref(nnz)) == OK
        rp = np.zeros(n.value + 1, np.int64)
        ci = np.zeros(nnz.value, np.int32)
        va = np.zeros(nnz.value)
        b = np.zeros(n.value)
        assert lib().o3_csr(self._h, _p(rp), _p(ci), _p(va), _p(b)) == OK
        return sp.csr_matrix((va, ci, rp), shape=(n.value, n.value)), b
