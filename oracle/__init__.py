"""Plain FP64 CPU oracle of the ghost-point multigrid Navier-Stokes method (arXiv:1911.00994).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP library: the C source next to
this file is compiled on its own (``build_oracle()``) and loaded through ctypes.

Every routine restates the paper; see the header of ``gpmg_oracle.c`` for the section map.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gpmg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

C_INACTIVE, C_INT, C_GHOST, C_WALLD, C_WALLG, C_EXT, C_GHOSTX = 0, 1, 2, 3, 4, 5, 7

OK, E_INVAL, E_NOMEM, E_HIP, E_GEOM, E_NOCONV, E_DIVERGED = 0, -1, -2, -3, -4, -5, -6


def build_oracle(force: bool = False) -> str:
    """Compile the oracle with plain gcc (no GPU code involved), portable flags, one thread."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def build_native(path: str, openmp: bool) -> str:
    """Compile the oracle for the CPU it runs on (-O3 -march=native, with or without OpenMP over the boxes of a
    colour, the ghost rows and the rows of the residual and transfers) into path: the CPU-baseline timing builds
    it on the host it times, so the machine code matches that host.  Results equal the portable build's to
    rounding (FMA contraction may differ)."""
    tmp = path + ".tmp"
    flags = ["-O3", "-march=native", "-std=c99", "-fPIC", "-shared"] + (["-fopenmp"] if openmp else [])
    subprocess.check_call(["gcc"] + flags + ["-o", tmp, _SRC, "-lm"])
    os.replace(tmp, path)
    return path


_lib = None


def lib(path: str = None):
    """the portable library (default) or, with path, a library built by build_native (loaded as the module's
    library from then on)"""
    global _lib
    if path is not None:
        _lib = None
    if _lib is None:
        _lib = ctypes.CDLL(path or build_oracle())
        L = _lib
        d, i, vp = ctypes.c_double, ctypes.c_int, ctypes.c_void_p
        L.or_create.restype = vp
        L.or_create.argtypes = [i, d, vp, vp]
        L.or_destroy.argtypes = [vp]
        for name, args in [
            ("or_levelset_analytic", [i, vp, vp, d, i, vp]),
            ("or_set_levelset", [vp, vp, d, vp]),
            ("or_num_levels", [vp]),
            ("or_level_n", [vp, i]),
            ("or_get_classes", [vp, i, vp]),
            ("or_get_ghost_rows", [vp, i, vp, vp, vp, vp, vp, vp, vp]),
            ("or_get_ext_rows", [vp, i, vp, vp, vp]),
            ("or_set_alpha", [vp, d]),
            ("or_get_csr_size", [vp, i, vp, vp]),
            ("or_get_csr", [vp, i, vp, vp, vp, vp]),
            ("or_relax", [vp, i, i]),
            ("or_cycle", [vp, vp]),
            ("or_solve", [vp, d, i, vp]),
            ("or_res_history", [vp, vp, i]),
            ("or_residual", [vp, vp, vp]),
            ("or_set_state", [vp, vp, vp, vp, d]),
            ("or_cn_step", [vp, d, vp, vp, vp, d, i, d, i, vp]),
            ("or_ext_fail_count", [vp, i]),
            ("or_test_restrict", [vp, i, vp, vp]),
            ("or_test_prolong", [vp, i, vp, vp]),
            ("or_threads", []),
            ("or_coupled_box_count", [vp, i, vp, vp]),
            ("or_get_coupled_boxes", [vp, i, vp, vp, vp, vp, vp, vp]),
            ("or_reinit", [vp, i, d, i, d, vp]),
        ]:
            f = getattr(L, name)
            f.restype = i
            f.argtypes = args
        for name, args in [
            ("or_st9_dirichlet", [d, d, vp]),
            ("or_st9_neumann", [d, d, d, d, d, d, d, vp]),
            ("or_set_walls", [vp, vp]),
            ("or_set_boundary_values", [vp, vp, vp, vp]),
            ("or_set_rhs", [vp, vp, vp, vp]),
            ("or_set_x", [vp, vp, vp, vp, d]),
            ("or_get_x", [vp, vp, vp, vp, vp]),
            ("or_get_b", [vp, vp]),
            ("or_ext_fill_finest", [vp]),
            ("or_set_conv_history", [vp, vp, vp, vp, vp, vp, vp, i]),
        ]:
            f = getattr(L, name)
            f.restype = None
            f.argtypes = args
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def st9_dirichlet(thx: float, thy: float) -> np.ndarray:
    """Weights of eq. (BCu): w[ky, kx] = T_kx(theta_x) T_ky(theta_y)."""
    w = np.zeros(9)
    lib().or_st9_dirichlet(thx, thy, _p(w))
    return w.reshape(3, 3)


def st9_neumann(thx, thy, sx, sy, nx, ny, h) -> np.ndarray:
    w = np.zeros(9)
    lib().or_st9_neumann(thx, thy, sx, sy, nx, ny, h, _p(w))
    return w.reshape(3, 3)


def levelset_analytic(kind: int, sp, motion, t: float, N: int) -> np.ndarray:
    """phi on the (2N+1)^2 half-step lattice, positive inside the body (Sect. 3.1)."""
    phi = np.zeros((2 * N + 1, 2 * N + 1))
    sp = _f64(np.asarray(list(sp) + [0.0] * (4 - len(sp))))
    mo = _f64(np.asarray(list(motion) + [0.0] * (6 - len(motion))))
    st = lib().or_levelset_analytic(kind, _p(sp), _p(mo), t, N, _p(phi))
    assert st == OK
    return phi


def reinit(phi0, dx: float, iters: int, cfl: float = 0.3) -> np.ndarray:
    """Reinitialisation of a level set sampled on a square lattice of spacing dx towards the signed distance
    (Sect. 3.1, eq. (sdf)); the discretisation is described at or_reinit."""
    a = _f64(np.asarray(phi0))
    n = a.shape[0]
    assert a.shape == (n, n)
    out = np.zeros_like(a)
    st = lib().or_reinit(_p(a), n, dx, iters, cfl, _p(out))
    assert st == OK, st
    return out


class Oracle:
    """Handle on one oracle solver (all levels of one grid hierarchy)."""

    def __init__(self, N, Re=100.0, nu1=2, nu2=2, gamma=1, lam=2, coarsest_n=8, march_max=8, ext_radius=4,
                 perm_seed=0, dtau_dir=0.9, dtau_neu_over_h=0.9, eps_over_h=0.01, cg_min=0.1, bnd_sweeps=0, bnd_radius=2,
                 ghost_boxes=1, lex_order=0, krylov=8, ghost_box_levels=1):
        self.N, self.W, self.Re = N, N + 2, Re
        ip = np.array([nu1, nu2, gamma, lam, coarsest_n, march_max, ext_radius, perm_seed, bnd_sweeps, bnd_radius,
                       ghost_boxes, lex_order, krylov, ghost_box_levels], dtype=np.int32)
        dp = np.array([dtau_dir, dtau_neu_over_h, eps_over_h, cg_min], dtype=np.float64)
        self._h = lib().or_create(N, Re, _p(ip), _p(dp))
        if not self._h:
            raise ValueError("oracle: invalid grid parameters")
        self.nlev = lib().or_num_levels(self._h)

    def __del__(self):
        if getattr(self, "_h", None):
            lib().or_destroy(self._h)
            self._h = None

    # geometry -------------------------------------------------------------------------------
    def set_levelset(self, phi, t=0.0, motion=None) -> int:
        mo = None if motion is None else _f64(np.asarray(list(motion) + [0.0] * (6 - len(motion))))
        return lib().or_set_levelset(self._h, _p(_f64(phi)), t, _p(mo))

    def set_walls(self, walls):
        lib().or_set_walls(self._h, _p(_f64(np.asarray(walls, dtype=np.float64))))

    def set_boundary_values(self, bu=None, bv=None, bp=None):
        lib().or_set_boundary_values(self._h, _p(_f64(bu)), _p(_f64(bv)), _p(_f64(bp)))

    def level_n(self, l):
        return lib().or_level_n(self._h, l)

    def classes(self, l=0) -> np.ndarray:
        W = self.level_n(l) + 2
        out = np.zeros(3 * W * W, dtype=np.uint8)
        assert lib().or_get_classes(self._h, l, _p(out)) == OK
        return out.reshape(3, W, W)

    def ghost_rows(self, l=0) -> dict:
        W = self.level_n(l) + 2
        P = 3 * W * W
        B = np.zeros(2 * P)
        nB = np.zeros(2 * P)
        th = np.zeros(2 * P)
        w9 = np.zeros(9 * P)
        c9 = np.zeros(9 * P, dtype=np.int32)
        dt = np.zeros(P)
        va = np.zeros(P, dtype=np.int32)
        assert lib().or_get_ghost_rows(self._h, l, _p(B), _p(nB), _p(th), _p(w9), _p(c9), _p(dt), _p(va)) == OK
        return dict(B=B.reshape(P, 2), nB=nB.reshape(P, 2), theta=th.reshape(P, 2), w=w9.reshape(P, 9),
                    col=c9.reshape(P, 9), dtau=dt, valid=va)

    def coupled_boxes(self, l=0) -> dict:
        """The coupled-box table of level l (boxes in visiting order: colour, then cell index)."""
        nb, ns = ctypes.c_int(0), ctypes.c_int(0)
        assert lib().or_coupled_box_count(self._h, l, ctypes.byref(nb), ctypes.byref(ns)) == OK
        cell = np.zeros(max(nb.value, 1), dtype=np.int32)
        off = np.zeros(nb.value + 1, dtype=np.int32)
        nbx = np.zeros(max(nb.value, 1), dtype=np.int32)
        idx = np.zeros(max(ns.value, 1), dtype=np.int32)
        wr = np.zeros(max(ns.value, 1), dtype=np.uint8)
        coff = np.zeros(6, dtype=np.int32)
        assert lib().or_get_coupled_boxes(self._h, l, _p(cell), _p(off), _p(nbx), _p(idx), _p(wr), _p(coff)) == OK
        return dict(cell=cell[:nb.value], off=off, nbox=nbx[:nb.value], idx=idx[:ns.value], wr=wr[:ns.value],
                    coff=coff)

    def ext_rows(self, l=0):
        W = self.level_n(l) + 2
        P = 3 * W * W
        src = np.zeros(3 * P, dtype=np.int32)
        w = np.zeros(3 * P)
        fail = ctypes.c_int(0)
        assert lib().or_get_ext_rows(self._h, l, _p(src), _p(w), ctypes.byref(fail)) == OK
        return src.reshape(P, 3), w.reshape(P, 3), fail.value

    # linear system ---------------------------------------------------------------------------
    def set_alpha(self, alpha) -> int:
        return lib().or_set_alpha(self._h, alpha)

    def csr(self, l=0):
        import scipy.sparse as sp
        n = ctypes.c_int(0)
        nnz = ctypes.c_int(0)
        lib().or_get_csr_size(self._h, l, ctypes.byref(n), ctypes.byref(nnz))
        rp = np.zeros(n.value + 1, dtype=np.int32)
        ci = np.zeros(nnz.value, dtype=np.int32)
        va = np.zeros(nnz.value)
        b = np.zeros(n.value)
        lib().or_get_csr(self._h, l, _p(rp), _p(ci), _p(va), _p(b))
        return sp.csr_matrix((va, ci, rp), shape=(n.value, n.value)), b

    def set_rhs(self, fu=None, fv=None, g=None):
        lib().or_set_rhs(self._h, _p(_f64(fu)), _p(_f64(fv)), _p(_f64(g)))

    def set_x(self, u, v, p, xi=0.0):
        lib().or_set_x(self._h, _p(_f64(u)), _p(_f64(v)), _p(_f64(p)), xi)

    def get_x(self):
        W = self.W
        u, v, p = np.zeros(W * W), np.zeros(W * W), np.zeros(W * W)
        xi = ctypes.c_double(0)
        lib().or_get_x(self._h, _p(u), _p(v), _p(p), ctypes.byref(xi))
        return u.reshape(W, W), v.reshape(W, W), p.reshape(W, W), xi.value

    def get_b(self):
        b = np.zeros(3 * self.W * self.W + 1)
        lib().or_get_b(self._h, _p(b))
        return b

    def relax(self, l, steps=1):
        return lib().or_relax(self._h, l, steps)

    def cycle(self):
        r = ctypes.c_double(0)
        st = lib().or_cycle(self._h, ctypes.byref(r))
        return st, r.value

    def solve(self, tol=1e-10, max_cycles=100):
        stats = np.zeros(4)
        st = lib().or_solve(self._h, tol, max_cycles, _p(stats))
        return st, dict(cycles=int(stats[0]), res0=stats[1], res=stats[2], rho=stats[3])

    def res_history(self):
        out = np.zeros(1024)
        m = lib().or_res_history(self._h, _p(out), 1024)
        return out[:m].copy()

    def residual(self):
        r = np.zeros(3 * self.W * self.W + 1)
        ri = ctypes.c_double(0)
        lib().or_residual(self._h, _p(r), ctypes.byref(ri))
        return r, ri.value

    def test_restrict(self, l, r_fine):
        Wc = self.level_n(l + 1) + 2
        out = np.zeros(3 * Wc * Wc + 1)
        assert lib().or_test_restrict(self._h, l, _p(_f64(r_fine)), _p(out)) == OK
        return out

    def test_prolong(self, l, e_coarse, x_fine):
        x = _f64(np.array(x_fine, dtype=np.float64, copy=True))
        assert lib().or_test_prolong(self._h, l, _p(_f64(e_coarse)), _p(x)) == OK
        return x

    def ext_fill_finest(self):
        lib().or_ext_fill_finest(self._h)

    def ext_fail_count(self, l=0):
        return lib().or_ext_fail_count(self._h, l)

    # time stepping ---------------------------------------------------------------------------
    def set_conv_history(self, cu, cv, nstep):
        """Test hook: convection histories [c^n, c^{n-1}, c^{n-2}] for the u and v grids."""
        a = [_f64(np.asarray(x)) for x in (cu[0], cv[0], cu[1], cv[1], cu[2], cv[2])]
        lib().or_set_conv_history(self._h, *[_p(x) for x in a], nstep)

    def set_state(self, u, v, p, xi=0.0) -> int:
        return lib().or_set_state(self._h, _p(_f64(u)), _p(_f64(v)), _p(_f64(p)), xi)

    def cn_step(self, dt, fu=None, fv=None, g=None, tol=1e-10, max_cycles=100, picard_eps=1e-6, picard_max=20):
        stats = np.zeros(5)
        st = lib().or_cn_step(self._h, dt, _p(_f64(fu)), _p(_f64(fv)), _p(_f64(g)), tol, max_cycles, picard_eps,
                              picard_max, _p(stats))
        return st, dict(cycles=int(stats[0]), picard=int(stats[1]), res=stats[2], rho=stats[3], picard_res=stats[4])
