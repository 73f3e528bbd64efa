"""Python binding of the gpmg HIP library (include/gpmg.h).

Argument marshalling only: every computation happens in the HIP kernels of libgpmg.so.  The library is
loaded from this package directory; if it is missing the import of a GPU entry point fails loudly (there is no
CPU fallback).  Arrays are numpy host arrays (copied in/out) or, with ``on_device=True``, device pointers
given as integers (e.g. ``torch.Tensor.data_ptr()``).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libgpmg.so")

GP_OK, GP_EINVAL, GP_ENOMEM, GP_EHIP, GP_EGEOM, GP_ENOCONV, GP_EDIVERGED, GP_ESCRATCH = 0, -1, -2, -3, -4, -5, -6, -7
GP_FP64, GP_MIXED = 0, 1

EXPORTS = [
    "gp_default_params", "gp_setup_grid", "gp_destroy", "gp_num_levels", "gp_strerror", "gp_last_hip_error",
    "gp_set_levelset", "gp_set_levelset_analytic", "gp_prepare_levelset_analytic", "gp_set_walls",
    "gp_reinit_levelset",
    "gp_get_boundary_geometry",
    "gp_set_boundary_values", "gp_set_alpha", "gp_set_rhs", "gp_set_x", "gp_get_x", "gp_mg_vcycle", "gp_solve", "gp_solve_noalloc",
    "gp_residual", "gp_set_state", "gp_cn_step", "gp_get_classes", "gp_get_ghost_rows", "gp_get_ext_rows",
    "gp_get_band_layout", "gp_get_coupled_boxes",
    "gp_relax", "gp_time_kernel", "gp_probe_start", "gp_probe_stop", "gp_apply_mt", "gp_adjoint_solve", "gp_apply_cycle", "gp_apply_cycle_t",
    "gp_tape_forward", "gp_tape_backward", "gp_tape_path_gradient",
]


class GpParams(ctypes.Structure):
    _fields_ = [("nu1", ctypes.c_int), ("nu2", ctypes.c_int), ("gamma", ctypes.c_int), ("lambda_ghost", ctypes.c_int),
                ("coarsest_n", ctypes.c_int), ("march_max", ctypes.c_int), ("ext_radius", ctypes.c_int),
                ("dtau_dir", ctypes.c_double), ("dtau_neu_over_h", ctypes.c_double),
                ("bisect_eps_over_h", ctypes.c_double), ("cg_min", ctypes.c_double),
                ("mixed_inner_cycles", ctypes.c_int), ("bnd_sweeps", ctypes.c_int), ("bnd_radius", ctypes.c_int),
                ("fuse_small_levels", ctypes.c_int), ("band_split_min", ctypes.c_int),
                ("graph_iterations", ctypes.c_int), ("band_sector_min", ctypes.c_int),
                ("queue_ahead", ctypes.c_int), ("ghost_boxes", ctypes.c_int), ("krylov", ctypes.c_int),
                ("ghost_box_levels", ctypes.c_int)]


class GpRigid(ctypes.Structure):
    _fields_ = [("X0x", ctypes.c_double), ("X0y", ctypes.c_double), ("Ux", ctypes.c_double), ("Uy", ctypes.c_double),
                ("omega", ctypes.c_double)]


class GpShape(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("p", ctypes.c_double * 4)]


class GpStats(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int), ("outer", ctypes.c_int), ("res0", ctypes.c_double), ("res", ctypes.c_double),
                ("rho", ctypes.c_double), ("seconds", ctypes.c_double), ("bytes_alg", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class GpmgError(RuntimeError):
    def __init__(self, status, where, detail=""):
        self.status = status
        super().__init__(f"{where}: status {status}{(' ' + detail) if detail else ''}")


_lib = None


def lib():
    """Load libgpmg.so (built by __graft_entry__.build() / paper_1911_00994_amd/build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise RuntimeError(f"libgpmg.so not built ({LIBPATH}); run __graft_entry__.build()")
    # PyTorch carries its own HIP runtime under the same soname: loading it first makes it the one runtime of
    # the process, shared by the library (device pointers and streams pass between the two).  Loaded the other
    # way round, PyTorch finds no GPU.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIBPATH)
    vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    sigs = {
        "gp_default_params": (None, [ctypes.POINTER(GpParams)]),
        "gp_setup_grid": (i, [ctypes.POINTER(vp), i, d, ctypes.POINTER(GpParams), vp]),
        "gp_destroy": (None, [vp]),
        "gp_num_levels": (i, [vp]),
        "gp_strerror": (ctypes.c_char_p, [i]),
        "gp_last_hip_error": (ctypes.c_char_p, [vp]),
        "gp_set_levelset": (i, [vp, vp, i, d, ctypes.POINTER(GpRigid)]),
        "gp_set_levelset_analytic": (i, [vp, ctypes.POINTER(GpShape), d, ctypes.POINTER(GpRigid)]),
        "gp_prepare_levelset_analytic": (i, [vp, ctypes.POINTER(GpShape), d, ctypes.POINTER(GpRigid)]),
        "gp_set_walls": (i, [vp, vp]),
        "gp_reinit_levelset": (i, [vp, vp, i, i, d]),
        "gp_get_boundary_geometry": (i, [vp, vp, vp]),
        "gp_set_boundary_values": (i, [vp, vp, vp, vp, i]),
        "gp_set_alpha": (i, [vp, d]),
        "gp_set_rhs": (i, [vp, vp, vp, vp, i]),
        "gp_set_x": (i, [vp, vp, vp, vp, d, i]),
        "gp_get_x": (i, [vp, vp, vp, vp, vp, i]),
        "gp_mg_vcycle": (i, [vp, i, vp]),
        "gp_solve": (i, [vp, i, d, i, ctypes.POINTER(GpStats)]),
        "gp_solve_noalloc": (i, [vp, d, i, ctypes.POINTER(GpStats)]),
        "gp_residual": (i, [vp, vp, vp]),
        "gp_set_state": (i, [vp, vp, vp, vp, d, i]),
        "gp_cn_step": (i, [vp, d, vp, vp, vp, i, i, d, i, d, i, ctypes.POINTER(GpStats)]),
        "gp_get_classes": (i, [vp, i, vp]),
        "gp_get_band_layout": (i, [vp, i, vp]),
        "gp_get_coupled_boxes": (i, [vp, i, vp, vp, vp, vp, vp, vp]),
        "gp_get_ghost_rows": (i, [vp, i, vp, vp, vp, vp, vp, vp, vp]),
        "gp_get_ext_rows": (i, [vp, i, vp, vp]),
        "gp_relax": (i, [vp, i, i]),
        "gp_time_kernel": (i, [vp, i, i, i, vp]),
        "gp_probe_start": (i, [vp, i, i]),
        "gp_probe_stop": (i, [vp, vp, vp]),
        "gp_apply_mt": (i, [vp, vp, vp, i]),
        "gp_adjoint_solve": (i, [vp, vp, vp, i, d, i, ctypes.POINTER(GpStats)]),
        "gp_apply_cycle": (i, [vp, vp, vp, i]),
        "gp_apply_cycle_t": (i, [vp, vp, vp, i]),
        "gp_tape_forward": (i, [vp, ctypes.POINTER(GpShape), ctypes.POINTER(GpRigid), d, d, i, vp, vp, i, vp, d, i, d, i,
                                i, ctypes.POINTER(GpStats)]),
        "gp_tape_backward": (i, [vp, vp, vp, i, d, i, vp, vp, vp, vp, vp, ctypes.POINTER(GpStats)]),
        "gp_tape_path_gradient": (i, [vp, vp, vp]),
    }
    for name, (res, args) in sigs.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def default_params(**overrides) -> GpParams:
    p = GpParams()
    lib().gp_default_params(ctypes.byref(p))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def _host(a, dtype=np.float64):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, int):
        return ctypes.c_void_p(a)
    return a.ctypes.data_as(ctypes.c_void_p)


class Solver:
    """One gpmg context (grid hierarchy, geometry, state) on the current HIP device."""

    def __init__(self, N, Re=100.0, stream=None, **params):
        self.N, self.W, self.Re = N, N + 2, Re
        self._p = default_params(**params)
        h = ctypes.c_void_p()
        st = lib().gp_setup_grid(ctypes.byref(h), N, Re, ctypes.byref(self._p), ctypes.c_void_p(stream or 0))
        self._check(st, "gp_setup_grid", h)
        self._h = h
        self.nlev = lib().gp_num_levels(self._h)

    def _check(self, st, where, h=None):
        if st != GP_OK:
            hh = h if h is not None else getattr(self, "_h", None)
            detail = lib().gp_strerror(st).decode()
            if st == GP_EHIP and hh:
                detail += " (" + lib().gp_last_hip_error(hh).decode() + ")"
            raise GpmgError(st, where, detail)
        return st

    def close(self):
        if getattr(self, "_h", None):
            lib().gp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except TypeError:  # interpreter shutdown: module globals already cleared, the process frees the device
            pass

    def level_n(self, l):
        return self.N >> l

    # geometry -----------------------------------------------------------------------------------
    def set_levelset(self, phi, t=0.0, motion=None, on_device=False, check=True):
        m = None if motion is None else GpRigid(*[float(v) for v in list(motion)[:5]])
        src = phi if on_device else _host(phi)
        st = lib().gp_set_levelset(self._h, _ptr(src), int(on_device), t, ctypes.byref(m) if m else None)
        return self._check(st, "gp_set_levelset") if check else st

    def set_levelset_analytic(self, kind, params, t=0.0, motion=None, check=True):
        sh = GpShape(kind, (ctypes.c_double * 4)(*(list(params) + [0.0] * (4 - len(params)))))
        m = None if motion is None else GpRigid(*[float(v) for v in list(motion)[:5]])
        st = lib().gp_set_levelset_analytic(self._h, ctypes.byref(sh), t, ctypes.byref(m) if m else None)
        return self._check(st, "gp_set_levelset_analytic") if check else st

    def prepare_levelset_analytic(self, kind, params, t=0.0, motion=None):
        """start building in the background the geometry that set_levelset_analytic with the same arguments
        will then take"""
        sh = GpShape(kind, (ctypes.c_double * 4)(*(list(params) + [0.0] * (4 - len(params)))))
        m = None if motion is None else GpRigid(*[float(v) for v in list(motion)[:5]])
        st = lib().gp_prepare_levelset_analytic(self._h, ctypes.byref(sh), t, ctypes.byref(m) if m else None)
        self._check(st, "gp_prepare_levelset_analytic")

    def reinit_levelset(self, phi, iters, cfl=0.3, on_device=False):
        """gp_reinit_levelset: returns the reinitialised lattice (host arrays) or updates the device buffer in place
        (on_device: phi is a device pointer)"""
        if on_device:
            self._check(lib().gp_reinit_levelset(self._h, ctypes.c_void_p(phi), 1, iters, cfl), "gp_reinit_levelset")
            return phi
        a = _host(phi).copy()
        self._check(lib().gp_reinit_levelset(self._h, _ptr(a), 0, iters, cfl), "gp_reinit_levelset")
        return a

    def set_walls(self, walls):
        self._check(lib().gp_set_walls(self._h, _ptr(_host(walls))), "gp_set_walls")

    def boundary_geometry(self):
        W = self.W
        B = np.zeros(3 * W * W * 2)
        nB = np.zeros(3 * W * W * 2)
        self._check(lib().gp_get_boundary_geometry(self._h, _ptr(B), _ptr(nB)), "gp_get_boundary_geometry")
        B = B.reshape(3, W, W, 2)
        nB = nB.reshape(3, W, W, 2)
        return dict(B=(B[0], B[1], B[2]), nB=(nB[0], nB[1], nB[2]))

    def set_boundary_values(self, bu=None, bv=None, bp=None, on_device=False):
        args = [a if on_device else _host(a) for a in (bu, bv, bp)]
        self._check(lib().gp_set_boundary_values(self._h, *[_ptr(a) for a in args], int(on_device)),
                    "gp_set_boundary_values")

    # linear system --------------------------------------------------------------------------------
    def set_alpha(self, alpha):
        self._check(lib().gp_set_alpha(self._h, alpha), "gp_set_alpha")

    def set_rhs(self, fu=None, fv=None, g=None, on_device=False):
        args = [a if on_device else _host(a) for a in (fu, fv, g)]
        self._check(lib().gp_set_rhs(self._h, *[_ptr(a) for a in args], int(on_device)), "gp_set_rhs")

    def set_x(self, u, v, p, xi=0.0, on_device=False):
        args = [a if on_device else _host(a) for a in (u, v, p)]
        self._check(lib().gp_set_x(self._h, *[_ptr(a) for a in args], xi, int(on_device)), "gp_set_x")

    def get_x(self, device_out=None):
        """(u, v, p, xi) as host arrays; with device_out = (u, v, p) device addresses (W*W doubles each), the grids
        are copied there instead and only xi is returned"""
        W = self.W
        xi = ctypes.c_double(0)
        if device_out is not None:
            self._check(lib().gp_get_x(self._h, *[_ptr(int(a)) for a in device_out], ctypes.byref(xi), 1), "gp_get_x")
            return xi.value
        u, v, p = np.zeros((W, W)), np.zeros((W, W)), np.zeros((W, W))
        self._check(lib().gp_get_x(self._h, _ptr(u), _ptr(v), _ptr(p), ctypes.byref(xi), 0), "gp_get_x")
        return u, v, p, xi.value

    def cycle(self, precision=GP_FP64):
        r = ctypes.c_double(0)
        st = lib().gp_mg_vcycle(self._h, precision, ctypes.byref(r))
        self._check(st, "gp_mg_vcycle")
        return r.value

    def solve(self, tol=1e-10, max_cycles=100, precision=GP_FP64, check=True):
        s = GpStats()
        st = lib().gp_solve(self._h, precision, tol, max_cycles, ctypes.byref(s))
        if check and st not in (GP_OK,):
            self._check(st, "gp_solve")
        return st, s.as_dict()

    def solve_noalloc(self, tol=1e-10, max_cycles=100, check=True):
        """gp_solve_noalloc: the FP64 solve without device allocation (workspace in the library's static array)"""
        s = GpStats()
        st = lib().gp_solve_noalloc(self._h, tol, max_cycles, ctypes.byref(s))
        if check and st not in (GP_OK,):
            self._check(st, "gp_solve_noalloc")
        return st, s.as_dict()

    def residual(self):
        r = np.zeros(3 * self.W * self.W + 1)
        ri = ctypes.c_double(0)
        self._check(lib().gp_residual(self._h, _ptr(r), ctypes.byref(ri)), "gp_residual")
        return r, ri.value

    def time_kernel(self, which, level=0, reps=10):
        """average device microseconds of one launch (HIP events on the context's stream)"""
        us = ctypes.c_double(0)
        self._check(lib().gp_time_kernel(self._h, which, level, reps, ctypes.byref(us)), "gp_time_kernel")
        return us.value

    def probe_start(self, max_launches=4096, every=1):
        """record HIP events around every every-th finest-level five-colour box launch of the FP64 cycle from now
        on"""
        self._check(lib().gp_probe_start(self._h, max_launches, every), "gp_probe_start")

    def probe_stop(self):
        """(average device microseconds of the recorded launches, their number)"""
        us = ctypes.c_double(0)
        n = ctypes.c_int(0)
        self._check(lib().gp_probe_stop(self._h, ctypes.byref(us), ctypes.byref(n)), "gp_probe_stop")
        return us.value, n.value

    def relax(self, level=0, steps=1):
        self._check(lib().gp_relax(self._h, level, steps), "gp_relax")

    # time stepping ------------------------------------------------------------------------------
    def set_state(self, u, v, p, xi=0.0, on_device=False):
        args = [a if on_device else _host(a) for a in (u, v, p)]
        self._check(lib().gp_set_state(self._h, *[_ptr(a) for a in args], xi, int(on_device)), "gp_set_state")

    def cn_step(self, dt, fu=None, fv=None, g=None, on_device=False, precision=GP_FP64, tol=1e-10, max_cycles=100,
                picard_eps=1e-6, picard_max=20, check=True):
        args = [a if on_device else _host(a) for a in (fu, fv, g)]
        s = GpStats()
        st = lib().gp_cn_step(self._h, dt, *[_ptr(a) for a in args], int(on_device), precision, tol, max_cycles,
                              picard_eps, picard_max, ctypes.byref(s))
        if check and st != GP_OK:
            self._check(st, "gp_cn_step")
        return st, s.as_dict()

    # inspection ---------------------------------------------------------------------------------
    def classes(self, level=0):
        W = self.level_n(level) + 2
        out = np.zeros(3 * W * W, dtype=np.uint8)
        self._check(lib().gp_get_classes(self._h, level, _ptr(out)), "gp_get_classes")
        return out.reshape(3, W, W)

    def band_layout(self, level=0):
        """Band cells, body ghost rows, angular sectors (0: none) and whether the one-workgroup kernel fits."""
        out = np.zeros(4, dtype=np.int32)
        self._check(lib().gp_get_band_layout(self._h, level, _ptr(out)), "gp_get_band_layout")
        return {"nband": int(out[0]), "nbg": int(out[1]), "sectors": int(out[2]), "lds_ok": bool(out[3])}

    def coupled_boxes(self, level=0):
        """The coupled-box table of one level (boxes in visiting order: colour, then cell)."""
        cnt = np.zeros(2, dtype=np.int32)
        self._check(lib().gp_get_coupled_boxes(self._h, level, _ptr(cnt), None, None, None, None, None),
                    "gp_get_coupled_boxes")
        nb, ns = int(cnt[0]), int(cnt[1])
        cell = np.zeros(max(nb, 1), dtype=np.int32)
        off = np.zeros(nb + 1, dtype=np.int32)
        idx = np.zeros(max(ns, 1), dtype=np.int32)
        wr = np.zeros(max(ns, 1), dtype=np.uint8)
        coff = np.zeros(6, dtype=np.int32)
        self._check(lib().gp_get_coupled_boxes(self._h, level, _ptr(cnt), _ptr(cell), _ptr(off), _ptr(idx), _ptr(wr),
                                               _ptr(coff)), "gp_get_coupled_boxes")
        return dict(cell=cell[:nb], off=off, idx=idx[:ns], wr=wr[:ns], coff=coff)

    def ghost_rows(self, level=0):
        W = self.level_n(level) + 2
        P = 3 * W * W
        B, nB, th = np.zeros(2 * P), np.zeros(2 * P), np.zeros(2 * P)
        w9 = np.zeros(9 * P)
        c9 = np.zeros(9 * P, dtype=np.int32)
        dt = np.zeros(P)
        kind = np.zeros(P, dtype=np.int32)
        self._check(lib().gp_get_ghost_rows(self._h, level, _ptr(B), _ptr(nB), _ptr(th), _ptr(w9), _ptr(c9), _ptr(dt),
                                            _ptr(kind)), "gp_get_ghost_rows")
        return dict(B=B.reshape(P, 2), nB=nB.reshape(P, 2), theta=th.reshape(P, 2), w=w9.reshape(P, 9),
                    col=c9.reshape(P, 9), dtau=dt, valid=kind)

    def ext_rows(self, level=0):
        W = self.level_n(level) + 2
        P = 3 * W * W
        src = np.zeros(3 * P, dtype=np.int32)
        w = np.zeros(3 * P)
        self._check(lib().gp_get_ext_rows(self._h, level, _ptr(src), _ptr(w)), "gp_get_ext_rows")
        return src.reshape(P, 3), w.reshape(P, 3)

    # transposed system ----------------------------------------------------------------------------
    def nvec(self):
        return 3 * self.W * self.W + 1

    def _vec_op(self, name, v):
        v = _host(v)
        assert v.size == self.nvec()
        out = np.zeros(self.nvec())
        self._check(getattr(lib(), name)(self._h, _ptr(v), _ptr(out), 0), name)
        return out

    def apply_mt(self, lam):
        """y = M^T lam (full unknown vectors of length 3 W^2 + 1)."""
        return self._vec_op("gp_apply_mt", lam)

    def apply_cycle(self, b):
        """x = B' b: one FP64 cycle from x = 0 (overwrites the current x and b)."""
        return self._vec_op("gp_apply_cycle", b)

    def apply_cycle_t(self, xbar):
        """bbar = B'^T xbar (the transposed cycle)."""
        return self._vec_op("gp_apply_cycle_t", xbar)

    def adjoint_solve(self, g, tol=1e-10, max_cycles=200, check=True):
        g = _host(g)
        lam = np.zeros(self.nvec())
        s = GpStats()
        st = lib().gp_adjoint_solve(self._h, _ptr(g), _ptr(lam), 0, tol, max_cycles, ctypes.byref(s))
        if check and st != GP_OK:
            self._check(st, "gp_adjoint_solve")
        return lam, st, s.as_dict()

    # reverse mode of a run of steps ---------------------------------------------------------------
    def tape_forward(self, kind, params, motion, t0, dt, nsteps, fu=None, fv=None, ub_offset=None, tol=1e-10,
                     max_cycles=100, picard_eps=1e-6, picard_max=20, checkpoint_every=8, on_device=False):
        """fu, fv: host arrays, or device addresses when on_device"""
        sh = GpShape()
        sh.kind = kind
        for q, v in enumerate(list(params)[:4]):
            sh.p[q] = v
        mo = GpRigid(*[float(v) for v in motion[:5]])
        off = None if ub_offset is None else np.ascontiguousarray(ub_offset, dtype=np.float64)
        s = GpStats()
        f = [_ptr(None if a is None else int(a)) if on_device else _ptr(_host(a)) for a in (fu, fv)]
        st = lib().gp_tape_forward(self._h, ctypes.byref(sh), ctypes.byref(mo), t0, dt, nsteps, f[0], f[1],
                                   int(on_device), _ptr(off), tol, max_cycles, picard_eps, picard_max,
                                   checkpoint_every, ctypes.byref(s))
        self._check(st, "gp_tape_forward")
        return s.as_dict()

    def tape_backward(self, seed_u, seed_v, tol=1e-10, max_cycles=200, device_out=None):
        """host seeds and outputs; with device_out = (dfu, dfv, du0, dv0) device addresses (any may be None), the
        seeds are device addresses too and the grids go there (the dict then holds dU and stats only)"""
        W = self.W
        dU = np.zeros(2)
        s = GpStats()
        if device_out is not None:
            outs = [_ptr(None if a is None else int(a)) for a in device_out]
            st = lib().gp_tape_backward(self._h, _ptr(int(seed_u)), _ptr(int(seed_v)), 1, tol, max_cycles, outs[0],
                                        outs[1], _ptr(dU), outs[2], outs[3], ctypes.byref(s))
            self._check(st, "gp_tape_backward")
            return dict(dU=dU, stats=s.as_dict())
        dfu, dfv, du0, dv0 = (np.zeros((W, W)) for _ in range(4))
        st = lib().gp_tape_backward(self._h, _ptr(_host(seed_u)), _ptr(_host(seed_v)), 0, tol, max_cycles, _ptr(dfu),
                                    _ptr(dfv), _ptr(dU), _ptr(du0), _ptr(dv0), ctypes.byref(s))
        self._check(st, "gp_tape_backward")
        return dict(dfu=dfu, dfv=dfv, dU=dU, du0=du0, dv0=dv0, stats=s.as_dict())

    def tape_path_gradient(self):
        """(dJ/dU through the body path, count of rows whose Alg. 1 path was not reproduced) of the last
        tape_backward; the total derivative along the motion's velocity is dU + this"""
        g = np.zeros(2)
        m = ctypes.c_int()
        self._check(lib().gp_tape_path_gradient(self._h, _ptr(g), ctypes.byref(m)), "gp_tape_path_gradient")
        return g, m.value
