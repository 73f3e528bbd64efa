"""gp_solve_noalloc, the allocation-free FP64 solve, called through the C ABI: its result equals gp_solve's on the
same problem (same iteration; compared at the FP64 parity bar of 1e-10 relative), on two calls in a row on two
contexts, the second with a smaller grid (both share the library's static scratch array), and a problem whose
workspace exceeds the array is refused with GP_ESCRATCH."""
import sys

import numpy as np
import pytest

from paper_1911_00994_amd import workloads as wl

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _problem(gpmg, N, **prm):
    """the translating-ellipse manufactured linear problem at t = 0.3 on a fresh context"""
    s = gpmg.Solver(N, Re=100.0, **prm)
    sh = wl.Shape(wl.ELLIPSE_SQRT, (0.4, 0.2, 0.0))
    mo = wl.Motion(U=(0.5, 0.0)).as_array()
    s.set_levelset_analytic(sh.kind, sh.params, 0.3, mo[:5])
    alpha = 0.64 * (2.0 / N) ** 2
    s.set_alpha(alpha)
    m = wl.TaylorGreenMMS()
    fu, fv, g = wl.mms_linear_rhs(m, N, 0.3, alpha)
    geo = s.boundary_geometry()
    bu, bv, bp = wl.boundary_values_from(m, _with_walls(s, geo), 0.3, 0.3)
    s.set_boundary_values(bu, bv, bp)
    s.set_rhs(fu, fv, g)
    W = N + 2
    z = np.zeros((W, W))
    s.set_x(z, z, z, 0.0)
    return s


def _with_walls(s, g):
    import oracle as O
    B = [b.copy() for b in g["B"]]
    cls = s.classes()
    for k in range(3):
        x, y = wl.node_coords(s.N, k)
        msk = cls[k] == O.C_WALLD
        B[k][msk, 0] = x[msk]
        B[k][msk, 1] = y[msk]
    return dict(B=tuple(B), nB=g["nB"])


def _flat(s):
    u, v, p, xi = s.get_x()
    return np.concatenate([u.ravel(), v.ravel(), p.ravel(), [xi]])


def test_noalloc_solve_matches_solve_on_two_calls():
    from paper_1911_00994_amd import gpmg
    for N in (256, 128):
        say(f"[noalloc] N={N}: gp_solve reference")
        ref = _problem(gpmg, N)
        st, info = ref.solve(1e-10, 60)
        assert st == gpmg.GP_OK, info
        a = _flat(ref)
        cls = ref.classes().ravel()
        ref.close()
        say(f"[noalloc] N={N}: gp_solve_noalloc")
        s = _problem(gpmg, N)
        st, info2 = s.solve_noalloc(1e-10, 60)
        assert st == gpmg.GP_OK, info2
        b = _flat(s)
        s.close()
        act = np.concatenate([(cls == 1) | (cls == 2) | (cls == 3) | (cls == 4) | (cls == 7), [True]])
        d = np.abs(a - b)[act].max() / max(1.0, np.abs(a[act]).max())
        say(f"  cycles {info['cycles']} / {info2['cycles']}, rel diff {d:.2e}")
        assert info["cycles"] == info2["cycles"]
        assert d < 1e-10, d


def test_noalloc_plain_cycle_any_size_and_refusal():
    from paper_1911_00994_amd import gpmg
    say("[noalloc] N=512 krylov=0 (no workspace) against gp_solve")
    ref = _problem(gpmg, 512, krylov=0, ghost_box_levels=99)
    st, info = ref.solve(1e-9, 80)
    a = _flat(ref)
    ref.close()
    s = _problem(gpmg, 512, krylov=0, ghost_box_levels=99)
    st2, info2 = s.solve_noalloc(1e-9, 80, check=False)
    b = _flat(s)
    s.close()
    assert st == st2 and info["cycles"] == info2["cycles"], (st, st2, info, info2)
    assert np.array_equal(a, b)
    say("[noalloc] N=512, default krylov = 8: refused (workspace beyond the static array)")
    s = _problem(gpmg, 512)
    st3, _ = s.solve_noalloc(1e-9, 80, check=False)
    msg = gpmg.lib().gp_last_hip_error(s._h).decode()
    s.close()
    say(f"  status {st3}: {msg}")
    assert st3 == gpmg.GP_ESCRATCH and "exceeds" in msg
