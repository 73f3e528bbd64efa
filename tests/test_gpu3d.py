"""The 3-D path on the GPU (include/gpmg3.h) against the 3-D oracle, element by element:
* geometry on every level: classes bit-identical; boundary points, theta, the 27 weights and columns, dtau within
  1e-12 (sphere and ellipsoid, N = 16 and 32);
* relaxation steps and plain cycles from the same iterate within 1e-11;
* the converged GCR solve within 1e-10 of the oracle's, and the L1 velocity error of a manufactured solution
  second order on the GPU from N = 32 to 64 to 128.
Every case prints its name before it touches the GPU."""
import sys

import numpy as np
import pytest

from oracle import o3

pytestmark = pytest.mark.gpu

CASES = [(o3.SPHERE, (0.35, 0, 0, 0.02, -0.03, 0.01)), (o3.ELLIPSOID, (0.5, 0.3, 0.35, -0.05, 0.02, 0.0))]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def pair(N, kind, params, **kw):
    from paper_1911_00994_amd import gpmg3
    h = 2.0 / N
    o = o3.Oracle3(N, **kw)
    assert o.set_levelset(o3.levelset_analytic(kind, params, N)) == o3.OK
    o.set_alpha(0.64 * h * h)
    s = gpmg3.Solver3(N, **{k: v for k, v in kw.items() if k in ("krylov", "nu1", "nu2", "gamma")})
    s.set_levelset_analytic(kind, params)
    s.set_alpha(0.64 * h * h)
    return o, s


def active(cls):
    return np.concatenate([np.isin(cls.ravel(), [1, 2, 3, 4, 7]), [True]])


@pytest.mark.parametrize("N", [16, 32])
@pytest.mark.parametrize("case", [0, 1])
def test_geometry_parity(N, case):
    kind, params = CASES[case]
    say(f"[3d geometry] N={N} kind={kind}")
    o, s = pair(N, kind, params)
    for l in range(s.num_levels()):
        co, cs = o.classes(l), s.classes(l)
        assert np.array_equal(co, cs), (l, np.argwhere(co != cs)[:5])
        go, gs = o.ghost_rows(l), s.ghost_rows(l)
        rows = np.isin(co.ravel(), [2, 4, 7])
        for k in ("B", "theta", "w"):
            d = np.abs(np.nan_to_num(go[k][rows]) - np.nan_to_num(gs[k][rows])).max()
            assert d < 1e-12, (l, k, d)
        assert np.array_equal(go["col"][rows], gs["col"][rows]), l
        assert np.abs(go["dtau"][rows] - gs["dtau"][rows]).max() < 1e-15
    say(f"  {s.num_levels()} levels, {int(np.isin(co, [2, 7]).sum())} coarsest ghosts")
    s.close()


def _random_problem(o, s, N, seed):
    rng = np.random.default_rng(seed)
    W = N + 2
    f = [rng.standard_normal(W ** 3) for _ in range(4)]
    bv = [rng.standard_normal(W ** 3) for _ in range(4)]
    x0 = rng.standard_normal(4 * W ** 3 + 1)
    for side in (o, s):
        side.set_rhs(*f)
        side.set_boundary_values(*bv)
        side.set_x(x0)


@pytest.mark.parametrize("case", [0, 1])
def test_relaxation_and_cycle_parity(case):
    kind, params = CASES[case]
    N = 32
    say(f"[3d relax/cycle] N={N} kind={kind}")
    o, s = pair(N, kind, params, krylov=0)
    _random_problem(o, s, N, 3)
    act = active(o.classes())
    o.relax(0, 2)
    s.relax(2)
    a, b = o.get_x(), s.get_x()
    d = np.abs(a - b)[act].max() / max(1.0, np.abs(a[act]).max())
    say(f"  two relaxation steps: rel diff {d:.2e}")
    assert d < 1e-11
    for c in range(3):
        so, _ = o.solve(1e-300, 1)  # one cycle (and the mean projection)
        s.cycle()
        a, b = o.get_x(), s.get_x()
        d = np.abs(a - b)[act].max() / max(1.0, np.abs(a[act]).max())
        say(f"  cycle {c}: rel diff {d:.2e}")
        assert d < 1e-10
    s.close()


@pytest.mark.parametrize("case", [0, 1])
def test_solve_parity(case):
    kind, params = CASES[case]
    N = 32
    say(f"[3d solve] N={N} kind={kind}")
    o, s = pair(N, kind, params)
    _random_problem(o, s, N, 4)
    W = N + 2
    z = np.zeros(4 * W ** 3 + 1)
    o.set_x(z)
    s.set_x(z)
    so, io = o.solve(1e-11, 80)
    ss, is_ = s.solve(1e-11, 80)
    assert so == 0 and ss == 0, (so, io, ss, is_)
    a, b = o.get_x(), s.get_x()
    act = active(o.classes())
    d = np.abs(a - b)[act].max() / max(1.0, np.abs(a[act]).max())
    say(f"  oracle {io['cycles']} / GPU {is_['cycles']} GCR iterations, rel diff {d:.2e}")
    assert d < 1e-10
    s.close()


def test_second_order_on_the_gpu():
    from paper_1911_00994_amd import gpmg3
    from tests.test_oracle3d import _MMS
    m = _MMS()
    errs = []
    for N in (32, 64, 128):
        say(f"[3d accuracy] N={N}")
        h = 2.0 / N
        alpha = 0.64 * h * h
        s = gpmg3.Solver3(N)
        c0 = np.array([0.02, -0.03, 0.01])
        s.set_levelset_analytic(o3.SPHERE, (0.35, 0, 0, *c0))
        s.set_alpha(alpha)
        grids = [o3.node_coords(N, g) for g in range(4)]
        f = [(m.f(g, *grids[g]) - alpha * m.lap(g, *grids[g]) + m.f(3, *grids[g], d=g)).ravel() for g in range(3)]
        div = sum(m.f(g, *grids[3], d=g) for g in range(3)).ravel()
        s.set_rhs(f[0], f[1], f[2], div)
        gr = s.ghost_rows()
        W = N + 2
        cls = s.classes()
        bv = []
        for g in range(4):
            B = gr["B"][g * W ** 3:(g + 1) * W ** 3]
            walld = cls[g].ravel() == o3.C_WALLD
            Xg = [a.ravel() for a in grids[g]]
            Bc = [np.where(walld, Xg[d], np.nan_to_num(B[:, d])) for d in range(3)]
            if g < 3:
                bv.append(m.f(g, *Bc))
            else:
                nn = np.stack([Bc[d] - c0[d] for d in range(3)])
                nn = -nn / np.maximum(np.linalg.norm(nn, axis=0), 1e-300)
                bv.append(sum(nn[d] * m.f(3, *Bc, d=d) for d in range(3)))
        s.set_boundary_values(*bv)
        s.set_x(np.zeros(s.n))
        st, info = s.solve(1e-10, 100)
        assert st == 0, (N, info)
        x = s.get_x()
        e = 0
        for g in range(3):
            sel = cls[g].ravel() == o3.C_INT
            ex = m.f(g, *grids[g]).ravel()
            e = max(e, np.abs(x[g * W ** 3:(g + 1) * W ** 3] - ex)[sel].mean())
        say(f"  {info['cycles']} GCR iterations, {info['seconds'] * 1e3:.1f} ms, L1 velocity error {e:.3e}")
        errs.append(e)
        s.close()
    say(f"  ratios {errs[0] / errs[1]:.2f} {errs[1] / errs[2]:.2f}")
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0
