"""Parity of the HIP path with the CPU oracle (element by element, same seeded inputs).

FP64 bar: geometry tables within 1e-12 (classes and coupled-box tables bit-exact), one relaxation step / one
cycle within 1e-11 relative, converged solves and Crank-Nicolson steps within 1e-10 relative (the measured
difference is printed).  Every case prints its name before touching the GPU.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1911_00994_amd import workloads as wl
from tests.common import active_mask, oracle_geom

pytestmark = pytest.mark.gpu

CIRCLE = wl.Shape(wl.CIRCLE_DIST, (0.3,))
ELLIPSE = wl.Shape(wl.ELLIPSE_SQRT, (0.4, 0.2, 0.0))
FLOWER = wl.Shape(wl.PETALS, (0.35, 0.07, 0.0, 5.0))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_solver(N, Re=100.0, **kw):
    from paper_1911_00994_amd import gpmg
    return gpmg.Solver(N, Re=Re, **kw)


# solver parameters that exist on both sides under the same name (the oracle's lambda is lam)
SHARED = ("nu1", "nu2", "gamma", "ghost_boxes", "krylov", "ghost_box_levels", "bnd_sweeps")


def pair(N, shape, alpha, motion=None, t=0.0, m=None, Re=100.0, zero_x=True, **gpu_params):
    """oracle and GPU solver on the same level set, alpha, rhs and boundary data (shared solver parameters go
    to both sides)"""
    o = O.Oracle(N, Re=Re, **{k: v for k, v in gpu_params.items() if k in SHARED})
    mo = motion.as_array() if motion is not None else np.zeros(6)
    phi = O.levelset_analytic(shape.kind, shape.padded(), mo, t, N)
    assert o.set_levelset(phi, t, mo) == O.OK
    o.set_alpha(alpha)
    s = gpu_solver(N, Re=Re, **gpu_params)
    s.set_levelset(phi, t, mo[:5])
    s.set_alpha(alpha)
    m = m or wl.TaylorGreenMMS()
    fu, fv, g = wl.mms_linear_rhs(m, N, t, alpha)
    bu, bv, bp = wl.boundary_values_from(m, oracle_geom(o), t, t)
    W = N + 2
    if zero_x:
        z = np.zeros((W, W))
        o.set_x(z, z, z, 0.0)
        s.set_x(z, z, z, 0.0)
    for side in (o, s):
        side.set_boundary_values(bu, bv, bp)
        side.set_rhs(fu, fv, g)
    return o, s


def flat(xs):
    u, v, p, xi = xs
    return np.concatenate([u.ravel(), v.ravel(), p.ravel(), [xi]])


def rel_diff(a, b, mask):
    d = np.abs(a - b)[mask].max()
    return d / max(1.0, np.abs(a[mask]).max())


@pytest.mark.parametrize("N,shape", [(64, CIRCLE), (128, ELLIPSE), (256, FLOWER), (256, wl.paper_flower())])
def test_geometry_parity(N, shape):
    say(f"[geometry] N={N} shape={shape}")
    o, s = pair(N, shape, 0.64 * (2.0 / N) ** 2)
    for l in range(o.nlev):
        co, cg = o.classes(l), s.classes(l)
        assert np.array_equal(co, cg), (l, np.argwhere(co != cg)[:5])
        go, gg = o.ghost_rows(l), s.ghost_rows(l)
        rows = go["valid"] >= 0
        assert np.array_equal(rows, gg["valid"] >= 0)
        assert np.array_equal(go["valid"][rows], gg["valid"][rows])
        assert np.array_equal(go["col"][rows], gg["col"][rows])
        for key in ("w", "theta", "B", "nB", "dtau"):
            a, b = go[key][rows], gg[key][rows]
            fin = np.isfinite(a)
            assert np.array_equal(fin, np.isfinite(b)), key
            assert np.abs(a[fin] - b[fin]).max(initial=0) < 1e-12 * max(1.0, np.abs(a[fin]).max(initial=0)), (l, key)
        so, wo, _ = o.ext_rows(l)
        sg, wg = s.ext_rows(l)
        assert np.array_equal(so, sg), l
        fin = so[:, 0] >= 0
        assert np.abs(wo[fin] - wg[fin]).max(initial=0) < 1e-12


def test_analytic_levelset_on_device_matches_oracle():
    N = 256
    say(f"[levelset] N={N}")
    mo = wl.Motion(omega=1.0)
    o = O.Oracle(N, Re=400.0)
    phi = O.levelset_analytic(FLOWER.kind, FLOWER.padded(), mo.as_array(), 0.3, N)
    assert o.set_levelset(phi, 0.3, mo.as_array()) == O.OK
    s = gpu_solver(N, Re=400.0)
    s.set_levelset_analytic(FLOWER.kind, FLOWER.params, 0.3, mo.as_array()[:5])
    for l in range(o.nlev):
        assert np.array_equal(o.classes(l), s.classes(l))
    go, gg = o.ghost_rows(0), s.ghost_rows(0)
    rows = go["valid"] >= 0
    assert np.abs(go["w"][rows] - gg["w"][rows]).max() < 1e-9


@pytest.mark.parametrize("shape", [CIRCLE, ELLIPSE])
def test_relaxation_parity(shape):
    N = 64
    say(f"[relax] N={N} shape={shape}")
    o, s = pair(N, shape, 0.64 * (2.0 / N) ** 2, zero_x=False)
    rng = np.random.default_rng(5)
    W = N + 2
    x0 = [rng.standard_normal((W, W)) for _ in range(3)]
    o.set_x(*x0, 0.1)
    s.set_x(*x0, 0.1)
    for side in (o, s):  # wall Dirichlet values from the boundary data
        pass
    bo = o.get_b()
    # put the wall values in x on both sides the way a solve does
    cls = o.classes().ravel()
    xw = flat((*x0, 0.1))
    walld = np.concatenate([cls == O.C_WALLD, [False]])
    xw[walld] = bo[walld]
    o.set_x(xw[:W * W].reshape(W, W), xw[W * W:2 * W * W].reshape(W, W), xw[2 * W * W:3 * W * W].reshape(W, W), 0.1)
    s.set_x(xw[:W * W].reshape(W, W), xw[W * W:2 * W * W].reshape(W, W), xw[2 * W * W:3 * W * W].reshape(W, W), 0.1)
    for steps in (1, 2):
        o.relax(0, 1)
        s.relax(0, 1)
        a, b = flat(o.get_x()), flat(s.get_x())
        act = np.concatenate([active_mask(cls), [True]])
        assert rel_diff(a, b, act) < 1e-11, (steps, rel_diff(a, b, act))


@pytest.mark.parametrize("N,shape", [(32, CIRCLE), (128, ELLIPSE), (256, FLOWER)])
def test_cycle_parity(N, shape):
    say(f"[cycle] N={N} shape={shape}")
    o, s = pair(N, shape, 0.64 * (2.0 / N) ** 2)
    check_cycles(o, s)


# device layouts of the same cycle: levels N <= 32 per level or in one workgroup; the band in one workgroup or
# in device-wide launches
@pytest.mark.parametrize("fuse,split", [(0, 3000), (1, 1), (0, 1)])
def test_cycle_parity_layouts(fuse, split):
    N = 128
    say(f"[cycle layout] N={N} fuse_small_levels={fuse} band_split_min={split}")
    o, s = pair(N, FLOWER, 0.64 * (2.0 / N) ** 2, motion=wl.Motion(omega=1.0), t=0.2, fuse_small_levels=fuse,
                band_split_min=split)
    check_cycles(o, s)


def check_cycles(o, s, cycles=3):
    cls = o.classes().ravel()
    act = np.concatenate([active_mask(cls), [True]])
    for c in range(cycles):
        _, ro = o.cycle()
        rg = s.cycle()
        a, b = flat(o.get_x()), flat(s.get_x())
        d = rel_diff(a, b, act)
        say(f"  cycle {c}: residual oracle {ro:.6e} gpu {rg:.6e}, iterate rel diff {d:.2e}")
        assert d < 1e-11, (c, d)
        # the residual norms relative to each other (they are summed in another order on each side)
        assert abs(ro - rg) <= 1e-8 * ro, (c, ro, rg)


@pytest.mark.parametrize("N", [512, 1024])
def test_band_sectors_against_single_band_layouts(N):
    """The optional extra band relaxation (bnd_sweeps = 1) relaxed over angular sectors (one workgroup each,
    redundant near the sector edges) against the one-workgroup and device-wide layouts: three cycles of the
    rotating flower, same iterates to rounding (the wall ghost rows sum their terms in another order in the
    device-wide layout)."""
    from paper_1911_00994_amd import gpmg
    say(f"[band sectors] N={N}")
    h = 2.0 / N
    mo = wl.Motion(omega=1.0).as_array()
    fu, fv = wl.fourier_forcing(N, 0)
    out = []
    for smin in (1500, 1 << 30):
        s = gpu_solver(N, Re=400.0, band_sector_min=smin, bnd_sweeps=1)
        s.set_levelset_analytic(FLOWER.kind, FLOWER.params, 0.0, mo[:5])
        s.set_alpha(h / 800.0)
        s.set_rhs(fu, fv, None)
        lay = s.band_layout(0)
        # sixteen sectors where the margin allows it (N = 1024), eight otherwise; none when sectors are off
        assert lay["sectors"] == ((16 if N >= 1024 else 8) if smin == 1500 else 0), lay
        res = [s.cycle() for _ in range(3)]
        out.append((flat(s.get_x()), res))
        cls = s.classes().ravel()
        s.close()
    act = np.concatenate([active_mask(cls), [True]])
    d = rel_diff(out[0][0], out[1][0], act)
    say(f"  residuals {out[0][1]} vs {out[1][1]}, rel diff {d:.2e}")
    assert d < 1e-12
    assert np.all(np.isfinite(out[0][0]))


@pytest.mark.parametrize("N,gamma,nu2", [(128, 2, 1), (256, 2, 1)])
def test_w_cycle_parity(N, gamma, nu2):
    """The paper's cycle shape, W(2,1) (Sect. 4.3, Sect. 5.3), colour order, against the oracle"""
    say(f"[W cycle] N={N} gamma={gamma} nu2={nu2}")
    o, s = pair(N, wl.paper_flower(), 0.64 * (2.0 / N) ** 2, gamma=gamma, nu2=nu2)
    check_cycles(o, s)


@pytest.mark.parametrize("N,shape,motion", [(256, FLOWER, wl.Motion(omega=1.0)), (1024, FLOWER, wl.Motion(omega=1.0)),
                                            (128, wl.paper_ellipse(), None)])
def test_coupled_box_table_parity(N, shape, motion):
    """The coupled-box table (cells in visiting order, unknowns, write flags, colour offsets): bit-exact"""
    say(f"[coupled boxes] N={N} shape={shape}")
    # every level builds its table (the default relaxes the coupled boxes on the finest level only)
    o, s = pair(N, shape, 0.64 * (2.0 / N) ** 2, motion=motion, t=0.3, ghost_box_levels=99)
    for lv in range(o.nlev):
        a, b = o.coupled_boxes(lv), s.coupled_boxes(lv)
        for key in ("cell", "off", "idx", "wr", "coff"):
            assert np.array_equal(a[key], b[key]), (lv, key)
    say(f"  level 0: {len(a['cell'])} boxes, {len(a['idx'])} slots")


@pytest.mark.parametrize("N,shape", [(64, CIRCLE), (128, FLOWER)])
def test_converged_solve_parity(N, shape):
    say(f"[solve] N={N} shape={shape}")
    o, s = pair(N, shape, 0.64 * (2.0 / N) ** 2, m=wl.PaperMMS(), t=0.4)
    st_o, so = o.solve(1e-11, 200)
    st_g, sg = s.solve(1e-11, 200)
    assert st_o == O.OK and st_g == 0
    cls = o.classes().ravel()
    act = np.concatenate([active_mask(cls), [True]])
    d = rel_diff(flat(o.get_x()), flat(s.get_x()), act)
    say(f"  cycles oracle {so['cycles']} gpu {sg['cycles']}, rel diff {d:.2e}")
    assert abs(so["cycles"] - sg["cycles"]) <= 1
    assert d < 1e-10


@pytest.mark.parametrize("mixed,split", [(0, 3000), (0, 1), (1, 3000)])
def test_graph_replayed_solve_matches_issued_launches(mixed, split):
    """the solver iterations replayed from a captured HIP graph give the same iterates as launches issued one by
    one (same kernels, same arguments), and the converged solution agrees with the oracle's"""
    from paper_1911_00994_amd import gpmg
    N = 128
    prec = gpmg.GP_MIXED if mixed else gpmg.GP_FP64
    say(f"[graph solve] N={N} mixed={mixed} band_split_min={split}")
    out = []
    for g in (0, 1):
        o, s = pair(N, FLOWER, 0.64 * (2.0 / N) ** 2, m=wl.PaperMMS(), t=0.4, graph_iterations=g,
                    band_split_min=split)
        for rep in range(2):  # the second solve updates the executable graph of the first
            s.set_x(*[np.zeros((N + 2, N + 2))] * 3, 0.0)
            st, info = s.solve(1e-10, 100, precision=prec)
            assert st == 0, info
        out.append((flat(s.get_x()), info["cycles"]))
    assert out[0][1] == out[1][1]
    assert np.array_equal(out[0][0], out[1][0])
    st_o, _ = o.solve(1e-12, 200)
    assert st_o == O.OK
    cls = o.classes().ravel()
    act = np.concatenate([active_mask(cls), [True]])
    assert rel_diff(flat(o.get_x()), out[1][0], act) < 1e-7


@pytest.mark.gpu
def test_queued_first_sweep_gives_the_same_iterates():
    """queuing the next cycle's first box sweep before the host has read the residual norm (its workgroups return
    at once when the solve stops there) leaves the iterates, the cycle counts and the launch probe's count as
    when the host issues that sweep after its test: a solve cut off by max_cycles, the solve that goes on from it
    to convergence, and a solve that starts converged"""
    from paper_1911_00994_amd import gpmg
    N = 256
    say(f"[queued first sweep] N={N}")
    out = []
    for q in (0, 1):
        _, s = pair(N, FLOWER, 0.64 * (2.0 / N) ** 2, m=wl.PaperMMS(), t=0.4, queue_ahead=q)
        s.probe_start(4096)
        rec = []
        for tol, mc in ((1e-10, 3), (1e-10, 100), (1e-10, 100)):
            st, info = s.solve(tol, mc, precision=gpmg.GP_FP64, check=False)
            rec.append((st, info["cycles"], flat(s.get_x())))
        _, n = s.probe_stop()
        out.append((rec, n))
    (r0, n0), (r1, n1) = out
    assert r0[0][0] != 0 and r0[0][1] == 3  # cut off
    assert r0[1][0] == 0 and r0[1][1] > 0 and r0[2][1] == 0
    for a, b in zip(r0, r1):
        assert a[0] == b[0] and a[1] == b[1]
        assert np.array_equal(a[2], b[2])
    assert n0 == n1 == 4 * (r0[0][1] + r0[1][1])  # nu1 + nu2 = 4 finest sweeps per cycle


def _cn_lockstep(o, s, N, shape, motion, m, Re, nsteps, dt):
    """advance oracle and GPU together; both get the boundary data computed from the oracle's geometry"""
    mo = motion.as_array()
    t = 0.0
    xu, yu = wl.node_coords(N, 0)
    xv, yv = wl.node_coords(N, 1)
    xp, yp = wl.node_coords(N, 2)
    out = []
    for _ in range(nsteps):
        t1 = t + dt
        phi = O.levelset_analytic(shape.kind, shape.padded(), mo, t1, N)
        assert o.set_levelset(phi, t1, mo) == O.OK
        s.set_levelset(phi, t1, mo[:5])
        bu, bv, bp = wl.boundary_values_from(m, oracle_geom(o), t1, t + 0.5 * dt, p_scale=dt)
        fu, _ = m.forcing(xu, yu, t + 0.5 * dt, Re)
        _, fv = m.forcing(xv, yv, t + 0.5 * dt, Re)
        g = m.div(xp, yp, t1)
        res = []
        for side in (o, s):
            side.set_boundary_values(bu, bv, bp)
            st, info = side.cn_step(dt, fu, fv, g, tol=1e-12, max_cycles=200)
            assert st == 0, (st, info)
            res.append(flat(side.get_x()))
        out.append(res)
        t = t1
    return out


@pytest.mark.parametrize("N,shape,motion,m,steps", [
    (32, CIRCLE, wl.Motion(), wl.TaylorGreenMMS(), 1),
    (64, ELLIPSE, wl.Motion(U=(0.5, 0.0)), wl.BodyFrameMMS((0.5, 0.0)), 4),
])
def test_cn_step_parity(N, shape, motion, m, steps):
    say(f"[cn] N={N} shape={shape} steps={steps}")
    Re, dt = 100.0, 2.0 / N
    mo = motion.as_array()
    o = O.Oracle(N, Re=Re)
    s = gpu_solver(N, Re=Re)
    phi = O.levelset_analytic(shape.kind, shape.padded(), mo, 0.0, N)
    o.set_levelset(phi, 0.0, mo)
    s.set_levelset(phi, 0.0, mo[:5])
    u0, v0, p0 = wl.mms_fields(m, N, 0.0)
    o.set_state(u0, v0, dt * p0, 0.0)
    s.set_state(u0, v0, dt * p0, 0.0)
    out = _cn_lockstep(o, s, N, shape, motion, m, Re, steps, dt)
    cls = o.classes().ravel()
    act = np.concatenate([active_mask(cls), [True]])
    for k, (a, b) in enumerate(out):
        d = rel_diff(a, b, act)
        say(f"  step {k}: rel diff {d:.2e}")
        assert d < 1e-10, (k, d)


def test_full_size_cycle_parity():
    """The metric workload's geometry at its full size (N = 1024, rotating petal body, Re = 400, dt = h,
    random smooth forcing): three cycles compared element by element with the oracle."""
    N, Re = 1024, 400.0
    say(f"[full-size cycle] N={N}")
    h = 2.0 / N
    alpha = h / (2 * Re)
    mo = wl.Motion(omega=1.0).as_array()
    o = O.Oracle(N, Re=Re)
    phi = O.levelset_analytic(FLOWER.kind, FLOWER.padded(), mo, 0.0, N)
    assert o.set_levelset(phi, 0.0, mo) == O.OK
    o.set_alpha(alpha)
    s = gpu_solver(N, Re=Re)
    s.set_levelset_analytic(FLOWER.kind, FLOWER.params, 0.0, mo[:5])
    s.set_alpha(alpha)
    assert np.array_equal(o.classes(), s.classes())
    fu, fv = wl.fourier_forcing(N, 0)
    for side in (o, s):
        side.set_rhs(fu, fv, None)
    cls = o.classes().ravel()
    act = np.concatenate([active_mask(cls), [True]])
    for c in range(3):
        _, ro = o.cycle()
        rg = s.cycle()
        d = rel_diff(flat(o.get_x()), flat(s.get_x()), act)
        say(f"  cycle {c}: res oracle {ro:.3e} gpu {rg:.3e} rel diff {d:.2e}")
        assert d < 1e-10


@pytest.mark.parametrize("N,shape", [(128, ELLIPSE), (256, FLOWER)])
def test_mixed_precision_solve_against_oracle(N, shape):
    """FP32 cycles inside FP64 iterative refinement: at tolerance 1e-8 the solution differs from the converged
    FP64 oracle solution by no more than the FP64 solver at the same tolerance does, times 10 (stated bound),
    and the FP64 residual meets the tolerance."""
    say(f"[mixed] N={N} shape={shape}")
    from paper_1911_00994_amd import gpmg
    alpha = 0.64 * (2.0 / N) ** 2
    o, s = pair(N, shape, alpha, m=wl.PaperMMS(), t=0.4)
    st_o, _ = o.solve(1e-11, 300)
    assert st_o == O.OK
    xo = flat(o.get_x())
    cls = o.classes().ravel()
    act = np.concatenate([active_mask(cls), [True]])
    W = N + 2
    z = np.zeros((W, W))
    s.set_x(z, z, z, 0.0)
    st64, i64 = s.solve(1e-8, 200, precision=gpmg.GP_FP64)
    e64 = rel_diff(xo, flat(s.get_x()), act)
    s.set_x(z, z, z, 0.0)
    stm, im = s.solve(1e-8, 200, precision=gpmg.GP_MIXED)
    em = rel_diff(xo, flat(s.get_x()), act)
    say(f"  fp64: {i64['cycles']} cycles err {e64:.2e}; mixed: {im['cycles']} cycles err {em:.2e}")
    assert st64 == 0 and stm == 0
    bn = np.abs(o.get_b()).max()
    assert im["res"] <= 1e-8 * max(1.0, bn), im  # the FP64 residual meets the tolerance
    assert em <= 10 * e64 + 1e-10


def test_error_paths_on_the_device():
    """GP_EINVAL for N not a power of two, GP_EGEOM for a body that covers the box walls, GP_EDIVERGED for a NaN
    in the right-hand side (forced from the host; every kernel still runs to completion)"""
    from paper_1911_00994_amd import gpmg
    say("[error paths] N=48, wall body, NaN forcing")
    with pytest.raises(gpmg.GpmgError) as ei:
        gpmg.Solver(48)
    assert ei.value.status == gpmg.GP_EINVAL
    s = gpmg.Solver(32)
    st = s.set_levelset_analytic(wl.CIRCLE_DIST, (1.5,), 0.0, None, check=False)
    assert st == gpmg.GP_EGEOM
    assert s.set_levelset_analytic(wl.CIRCLE_DIST, (0.3,), 0.0, None) == 0
    s.set_alpha(0.64 * (2.0 / 32) ** 2)
    W = 34
    fu = np.zeros((W, W))
    fu[10, 10] = np.nan
    s.set_rhs(fu, np.zeros((W, W)), None)
    st, _ = s.solve(1e-10, 20, check=False)
    assert st == gpmg.GP_EDIVERGED
