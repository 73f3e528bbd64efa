"""Reverse mode of a run of Crank-Nicolson steps on the HIP path.

The gradient is the derivative of the discrete forward model, so it is checked against central differences of
a forward model: of the oracle's (the plain CPU implementation, independent of the HIP path) on a small grid,
and of the HIP path's own at a larger one.  J = h^2 (sum of u^2 over the internal u points + the same for v) at
the end of the run; parameters: the 64 stream-function forcing coefficients and the offset of the rigid
boundary velocity (body path held fixed).  Every case prints its name before touching the GPU.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1911_00994_amd import workloads as wl

pytestmark = pytest.mark.gpu

CIRCLE = wl.Shape(wl.CIRCLE_DIST, (0.25,))
TOL = 1e-13


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def objective(u, v, cls, h):
    return h * h * (float((u[cls[0] == O.C_INT] ** 2).sum()) + float((v[cls[1] == O.C_INT] ** 2).sum()))


def mode_fields(N, M=8):
    """forcing of each unit stream-function coefficient (the forcing is linear in the coefficients)"""
    out = np.zeros((M, M, 2, N + 2, N + 2))
    for m in range(M):
        for n in range(M):
            e = np.zeros((M, M))
            e[m, n] = 1.0
            out[m, n, 0], out[m, n, 1] = wl.streamfunction_forcing(N, e)
    return out


def gpu_run(N, coeffs, motion, nsteps, ub_offset=None, K=4, Re=100.0, keep=False):
    from paper_1911_00994_amd import gpmg
    h = 2.0 / N
    s = gpmg.Solver(N, Re=Re)
    s.set_levelset_analytic(CIRCLE.kind, CIRCLE.params, 0.0, motion.as_array()[:5])
    W = N + 2
    z = np.zeros((W, W))
    s.set_state(z, z, z, 0.0)
    fu, fv = wl.streamfunction_forcing(N, coeffs)
    s.tape_forward(CIRCLE.kind, CIRCLE.params, motion.as_array(), 0.0, h, nsteps, fu, fv, ub_offset=ub_offset, tol=TOL,
                   max_cycles=200, picard_eps=1e-13, picard_max=40, checkpoint_every=K)
    u, v, _, _ = s.get_x()
    cls = s.classes()
    J = objective(u, v, cls, h)
    return (J, s, u, v, cls) if keep else J


def oracle_run(N, coeffs, motion, nsteps, ub_offset=(0.0, 0.0), Re=100.0):
    h = 2.0 / N
    W = N + 2
    mo = motion.as_array()
    o = O.Oracle(N, Re=Re)
    phi = O.levelset_analytic(CIRCLE.kind, CIRCLE.padded(), mo, 0.0, N)
    assert o.set_levelset(phi, 0.0, mo) == O.OK
    z = np.zeros((W, W))
    assert o.set_state(z, z, z, 0.0) == O.OK
    fu, fv = wl.streamfunction_forcing(N, coeffs)
    for n in range(nsteps):
        t1 = (n + 1) * h
        phi = O.levelset_analytic(CIRCLE.kind, CIRCLE.padded(), mo, t1, N)
        assert o.set_levelset(phi, t1, mo) == O.OK
        if ub_offset[0] or ub_offset[1]:
            b = o.get_b()[:-1].reshape(3, W, W).copy()
            cls = o.classes()
            for g in range(2):
                b[g][cls[g] == O.C_GHOST] += ub_offset[g]
            o.set_boundary_values(b[0], b[1], b[2])
        st, info = o.cn_step(h, fu, fv, None, tol=TOL, max_cycles=300, picard_eps=1e-13, picard_max=40)
        assert st == O.OK, (n, info)
    u, v, _, _ = o.get_x()
    return objective(u, v, o.classes(), h)


def adjoint_gradient(N, coeffs, motion, nsteps, K):
    h = 2.0 / N
    J, s, u, v, cls = gpu_run(N, coeffs, motion, nsteps, K=K, keep=True)
    seed_u = np.where(cls[0] == O.C_INT, 2 * h * h * u, 0.0)
    seed_v = np.where(cls[1] == O.C_INT, 2 * h * h * v, 0.0)
    out = s.tape_backward(seed_u, seed_v, tol=TOL, max_cycles=300)
    modes = mode_fields(N)
    gc = np.einsum("mngij,gij->mn", modes, np.stack([out["dfu"], out["dfv"]]))
    return J, gc, out["dU"], out


def check(fd, ad, what, rtol):
    err = abs(fd - ad) / max(abs(fd), 1e-300)
    say(f"  {what}: fd {fd:.10e} adjoint {ad:.10e} rel {err:.2e}")
    assert err < rtol, (what, fd, ad)


def test_gradient_matches_oracle_finite_differences():
    """N = 32, 5 steps of the circle moving at U = (0.1, 0) (two fixed-point steps, three extrapolated),
    checkpoints every 2 steps: adjoint gradient against central differences of the oracle."""
    N, nsteps, K = 32, 5, 2
    motion = wl.Motion(U=(0.1, 0.0))
    coeffs = wl.adjoint_coeffs(seed=1)
    say(f"[tape vs oracle FD] N={N} steps={nsteps}")
    J, gc, gU, out = adjoint_gradient(N, coeffs, motion, nsteps, K)
    Jo = oracle_run(N, coeffs, motion, nsteps)
    assert abs(J - Jo) < 1e-10 * abs(Jo), (J, Jo)
    rng = np.random.default_rng(4)
    eps = 1e-5
    for trial in range(2):
        e = rng.standard_normal(coeffs.shape)
        fd = (oracle_run(N, coeffs + eps * e, motion, nsteps) - oracle_run(N, coeffs - eps * e, motion, nsteps)) / (2 * eps)
        check(fd, float((gc * e).sum()), f"direction {trial}", 1e-6)
    for comp in range(2):
        off = [0.0, 0.0]
        off[comp] = eps
        offm = [-x for x in off]
        fd = (oracle_run(N, coeffs, motion, nsteps, off) - oracle_run(N, coeffs, motion, nsteps, offm)) / (2 * eps)
        check(fd, float(gU[comp]), f"U offset {comp}", 1e-6)


def test_gradient_matches_gpu_finite_differences():
    """N = 64, 6 steps, checkpoints every 4 (one full and one partial segment): adjoint gradient against
    central differences of the HIP forward model; single forcing modes and the velocity offset."""
    N, nsteps, K = 64, 6, 4
    motion = wl.Motion(U=(0.5, 0.0))
    coeffs = wl.adjoint_coeffs(seed=1)
    say(f"[tape vs GPU FD] N={N} steps={nsteps}")
    J, gc, gU, out = adjoint_gradient(N, coeffs, motion, nsteps, K)
    eps = 1e-5
    for (m, n) in [(0, 0), (2, 5)]:
        e = np.zeros_like(coeffs)
        e[m, n] = 1.0
        fd = (gpu_run(N, coeffs + eps * e, motion, nsteps, K=K) - gpu_run(N, coeffs - eps * e, motion, nsteps, K=K)) / (2 * eps)
        check(fd, float(gc[m, n]), f"mode ({m},{n})", 1e-5)
    fd = (gpu_run(N, coeffs, motion, nsteps, ub_offset=[eps, 0.0], K=K)
          - gpu_run(N, coeffs, motion, nsteps, ub_offset=[-eps, 0.0], K=K)) / (2 * eps)
    check(fd, float(gU[0]), "U offset x", 1e-5)
    # the run is left at its end state
    assert out["stats"]["cycles"] > 0


def test_reverse_pass_is_deterministic():
    """Two identical forward runs and reverse passes give bit-identical gradients (no atomics in the scatters)."""
    N, nsteps, K = 64, 6, 2
    say(f"[tape determinism] N={N} steps={nsteps}")
    coeffs = wl.adjoint_coeffs(seed=1)
    motion = wl.Motion(U=(0.1, 0.0))
    outs = [adjoint_gradient(N, coeffs, motion, nsteps, K) for _ in range(2)]
    assert outs[0][0] == outs[1][0]
    assert np.array_equal(outs[0][1], outs[1][1])
    assert np.array_equal(np.asarray(outs[0][2]), np.asarray(outs[1][2]))


def _geometry_flips(N, motion_a, motion_b, times, eps_scale):
    """discrete decisions of the geometry that differ between two motions at any of the times: classes, or a body
    ghost's boundary point moving by more than eps_scale (a changed Alg. 1 branch moves it by a fixed fraction of h)"""
    from paper_1911_00994_amd import gpmg
    sides = [gpmg.Solver(N, Re=100.0) for _ in range(2)]
    flips = 0
    try:
        for t in times:
            rows = []
            for s, mo in zip(sides, (motion_a, motion_b)):
                s.set_levelset_analytic(CIRCLE.kind, CIRCLE.params, t, mo.as_array()[:5])
                rows.append((s.classes(), s.ghost_rows()))
            if not np.array_equal(rows[0][0], rows[1][0]):
                flips += 1
                continue
            Ba, Bb = rows[0][1]["B"], rows[1][1]["B"]
            m = ~np.isnan(Ba[:, 0])
            flips += int((np.abs(Ba[m] - Bb[m]).max() > eps_scale))
    finally:
        for s in sides:
            s.close()
    return flips


def test_path_gradient_matches_gpu_finite_differences():
    """dJ/dU through the body path (the rows and boundary data of every step's geometry move with X(t) = X0 + U t,
    discrete decisions frozen) plus the direct dependence of u_b on U, against central differences of the HIP
    forward model in the motion's velocity; the difference quotient is taken with a step at which no discrete
    decision of any step's geometry changes (checked)."""
    from paper_1911_00994_amd import gpmg
    N, nsteps, K = 64, 6, 2
    h = 2.0 / N
    coeffs = wl.adjoint_coeffs(seed=1)
    # a velocity whose positions X(t) put no lattice point exactly on the circle (where the classification, and
    # so the derivative, would be one-sided)
    U0 = np.array([0.1137, 0.0471])
    say(f"[path gradient] N={N} steps={nsteps} U={U0}")
    J, s, u, v, cls = gpu_run(N, coeffs, wl.Motion(U=tuple(U0)), nsteps, K=K, keep=True)
    seed_u = np.where(cls[0] == O.C_INT, 2 * h * h * u, 0.0)
    seed_v = np.where(cls[1] == O.C_INT, 2 * h * h * v, 0.0)
    out = s.tape_backward(seed_u, seed_v, tol=TOL, max_cycles=300)
    gpath, unmatched = s.tape_path_gradient()
    s.close()
    assert unmatched == 0
    total = np.asarray(out["dU"]) + gpath
    say(f"  offset part {out['dU']}, path part {gpath}")
    times = [(n + 1) * h for n in range(nsteps)]
    for comp in range(2):
        for eps in (1e-6, 3e-7, 1e-7, 3e-8):
            e = np.zeros(2)
            e[comp] = eps
            mp, mm = wl.Motion(U=tuple(U0 + e)), wl.Motion(U=tuple(U0 - e))
            if _geometry_flips(N, mp, mm, times, 1e3 * eps):
                say(f"  component {comp}: eps {eps:.0e} changes a discrete decision, smaller step")
                continue
            fd = (gpu_run(N, coeffs, mp, nsteps, K=K) - gpu_run(N, coeffs, mm, nsteps, K=K)) / (2 * eps)
            check(fd, float(total[comp]), f"dJ/dU_{comp} (path + direct)", 1e-5 if eps >= 1e-7 else 1e-4)
            break
        else:
            pytest.fail("every step size changed a discrete decision")
