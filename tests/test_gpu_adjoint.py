"""Transposed system on the HIP path: M^T lam against the oracle's assembled matrix, the transposed cycle
against the forward cycle (dot-product identity), and the transposed solve against a direct sparse solve of
the oracle's M^T.  Every case prints its name before touching the GPU.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1911_00994_amd import workloads as wl
from tests.test_gpu_parity import CIRCLE, ELLIPSE, FLOWER, pair

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def unknown_mask(o):
    cls = o.classes().ravel()
    m = (cls == O.C_INT) | (cls == O.C_GHOST) | (cls == O.C_GHOSTX) | (cls == O.C_WALLG) | (cls == O.C_WALLD)
    return np.concatenate([m, [True]])


CASES = [(32, CIRCLE, None), (64, FLOWER, wl.Motion(omega=1.0)), (64, ELLIPSE, wl.Motion(U=(0.5, 0.0)))]


@pytest.mark.parametrize("N,shape,motion", CASES)
def test_transposed_matvec_matches_oracle_matrix(N, shape, motion):
    say(f"[M^T] N={N} shape={shape}")
    o, s = pair(N, shape, 0.64 * (2.0 / N) ** 2, motion=motion, t=0.2)
    A, _ = o.csr()
    m = unknown_mask(o)
    rng = np.random.default_rng(11)
    lam = rng.standard_normal(m.size) * m
    y_ref = A.T @ lam
    y = s.apply_mt(lam)
    err = np.abs(y - y_ref)[m].max() / np.abs(y_ref[m]).max()
    assert err < 1e-13, err


@pytest.mark.parametrize("N,shape,motion", CASES + [(128, wl.paper_flower(), wl.Motion(omega=1.0))])
def test_transposed_cycle_dot_product(N, shape, motion):
    """<y, B' b> = <B'^T y, b> for random b and y: every step of the cycle is transposed exactly."""
    say(f"[B'^T] N={N} shape={shape}")
    _, s = pair(N, shape, 0.64 * (2.0 / N) ** 2, motion=motion, t=0.2)
    n = s.nvec()
    rng = np.random.default_rng(3)
    for trial in range(2):
        b = rng.standard_normal(n)
        y = rng.standard_normal(n)
        Bb = s.apply_cycle(b)
        Bty = s.apply_cycle_t(y)
        lhs, rhs = float(y @ Bb), float(Bty @ b)
        scale = np.abs(y).sum() * np.abs(Bb).max() + np.abs(Bty).max() * np.abs(b).sum()
        assert abs(lhs - rhs) < 1e-13 * scale, (trial, lhs, rhs)


@pytest.mark.parametrize("N,shape,motion", CASES)
def test_adjoint_solve_matches_direct_solve(N, shape, motion):
    import scipy.sparse.linalg as spla
    say(f"[adjoint solve] N={N} shape={shape}")
    o, s = pair(N, shape, 0.64 * (2.0 / N) ** 2, motion=motion, t=0.2)
    A, _ = o.csr()
    m = unknown_mask(o)
    rng = np.random.default_rng(21)
    g = rng.standard_normal(m.size) * m
    lam_ref = spla.spsolve(A.T.tocsc(), g)
    lam, st, info = s.adjoint_solve(g, tol=1e-12, max_cycles=200)
    assert st == 0, info
    err = np.abs(lam - lam_ref)[m].max() / np.abs(lam_ref[m]).max()
    assert err < 1e-9, (err, info)
    # the transposed iteration contracts like the forward one
    assert info["rho"] < 0.6, info


@pytest.mark.parametrize("N,shape,motion", [(128, wl.paper_flower(), wl.Motion(omega=1.0)),
                                            (64, ELLIPSE, wl.Motion(U=(0.5, 0.0)))])
def test_transposed_cycle_and_solve_are_deterministic(N, shape, motion):
    """The transposed scatters are gathers in a fixed order (entries keyed by their points, not by the numbering a
    geometry build gave the rows): repeated applications, and two contexts built from the same geometry, give
    bit-identical results."""
    say(f"[determinism] N={N} shape={shape}")
    o, s = pair(N, shape, 0.64 * (2.0 / N) ** 2, motion=motion, t=0.2)
    _, s2 = pair(N, shape, 0.64 * (2.0 / N) ** 2, motion=motion, t=0.2)
    n = s.nvec()
    rng = np.random.default_rng(5)
    y = rng.standard_normal(n)
    a = [s.apply_cycle_t(y) for _ in range(2)] + [s2.apply_cycle_t(y)]
    assert all(np.array_equal(a[0], x) for x in a[1:]), [int((a[0] != x).sum()) for x in a[1:]]
    m = unknown_mask(o)
    g = rng.standard_normal(m.size) * m
    sols = [side.adjoint_solve(g, tol=1e-12, max_cycles=200) for side in (s, s, s2)]
    assert all(q[1] == 0 for q in sols)
    assert all(np.array_equal(sols[0][0], q[0]) for q in sols[1:])
    assert all(sols[0][2]["cycles"] == q[2]["cycles"] for q in sols[1:])


def test_adjoint_after_alpha_change_matches_fresh_context():
    """What the transposed cycle keeps per geometry and alpha (the coefficients of the coupled-box tables, the
    coupled-box and coarsest inverses) follows a change of alpha: a context that solved at alpha1 and then at
    alpha2 gives, bit for bit, the result of a context built at alpha2."""
    N, shape, motion = 128, wl.paper_flower(), wl.Motion(omega=1.0)
    a1 = 0.64 * (2.0 / N) ** 2
    a2 = 2.5 * a1
    say(f"[alpha change] N={N} alpha {a1:.3e} -> {a2:.3e}")
    o, s = pair(N, shape, a1, motion=motion, t=0.2)
    _, s2 = pair(N, shape, a2, motion=motion, t=0.2)
    m = unknown_mask(o)
    rng = np.random.default_rng(9)
    g = rng.standard_normal(m.size) * m
    _, st0, _ = s.adjoint_solve(g, tol=1e-12, max_cycles=200)
    s.set_alpha(a2)
    lam1, st1, info1 = s.adjoint_solve(g, tol=1e-12, max_cycles=200)
    lam2, st2, info2 = s2.adjoint_solve(g, tol=1e-12, max_cycles=200)
    assert st0 == st1 == st2 == 0
    assert info1["cycles"] == info2["cycles"], (info1, info2)
    assert np.array_equal(lam1, lam2), int((lam1 != lam2).sum())
