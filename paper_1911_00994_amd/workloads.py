"""Seeded synthetic workloads: body shapes, rigid motions, forcing fields and manufactured solutions.

This module holds the *problem data* of the test and benchmark workloads -- analytic fields evaluated
at grid nodes, seeded random coefficients -- and none of the solver's arithmetic.  Both the oracle
tests and the GPU path take their inputs from here.

Grid conventions (shared by every array of the library): N cells per side on D = (-1, 1)^2, h = 2/N,
arrays of shape (N+2, N+2) indexed [j+1, i+1] for i, j in [-1, N]:
  u[i, j] at (x, y) = (-1 + i h,        -1 + (j + 1/2) h)   (vertical cell faces)
  v[i, j] at (x, y) = (-1 + (i + 1/2) h, -1 + j h)          (horizontal cell faces)
  p[i, j] at (x, y) = (-1 + (i + 1/2) h, -1 + (j + 1/2) h)  (cell centres)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# shape kinds understood by the level-set samplers (phi > 0 inside the body)
CIRCLE_DIST = 0     # R - r
CIRCLE_QUAD = 1     # R^2 - r^2                         (paper, eq. domains)
ELLIPSE_QUAD = 2    # 1 - (x'^2/A^2 + y'^2/B^2)         (paper, eq. domains)
ELLIPSE_SQRT = 3    # 1 - sqrt(x'^2/A^2 + y'^2/B^2)
PETALS = 4          # A + B cos(m (theta - theta0)) - r (paper flower with theta0 = pi/10, m = 5)
NO_BODY = 5


@dataclass
class Shape:
    kind: int
    params: tuple = (0.0, 0.0, 0.0, 0.0)

    def padded(self):
        return tuple(list(self.params) + [0.0] * (4 - len(self.params)))


@dataclass
class Motion:
    """Rigid motion: body frame point = R(-omega t) (x - X0 - U t)."""
    X0: tuple = (0.0, 0.0)
    U: tuple = (0.0, 0.0)
    omega: float = 0.0

    def as_array(self):
        return np.array([self.X0[0], self.X0[1], self.U[0], self.U[1], self.omega, 0.0])

    def velocity(self, x, y, t):
        X = self.X0[0] + self.U[0] * t
        Y = self.X0[1] + self.U[1] * t
        return self.U[0] - self.omega * (y - Y), self.U[1] + self.omega * (x - X)


# paper shapes (eq. domains)
def paper_circle():
    return Shape(CIRCLE_QUAD, (1.0 / math.sqrt(15.0), 0.0, 0.0, 0.0))


def paper_ellipse():
    return Shape(ELLIPSE_QUAD, (1.0 / math.sqrt(14.0), 1.0 / math.sqrt(2.0), math.pi / 6.0, 0.0))


def paper_flower():
    # Im((x+iy)^5)/r^5 = sin(5 theta) = cos(5 (theta - pi/10)); sign chosen so that phi > 0 inside
    return Shape(PETALS, (0.5, 0.15, math.pi / 10.0, 5.0))


def node_coords(N: int, grid: int):
    """x, y arrays of shape (N+2, N+2) for grid 0 (u), 1 (v), 2 (p)."""
    h = 2.0 / N
    idx = np.arange(-1, N + 1, dtype=np.float64)
    I, J = np.meshgrid(idx, idx)  # [j+1, i+1]
    if grid == 0:
        return -1.0 + I * h, -1.0 + (J + 0.5) * h
    if grid == 1:
        return -1.0 + (I + 0.5) * h, -1.0 + J * h
    return -1.0 + (I + 0.5) * h, -1.0 + (J + 0.5) * h


# ------------------------------------------------------------------------------------------------
# manufactured solutions
# ------------------------------------------------------------------------------------------------
class MMS:
    """Base class: exact u, v, p and the forcing of eq. (NSeq) that they satisfy."""

    def u(self, x, y, t):
        raise NotImplementedError

    def v(self, x, y, t):
        raise NotImplementedError

    def p(self, x, y, t):
        raise NotImplementedError

    def grad(self, f, x, y, t, eps=1e-5):
        return ((f(x + eps, y, t) - f(x - eps, y, t)) / (2 * eps), (f(x, y + eps, t) - f(x, y - eps, t)) / (2 * eps))

    # subclasses provide exact derivatives where convenient; defaults use them
    def forcing(self, x, y, t, Re):
        raise NotImplementedError

    def div(self, x, y, t):
        raise NotImplementedError

    def dpdn(self, x, y, t, nx, ny):
        gx, gy = self.p_grad(x, y, t)
        return gx * nx + gy * ny


class TaylorGreenMMS(MMS):
    """u = sin(pi x) cos(pi y) c(t), v = -cos(pi x) sin(pi y) c(t), p = cos(pi x) cos(pi y) s(t);
    divergence free; c = cos t, s = sin t."""

    def __init__(self, amp=1.0):
        self.A = amp

    def u(self, x, y, t):
        return self.A * np.sin(np.pi * x) * np.cos(np.pi * y) * np.cos(t)

    def v(self, x, y, t):
        return -self.A * np.cos(np.pi * x) * np.sin(np.pi * y) * np.cos(t)

    def p(self, x, y, t):
        return np.cos(np.pi * x) * np.cos(np.pi * y) * np.sin(t)

    def p_grad(self, x, y, t):
        return (-np.pi * np.sin(np.pi * x) * np.cos(np.pi * y) * np.sin(t),
                -np.pi * np.cos(np.pi * x) * np.sin(np.pi * y) * np.sin(t))

    def div(self, x, y, t):
        return np.zeros_like(np.asarray(x, dtype=np.float64) + np.asarray(y, dtype=np.float64))

    def forcing(self, x, y, t, Re):
        A, pi = self.A, np.pi
        sx, cx, sy, cy = np.sin(pi * x), np.cos(pi * x), np.sin(pi * y), np.cos(pi * y)
        u = A * sx * cy * np.cos(t)
        v = -A * cx * sy * np.cos(t)
        ut = -A * sx * cy * np.sin(t)
        vt = A * cx * sy * np.sin(t)
        ux = A * pi * cx * cy * np.cos(t)
        uy = -A * pi * sx * sy * np.cos(t)
        vx = A * pi * sx * sy * np.cos(t)
        vy = -A * pi * cx * cy * np.cos(t)
        lapu = -2 * pi * pi * u
        lapv = -2 * pi * pi * v
        px, py = self.p_grad(x, y, t)
        fu = ut + u * ux + v * uy + px - lapu / Re
        fv = vt + u * vx + v * vy + py - lapv / Re
        return fu, fv


class PaperMMS(MMS):
    """Exact solution of eq. (sol:exa); not divergence free, so the continuity equation carries
    g = div u_exa."""

    def u(self, x, y, t):
        return np.cos(5 * x) * np.cos(6 * y * np.log(t + 2))

    def v(self, x, y, t):
        return np.sin(4 * t) * np.sin(3 * x * x + 4 * y * y + 2)

    def p(self, x, y, t):
        return np.cos(6 * x * t) * np.sin(2 * y * t) * np.log(3 * t + 1) + np.sin(5 * t)

    def p_grad(self, x, y, t):
        L = np.log(3 * t + 1)
        return (-6 * t * np.sin(6 * x * t) * np.sin(2 * y * t) * L, 2 * t * np.cos(6 * x * t) * np.cos(2 * y * t) * L)

    def div(self, x, y, t):
        lg = np.log(t + 2)
        ux = -5 * np.sin(5 * x) * np.cos(6 * y * lg)
        vy = np.sin(4 * t) * np.cos(3 * x * x + 4 * y * y + 2) * 8 * y
        return ux + vy

    def forcing(self, x, y, t, Re):
        lg = np.log(t + 2)
        c5, s5 = np.cos(5 * x), np.sin(5 * x)
        a = 6 * y * lg
        ca, sa = np.cos(a), np.sin(a)
        u = c5 * ca
        ut = c5 * (-sa) * 6 * y / (t + 2)
        ux = -5 * s5 * ca
        uy = c5 * (-sa) * 6 * lg
        uxx = -25 * c5 * ca
        uyy = -c5 * ca * 36 * lg * lg
        q = 3 * x * x + 4 * y * y + 2
        s4, c4 = np.sin(4 * t), np.cos(4 * t)
        sq, cq = np.sin(q), np.cos(q)
        v = s4 * sq
        vt = 4 * c4 * sq
        vx = s4 * cq * 6 * x
        vy = s4 * cq * 8 * y
        vxx = s4 * (-sq * 36 * x * x + cq * 6)
        vyy = s4 * (-sq * 64 * y * y + cq * 8)
        px, py = self.p_grad(x, y, t)
        fu = ut + u * ux + v * uy + px - (uxx + uyy) / Re
        fv = vt + u * vx + v * vy + py - (vxx + vyy) / Re
        return fu, fv


class BodyFrameMMS(MMS):
    """Translating-body manufactured flow: u = U + W(x - U t, y), with W the Taylor-Green velocity at
    t = 0, and p = cos(pi (x - Ux t)) cos(pi y).  Steady in the body frame."""

    def __init__(self, U=(0.5, 0.0), amp=1.0):
        self.U = U
        self.A = amp

    def _xb(self, x, t):
        return x - self.U[0] * t

    def _yb(self, y, t):
        return y - self.U[1] * t

    def u(self, x, y, t):
        return self.U[0] + self.A * np.sin(np.pi * self._xb(x, t)) * np.cos(np.pi * self._yb(y, t))

    def v(self, x, y, t):
        return self.U[1] - self.A * np.cos(np.pi * self._xb(x, t)) * np.sin(np.pi * self._yb(y, t))

    def p(self, x, y, t):
        return np.cos(np.pi * self._xb(x, t)) * np.cos(np.pi * self._yb(y, t))

    def p_grad(self, x, y, t):
        X, Y = self._xb(x, t), self._yb(y, t)
        return -np.pi * np.sin(np.pi * X) * np.cos(np.pi * Y), -np.pi * np.cos(np.pi * X) * np.sin(np.pi * Y)

    def div(self, x, y, t):
        return np.zeros_like(np.asarray(x, dtype=np.float64) + np.asarray(y, dtype=np.float64))

    def forcing(self, x, y, t, Re):
        A, pi = self.A, np.pi
        X, Y = self._xb(x, t), self._yb(y, t)
        sx, cx, sy, cy = np.sin(pi * X), np.cos(pi * X), np.sin(pi * Y), np.cos(pi * Y)
        u = self.U[0] + A * sx * cy
        v = self.U[1] - A * cx * sy
        wx_u = A * pi * cx * cy   # d/dX of the u perturbation
        wy_u = -A * pi * sx * sy
        wx_v = A * pi * sx * sy
        wy_v = -A * pi * cx * cy
        ut = -self.U[0] * wx_u - self.U[1] * wy_u
        vt = -self.U[0] * wx_v - self.U[1] * wy_v
        lapu = -2 * pi * pi * A * sx * cy
        lapv = 2 * pi * pi * A * cx * sy
        px, py = self.p_grad(x, y, t)
        fu = ut + u * wx_u + v * wy_u + px - lapu / Re
        fv = vt + u * wx_v + v * wy_v + py - lapv / Re
        return fu, fv


# ------------------------------------------------------------------------------------------------
# grid fields of a manufactured solution
# ------------------------------------------------------------------------------------------------
def mms_fields(m: MMS, N: int, t: float):
    xu, yu = node_coords(N, 0)
    xv, yv = node_coords(N, 1)
    xp, yp = node_coords(N, 2)
    return m.u(xu, yu, t), m.v(xv, yv, t), m.p(xp, yp, t)


def mms_linear_rhs(m: MMS, N: int, t: float, alpha: float):
    """Right-hand side of the space problem eq. (spaceprobaug) that the exact fields satisfy:
    f^u = u - alpha lap u + dp/dx, f^v likewise, g = div u (continuous operators at the nodes)."""
    xu, yu = node_coords(N, 0)
    xv, yv = node_coords(N, 1)
    xp, yp = node_coords(N, 2)
    e = 1e-4

    def lap(f, x, y):
        return (f(x + e, y, t) + f(x - e, y, t) + f(x, y + e, t) + f(x, y - e, t) - 4 * f(x, y, t)) / (e * e)

    # exact Laplacians from the forcing decomposition are not available generically; a 4th-order
    # accurate finite difference with e = 1e-4 is far below the O(h^2) discretisation error
    def lap4(f, x, y):
        e2 = 1e-3
        def d2(g):
            return (-g(2) + 16 * g(1) - 30 * g(0) + 16 * g(-1) - g(-2)) / (12 * e2 * e2)
        return d2(lambda k: f(x + k * e2, y, t)) + d2(lambda k: f(x, y + k * e2, t))

    px_u, _ = m.p_grad(xu, yu, t)
    _, py_v = m.p_grad(xv, yv, t)
    fu = m.u(xu, yu, t) - alpha * lap4(m.u, xu, yu) + px_u
    fv = m.v(xv, yv, t) - alpha * lap4(m.v, xv, yv) + py_v
    g = m.div(xp, yp, t)
    del lap
    return fu, fv, g


def boundary_values_from(m: MMS, geom: dict, t_vel: float, t_p: float, p_scale: float = 1.0):
    """Boundary data arrays (u, v, p grids) from boundary points and normals:
    velocity rows take u_exa(B), pressure rows take p_scale * dp_exa/dn(B)."""
    Bu, Bv, Bp = geom["B"]  # each (N+2, N+2, 2), NaN where no boundary row
    nBp = geom["nB"][2]
    bu = np.nan_to_num(m.u(Bu[..., 0], Bu[..., 1], t_vel))
    bv = np.nan_to_num(m.v(Bv[..., 0], Bv[..., 1], t_vel))
    gx, gy = m.p_grad(Bp[..., 0], Bp[..., 1], t_p)
    bp = np.nan_to_num(p_scale * (gx * nBp[..., 0] + gy * nBp[..., 1]))
    return bu, bv, bp


# ------------------------------------------------------------------------------------------------
# random smooth forcing
# ------------------------------------------------------------------------------------------------
def fourier_forcing(N: int, seed: int = 0, modes: int = 10, kmax: int = 4):
    """f = sum_k a_k cos(pi (m_k x + n_k y) + phase_k) per component, (m, n) uniform in {1..kmax}^2,
    phases uniform in [0, 2 pi), coefficients uniform in [-1, 1]; each component rescaled so that its
    maximum modulus on its grid is 1."""
    rng = np.random.default_rng(seed)
    out = []
    for grid in (0, 1):
        mn = rng.integers(1, kmax + 1, size=(modes, 2))
        ph = rng.uniform(0.0, 2 * np.pi, size=modes)
        a = rng.uniform(-1.0, 1.0, size=modes)
        x, y = node_coords(N, grid)
        f = np.zeros_like(x)
        for k in range(modes):
            f += a[k] * np.cos(np.pi * (mn[k, 0] * x + mn[k, 1] * y) + ph[k])
        out.append(f / np.abs(f).max())
    return out[0], out[1]


def streamfunction_forcing(N: int, coeffs: np.ndarray):
    """Divergence-free forcing from psi = sum c_mn sin(m pi (x+1)/2) sin(n pi (y+1)/2):
    f = (dpsi/dy, -dpsi/dx)."""
    M = coeffs.shape[0]
    res = []
    for grid in (0, 1):
        x, y = node_coords(N, grid)
        f = np.zeros_like(x)
        for m in range(1, M + 1):
            for n in range(1, coeffs.shape[1] + 1):
                c = coeffs[m - 1, n - 1]
                a, b = m * np.pi / 2, n * np.pi / 2
                if grid == 0:
                    f += c * np.sin(a * (x + 1)) * b * np.cos(b * (y + 1))
                else:
                    f += -c * a * np.cos(a * (x + 1)) * np.sin(b * (y + 1))
        res.append(f)
    return res[0], res[1]


def adjoint_coeffs(seed: int = 1, M: int = 8):
    rng = np.random.default_rng(seed)
    m = np.arange(1, M + 1)[:, None]
    n = np.arange(1, M + 1)[None, :]
    return rng.standard_normal((M, M)) / (m * m + n * n)


# ------------------------------------------------------------------------------------------------
# named workloads
# ------------------------------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    N: int
    Re: float
    shape: Shape
    motion: Motion = field(default_factory=Motion)
    steps: int = 1
    walls: tuple = (0.0,) * 8  # bottom u,v  right u,v  top u,v  left u,v

    @property
    def h(self):
        return 2.0 / self.N


def config_circle32():
    """Single CN step, N = 32, fixed circle phi = 0.3 - r, Re = 100, dt = h, Taylor-Green MMS."""
    return Workload("circle-32-fixed-mms", 32, 100.0, Shape(CIRCLE_DIST, (0.3,)))


def config_ellipse256():
    """N = 256, ellipse phi = 1 - sqrt((x/0.4)^2 + (y/0.2)^2) translating at (0.5, 0), Re = 100,
    50 steps of dt = h, body-frame MMS."""
    return Workload("ellipse-256-translating-mms", 256, 100.0, Shape(ELLIPSE_SQRT, (0.4, 0.2, 0.0)),
                    Motion(U=(0.5, 0.0)), steps=50)


def config_flower1024():
    """N = 1024, petal body r = 0.35 (1 + 0.2 cos 5 theta) rotating at omega = 1, Re = 400,
    20 steps of dt = h, random smooth forcing (10 Fourier modes)."""
    return Workload("flower-1024-rotating", 1024, 400.0, Shape(PETALS, (0.35, 0.07, 0.0, 5.0)),
                    Motion(omega=1.0), steps=20)


def config_cavity2048():
    """N = 2048 lid-driven cavity (top lid u = 1) around a fixed circle r = 0.2, Re = 1000, 200 steps."""
    return Workload("cavity-2048-circle", 2048, 1000.0, Shape(CIRCLE_DIST, (0.2,)), steps=200,
                    walls=(0.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0))


def config_circle512_adjoint():
    """N = 512, circle r = 0.25 moving at (0.5, 0), Re = 100, 40 steps."""
    return Workload("circle-512-moving-adjoint", 512, 100.0, Shape(CIRCLE_DIST, (0.25,)), Motion(U=(0.5, 0.0)),
                    steps=40)
