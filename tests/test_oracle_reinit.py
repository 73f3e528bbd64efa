"""CPU pins of the oracle's level-set reinitialisation (Sect. 3.1, eq. (sdf)), the step before the solver path for
deforming bodies.  What the mathematics fixes, independent of the oracle's own code:
* a linear level set of any slope and direction is turned into the exact signed distance to its zero line (the
  upwind differences of a linear function are exact, and so is the interface estimate);
* the zero set stays where it was: no lattice value changes sign;
* on a circle, phi = R^2 - r^2, the result approaches the distance R - r: second order at the points next to the
  interface, first order over a band around it.
"""
import numpy as np
import pytest

import oracle as O


def lattice(n, dx, x0=-1.0):
    I, J = np.meshgrid(np.arange(n), np.arange(n))
    return x0 + I * dx, x0 + J * dx


@pytest.mark.parametrize("ang,slope", [(0.0, 3.0), (0.3, 3.0), (0.785398, 0.25), (2.0, 7.0), (4.0, 1.0)])
def test_linear_level_set_becomes_exact_distance(ang, slope):
    n, dx = 81, 0.025
    X, Y = lattice(n, dx)
    nx, ny = np.cos(ang), np.sin(ang)
    dist = nx * X + ny * Y - 0.1
    out = O.reinit(slope * dist, dx, 400)
    # the values at the lattice edges use one-sided data; judge the points whose characteristic (the normal
    # through the point) meets the zero line well inside the lattice
    fx, fy = X - dist * nx, Y - dist * ny
    m = (np.abs(fx) < 0.5) & (np.abs(fy) < 0.5) & (np.abs(dist) < 0.4)
    assert np.abs(out - dist)[m].max() < 1e-11


def test_zero_set_does_not_move():
    n, dx = 129, 1.0 / 64
    X, Y = lattice(n, dx)
    r = np.hypot(X, Y)
    th = np.arctan2(Y, X)
    phi0 = (0.5 + 0.15 * np.sin(5 * th)) ** 2 - r ** 2  # petal body, far from a distance function
    out = O.reinit(phi0, dx, 100)
    assert np.array_equal(np.sign(out), np.sign(phi0))


def test_circle_converges_to_distance():
    near, band = [], []
    for N in (32, 64, 128):
        n, dx = 2 * N + 1, 1.0 / N
        X, Y = lattice(n, dx)
        r = np.hypot(X, Y)
        R = 0.4
        out = O.reinit(R * R - r * r, dx, int(1.0 / (0.3 * dx)))
        e = np.abs(out - (R - r))
        near.append(e[np.abs(r - R) < 2 * dx].max())
        band.append(e[np.abs(r - R) < 0.3].max())
    assert near[0] / near[1] > 3.0 and near[1] / near[2] > 3.0, near
    assert band[0] / band[1] > 1.5 and band[1] / band[2] > 1.5, band
    assert band[-1] < 0.01
