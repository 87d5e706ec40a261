"""Pins of the oracle's velocities and explicit-midpoint step against what
the mathematics fixes (Sec. 2.1: velocity is the curl of the
streamfunction, taken on the faces and averaged to the nodes, then
interpolated to the vortices by the transpose of the regularization).

* Centred differences are exact for quadratic streamfunctions and M4'
  reproduces linear fields, so the whole velocity chain is exact for them:
  a transposed, sign-flipped or mis-scaled (u, v) fails.
* One vortex induces at another, distance d away, the Biot-Savart velocity
  Gamma/(2 pi d) along the counter-clockwise perpendicular; the lattice
  gives it to second order in dx/d.
* A co-rotating pair of equal vortices keeps its centroid; one midpoint
  step equals the midpoint rule applied with the exact point-vortex
  velocities up to the (second-order) velocity error, far below the
  difference to forward Euler or to a wrong half-step.
"""
import numpy as np
import pytest

from oracle.operators import (Grid, inv_laplacian_fft, node_velocity, regularize_vortices,
                              vortex_velocity)
from oracle.solve import Problem, rk2_step


def _biot_savart(xt, yt, xs, ys, g):
    """Velocity at (xt, yt) of a point vortex of strength g at (xs, ys):
    psi = -g/(2 pi) ln r, u = dpsi/dy, v = -dpsi/dx."""
    rx, ry = xt - xs, yt - ys
    r2 = rx * rx + ry * ry
    return -g / (2 * np.pi) * ry / r2, g / (2 * np.pi) * rx / r2


def test_node_velocity_exact_for_quadratic_streamfunction():
    n, dx = 24, 0.07
    grid = Grid.centered(n, dx)
    X, Y = np.meshgrid(grid.node_x(), grid.node_y())
    p, q, r, a, b = 0.3, -1.1, 0.45, 0.8, -0.6
    psi = p * X * X + q * X * Y + r * Y * Y + a * Y - b * X
    u, v = node_velocity(psi, dx)
    ue = q * X + 2 * r * Y + a            # dpsi/dy
    ve = -(2 * p * X + q * Y - b)         # -dpsi/dx
    assert np.max(np.abs(u[1:-1, :] - ue[1:-1, :])) < 1e-12
    assert np.max(np.abs(v[:, 1:-1] - ve[:, 1:-1])) < 1e-12
    # edge rows/columns carry no centred difference
    assert np.all(np.isnan(u[0, :])) and np.all(np.isnan(v[:, -1]))


def test_vortex_velocity_exact_for_quadratic_streamfunction():
    rng = np.random.default_rng(11)
    n, dx = 40, 0.05
    grid = Grid.centered(n, dx)
    X, Y = np.meshgrid(grid.node_x(), grid.node_y())
    p, q, r, a, b = -0.7, 0.25, 1.3, 0.1, 0.9
    psi = p * X * X + q * X * Y + r * Y * Y + a * Y - b * X
    h = (n - 1) * dx / 2 - 4 * dx
    xq, yq = rng.uniform(-h, h, 37), rng.uniform(-h, h, 37)
    uinf, vinf = 0.4, -0.3
    u, v = vortex_velocity(grid, psi, xq, yq, uinf, vinf)
    assert np.max(np.abs(u - (q * xq + 2 * r * yq + a + uinf))) < 1e-12
    assert np.max(np.abs(v - (-(2 * p * xq + q * yq - b) + vinf))) < 1e-12


@pytest.mark.parametrize("angle_deg", [0.0, 30.0, 137.0, 250.0])
def test_two_vortex_velocity_is_biot_savart(angle_deg):
    """Vortex 1 (zero strength, on a node) sees vortex 2 at distance d:
    the discrete velocity has the Biot-Savart direction and magnitude to
    second order: its error falls ~16-fold when d/dx grows four-fold."""
    n, dx = 128, 0.02
    grid = Grid.centered(n, dx)
    ang = np.deg2rad(angle_deg)
    x1, y1 = grid.x0 + 62 * dx, grid.y0 + 60 * dx
    errs = []
    for cells in (8, 16, 32):
        d = cells * dx
        x2, y2 = x1 + d * np.cos(ang), y1 + d * np.sin(ang)
        g2 = 0.7
        w = regularize_vortices(grid, [x1, x2], [y1, y2], [0.0, g2])
        s = inv_laplacian_fft(w, dx)
        u, v = vortex_velocity(grid, s, [x1], [y1])
        ue, ve = _biot_savart(x1, y1, x2, y2, g2)
        mag = np.hypot(ue, ve)
        assert abs(mag - g2 / (2 * np.pi * d)) < 1e-12 * mag
        err = np.hypot(u[0] - ue, v[0] - ve) / mag
        # measured constant 0.06-0.52 over directions (the lattice far
        # field's cos 4 theta term and the central differences)
        assert err <= 0.6 * (dx / d) ** 2, (cells, err)
        # the velocity is perpendicular to the separation, counter-clockwise
        cross = (x1 - x2) * v[0] - (y1 - y2) * u[0]
        assert cross > 0
        errs.append(err)
    assert errs[0] / errs[2] > 8.0     # 16 for exact second order


@pytest.mark.parametrize("cells,h", [(16, 0.2), (32, 0.2), (32, 0.1)])
def test_rk2_step_co_rotating_pair(cells, h):
    """Equal vortices +-d/2 about a node rotate at Omega = Gamma/(pi d^2).
    One oracle midpoint step with h = Omega dt: the centroid stays put to
    rounding, and the positions equal the midpoint rule with exact
    point-vortex velocities within dt U (dx/d)^2 (measured constant 0.45),
    which is at least 20x below the gap to forward Euler (h/2 dt U) or to
    a full first stage."""
    n, dx, g = 128, 0.02, 0.5
    grid = Grid.centered(n, dx)
    d = cells * dx
    xc, yc = grid.x0 + 64 * dx, grid.y0 + 64 * dx
    X = np.array([xc - d / 2, xc + d / 2])
    Y = np.array([yc, yc])
    om = g / (np.pi * d * d)
    dt = h / om
    U = g / (2 * np.pi * d)
    p = Problem(grid=grid, X=X, Y=Y, G=np.array([g, g]), mode="none")
    Xn, Yn, r1, r2 = rk2_step(p, None, dt)

    assert abs(Xn.mean() - xc) < 1e-14 and abs(Yn.mean() - yc) < 1e-14

    def vel(XX, YY):
        u0, v0 = _biot_savart(XX[0], YY[0], XX[1], YY[1], g)
        u1, v1 = _biot_savart(XX[1], YY[1], XX[0], YY[0], g)
        return np.array([u0, u1]), np.array([v0, v1])

    u, v = vel(X, Y)
    um, vm = vel(X + 0.5 * dt * u, Y + 0.5 * dt * v)
    Xe, Ye = X + dt * um, Y + dt * vm
    tol = 0.6 * dt * U * (dx / d) ** 2
    assert np.max(np.hypot(Xn - Xe, Yn - Ye)) <= tol

    # the tolerance separates the wrong schemes by a wide margin
    euler = np.max(np.hypot(X + dt * u - Xe, Y + dt * v - Ye))
    uf, vf = vel(X + dt * u, Y + dt * v)
    full_stage = np.max(np.hypot(X + dt * uf - Xe, Y + dt * vf - Ye))
    assert euler > 20 * tol and full_stage > 20 * tol

    # the first stage is the velocity at the start, the second at the midpoint
    assert np.max(np.hypot(r1.u - u, r1.v - v)) <= 0.6 * U * (dx / d) ** 2
    assert np.max(np.hypot(r2.u - um, r2.v - vm)) <= 0.6 * U * (dx / d) ** 2
    # counter-clockwise rotation by Omega dt, to the midpoint rule's third order
    a0 = np.arctan2(Y[1] - yc, X[1] - xc)
    a1 = np.arctan2(Yn[1] - yc, Xn[1] - xc)
    assert abs((a1 - a0) - h) <= h ** 3 / 6 * 1.05 + 0.6 * h * (dx / d) ** 2
