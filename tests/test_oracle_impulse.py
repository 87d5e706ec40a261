"""Pins of the oracle's impulse, added mass and geometry (Sec. 2.6.2-2.6.3,
appendix on discrete surfaces).

* node impulse of regularized vortices equals the point-vortex sums exactly
  (the M4' kernel reproduces polynomials up to degree two);
* classical translational added masses, approached at first order in dx:
  circular cylinder rho pi a^2 on each axis, ellipse rho pi b^2 / rho pi a^2
  along its axes, flat plate rho pi c^2 / 4 normal to it and none along it;
  the circle's rotation entry against the closed form of the discrete
  formula;
* vortices outside a cylinder at rest: the impulse of the vortices and
  their images, sum Gamma (1 - a^2 / r^2) (y, -x);
* a cylinder at rest in a uniform flow carries the impulse -pi a^2 U of a
  cylinder moving at -U through fluid at rest (body-motion term);
* with zero total circulation the impulse does not change when the whole
  configuration moves by whole cells (relative sign of fluid and sheet terms);
* area and centroid of a shifted circle and of an ellipse.
"""
import numpy as np
import pytest

from oracle.impulse import added_mass, impulse, node_impulse, solution_impulse, volume_centroid
from oracle.operators import Grid, regularize_vortices
from oracle.solve import Problem, solve
from paper_2102_11910_amd import workloads as wl
from tests.oracle_adapter import body_of, problem_of


def test_node_impulse_equals_vortex_sums():
    rng = np.random.default_rng(5)
    grid = Grid.centered(64, 0.05)
    X, Y = rng.uniform(-1.3, 1.3, 50), rng.uniform(-1.3, 1.3, 50)
    G = rng.normal(0, 1, 50)
    P = node_impulse(grid, regularize_vortices(grid, X, Y, G))
    ref = np.array([np.sum(G * Y), -np.sum(G * X), -0.5 * np.sum(G * (X * X + Y * Y))])
    assert np.max(np.abs(P - ref)) <= 1e-12 * np.max(np.abs(ref))


def _body(grid, surf):
    from oracle.body import body_setup
    return body_setup(grid, surf.xs, surf.ys, surf.ds)


def _cyl_added_mass(a, dx, n):
    grid = Grid.centered(n, dx)
    surf = wl.cylinder(a, int(round(2 * np.pi * a / (1.5 * dx))))
    return added_mass(_body(grid, surf), surf.nx, surf.ny)


def test_cylinder_added_mass():
    """rho pi a^2 on each axis, approached at first order in dx (the
    regularized surface is thicker than the circle by a fraction of a
    cell); no coupling between the axes.  Rotation: the circle's rotation
    streamfunction is uniform on it, so the sheet vanishes and the paper's
    formula leaves the rigid-motion term alone, Pi = -pi a^4 (a value of
    the discrete formula, not the classical added moment of inertia, 0)."""
    a = 0.5
    m = np.pi * a * a
    M1 = _cyl_added_mass(a, 0.02, 128)
    M2 = _cyl_added_mass(a, 0.01, 256)
    for M in (M1, M2):
        assert abs(M[0, 0] - M[1, 1]) <= 1e-3 * m
        assert abs(M[0, 1]) <= 1e-9 * m and abs(M[1, 0]) <= 1e-9 * m
        assert abs(M[2, 2] / (-np.pi * a ** 4) - 1) <= 1e-6
    e1, e2 = M1[0, 0] / m - 1, M2[0, 0] / m - 1
    assert 0 < e1 <= 0.06 and 0.4 <= e2 / e1 <= 0.6


def test_ellipse_added_mass():
    """Rotated ellipse: the translational block has the eigenvalues
    rho pi b^2 and rho pi a^2 along the axes, approached at first order."""
    a, b, rot = 0.6, 0.3, 0.4
    c, s = np.cos(rot), np.sin(rot)
    R = np.array([[c, -s], [s, c]])
    ref = R @ np.diag([np.pi * b * b, np.pi * a * a]) @ R.T
    errs = []
    for n, dx in [(128, 0.02), (256, 0.01)]:
        grid = Grid.centered(n, dx)
        surf = wl.ellipse(a, b, int(round(2.9 * np.pi * 0.45 / (1.5 * dx))), rot)
        M = added_mass(_body(grid, surf), surf.nx, surf.ny)
        T = R.T @ M[:2, :2] @ R                   # into the ellipse's axes
        assert abs(T[0, 1]) <= 0.01 * np.pi * a * a
        errs.append(max(abs(T[0, 0] / (np.pi * b * b) - 1), abs(T[1, 1] / (np.pi * a * a) - 1)))
    assert errs[0] <= 0.12 and 0.4 <= errs[1] / errs[0] <= 0.6


def test_flat_plate_added_mass():
    """Zero-thickness plate: rho pi c^2 / 4 for motion normal to it (first
    order in dx, the regularized plate being a little longer), nothing along
    it and no coupling."""
    c, alpha = 1.0, 30.0
    al = np.deg2rad(alpha)
    nrm = np.array([np.sin(al), np.cos(al)])
    tan = np.array([np.cos(al), -np.sin(al)])
    errs = []
    for n, dx in [(128, 0.02), (256, 0.01)]:
        grid = Grid.centered(n, dx)
        surf = wl.flat_plate(c, alpha, int(round(c / (1.5 * dx))))
        T = added_mass(_body(grid, surf))[:2, :2]      # no normals: zero thickness
        assert abs(tan @ T @ tan) <= 1e-9 and abs(tan @ T @ nrm) <= 1e-7
        errs.append(nrm @ T @ nrm / (np.pi * c * c / 4) - 1)
    assert 0 < errs[0] <= 0.09 and 0.45 <= errs[1] / errs[0] <= 0.65


@pytest.mark.parametrize("gamma_b", [0.0, 0.7])
def test_vortices_outside_cylinder_impulse_of_images(gamma_b):
    """Cylinder at rest: the vortices and their images (-Gamma at a^2/z*,
    +Gamma at the centre, and the bound circulation at the centre) carry
    sum Gamma (1 - a^2/r^2) (y, -x); first order in dx."""
    a = 0.5
    X = np.array([0.9, -0.3, 0.1]); Y = np.array([0.2, 0.8, -0.95]); G = np.array([1.0, -0.6, 0.4])
    k = 1.0 - a * a / (X * X + Y * Y)
    ref = np.array([np.sum(G * k * Y), -np.sum(G * k * X)])
    errs = []
    for n, dx in [(128, 0.02), (256, 0.01)]:
        grid = Grid.centered(n, dx)
        surf = wl.cylinder(a, int(round(2 * np.pi * a / (1.5 * dx))))
        body = _body(grid, surf)
        p = Problem(grid=grid, X=X, Y=Y, G=G, mode="circulation", gamma_b=gamma_b)
        res = solve(p, body)
        P = solution_impulse(p, body, res, surf.nx, surf.ny)
        errs.append(np.max(np.abs(P[:2] - ref)) / np.max(np.abs(ref)))
    assert errs[0] <= 0.015 and 0.4 <= errs[1] / errs[0] <= 0.6


def test_cylinder_in_uniform_flow_impulse():
    a = 0.5
    grid = Grid.centered(128, 0.02)
    surf = wl.cylinder(a, int(round(2 * np.pi * a / (1.5 * 0.02))))
    body = _body(grid, surf)
    p = Problem(grid=grid, X=np.zeros(0), Y=np.zeros(0), G=np.zeros(0), u_inf=1.0,
                mode="circulation", gamma_b=0.0)
    res = solve(p, body)
    P = solution_impulse(p, body, res, surf.nx, surf.ny)
    # the same as the added-mass path's unit x motion, reversed (a separate
    # route: the solve with a uniform flow vs S^-1 P^Gamma y_s)
    M = added_mass(body, surf.nx, surf.ny)
    assert abs(P[0] + M[0, 0]) <= 1e-10 and abs(P[1] + M[0, 1]) <= 1e-10
    assert abs(P[0] / (-np.pi * a * a) - 1) <= 0.06 and abs(P[1]) <= 1e-9


def test_impulse_invariant_under_whole_cell_shift():
    case = wl.random_case(41, 64, 0.04, 30, surface="plate", mode="shed")
    case.ub = case.vb = case.omega = 0.0
    p0, b0 = problem_of(case), body_of(case)
    r0 = solve(p0, b0)
    P0 = solution_impulse(p0, b0, r0)
    d = (3 * case.dx, -2 * case.dx)
    sh = wl.random_case(41, 64, 0.04, 30, surface="plate", mode="shed")
    sh.ub = sh.vb = sh.omega = 0.0
    sh.X, sh.Y = sh.X + d[0], sh.Y + d[1]
    sh.surface.xs, sh.surface.ys = sh.surface.xs + d[0], sh.surface.ys + d[1]
    sh.znew = tuple((z[0] + d[0], z[1] + d[1]) for z in sh.znew)
    p1, b1 = problem_of(sh), body_of(sh)
    r1 = solve(p1, b1)
    assert np.max(np.abs(r1.f - r0.f)) <= 1e-9 * np.max(np.abs(r0.f))
    P1 = solution_impulse(p1, b1, r1)
    assert np.max(np.abs(P1[:2] - P0[:2])) <= 1e-9 * np.max(np.abs(P0[:2]))


def test_area_and_centroid():
    surf = wl.cylinder(0.4, 200, center=(0.3, -0.2))
    V, xc, yc = volume_centroid(surf.xs, surf.ys, surf.ds, surf.nx, surf.ny)
    assert abs(V / (np.pi * 0.16) - 1) <= 1e-3
    assert abs(xc - 0.3) <= 1e-4 and abs(yc + 0.2) <= 1e-4
    e = wl.ellipse(0.6, 0.25, 300, 0.5)
    V, xc, yc = volume_centroid(e.xs, e.ys, e.ds, e.nx, e.ny)
    assert abs(V / (np.pi * 0.15) - 1) <= 1e-3 and abs(xc) <= 1e-4 and abs(yc) <= 1e-4
