"""Pins of the oracle's pressure (Sec. 2.6.1).

* the jump operator C_s L^-1 C_s^T of a circle is symmetric and negative
  semi-definite with its near-null vector close to uniform (the paper's
  stated properties, up to sign convention);
* the potential jump of a circle in a uniform flow U is the classical
  2 U a cos(theta) (first order in dx) and its derivative along the surface
  is the sheet strength;
* the pressure jump of the same steady flow from the surface Bernoulli
  equation is the classical exterior distribution -2 rho U^2 sin^2(theta)
  (the interior fluid is at rest), first order in dx;
* the grid pressure of a pair of opposite vortices (on nodes), which
  translates steadily, is the exact unsteady pressure rho U u - rho |v|^2/2
  away from the cores, second order in dx (the Lamb-vector term carries the
  unsteadiness);
* a plate's operator (open surface) has no near-null direction.
"""
import numpy as np
import pytest

from oracle import pressure as pr
from oracle.body import body_setup
from oracle.operators import Grid, inv_laplacian_fft, regularize_vortices
from oracle.solve import Problem, solve
from paper_2102_11910_amd import workloads as wl


def _cylinder_flow(n, dx, a=0.5):
    grid = Grid.centered(n, dx)
    surf = wl.cylinder(a, int(round(2 * np.pi * a / (1.5 * dx))))
    body = body_setup(grid, surf.xs, surf.ys, surf.ds)
    p = Problem(grid=grid, X=np.zeros(0), Y=np.zeros(0), G=np.zeros(0), u_inf=1.0,
                mode="circulation", gamma_b=0.0)
    return grid, surf, body, solve(p, body)


def test_jump_operator_properties():
    grid, surf, body, _ = _cylinder_flow(64, 0.04)
    M = pr.jump_operator(grid, body.xs, body.ys, body.ds, surf.nx, surf.ny)
    assert np.max(np.abs(M - M.T)) <= 1e-12 * np.max(np.abs(M))
    ev, V = np.linalg.eigh(M)
    assert ev[-1] <= 1e-12 * abs(ev[0])                 # negative semi-definite
    assert abs(ev[-1]) <= 2e-3 * abs(ev[0])             # one near-null direction
    v = V[:, -1] * np.sign(V[0, -1])
    assert np.ptp(v) <= 0.1 * np.mean(np.abs(v))        # close to uniform


def test_potential_jump_of_cylinder_in_uniform_flow():
    errs = []
    for n, dx in [(64, 0.04), (128, 0.02)]:
        grid, surf, body, res = _cylinder_flow(n, dx)
        dphi = pr.potential_jump(grid, body.xs, body.ys, body.ds, surf.nx, surf.ny, res.f, True)
        th = np.arctan2(body.ys, body.xs)
        A = np.linalg.lstsq(np.c_[np.cos(th), np.sin(th), np.ones_like(th)], dphi, rcond=None)[0]
        errs.append(abs(A[0] - 1.0))                    # 2 U a = 1
        assert abs(A[1]) <= 1e-9 and abs(np.dot(body.ds, dphi)) <= 1e-9
        # d(dphi)/ds is the sheet strength (low modes)
        dd = (np.roll(dphi, -1) - np.roll(dphi, 1)) / (2 * body.ds[0])
        B = np.linalg.lstsq(np.c_[np.sin(th)], dd, rcond=None)[0][0]
        F = np.linalg.lstsq(np.c_[np.sin(th)], res.f, rcond=None)[0][0]
        assert abs(B / F - 1.0) <= 0.03
    assert errs[1] <= 0.6 * errs[0] and errs[1] <= 0.02


def test_steady_pressure_jump_of_cylinder():
    """dp = -2 rho U^2 sin^2 theta + const = const' + rho U^2 cos 2theta."""
    errs = []
    for n, dx in [(64, 0.04), (128, 0.02)]:
        grid, surf, body, res = _cylinder_flow(n, dx)
        th = np.arctan2(body.ys, body.xs)
        z = np.zeros_like(th)
        dp = pr.pressure_jump(grid, body.xs, body.ys, surf.nx, surf.ny, res.f, res.s, z, z, z,
                              1.0, 1.0, 0.0)
        c = np.linalg.lstsq(np.c_[np.ones_like(th), np.cos(2 * th), np.sin(2 * th)], dp,
                            rcond=None)[0]
        errs.append(abs(c[1] - 1.0))
        assert abs(c[2]) <= 1e-6
    assert errs[1] <= 0.6 * errs[0] and errs[1] <= 0.02


def test_pressure_of_translating_vortex_pair():
    errs = []
    for n, dx in [(64, 0.04), (128, 0.02), (256, 0.01)]:
        grid = Grid.centered(n, dx)
        k = int(round(0.25 / dx))
        xn = grid.x0 + dx * (n // 2)
        yt, yb = grid.y0 + dx * (n // 2 + k), grid.y0 + dx * (n // 2 - k)
        X, Y, G = np.array([xn, xn]), np.array([yt, yb]), np.array([1.0, -1.0])
        w = regularize_vortices(grid, X, Y, G)
        s = inv_laplacian_fft(w, dx)
        e = np.zeros(0)
        P = pr.grid_pressure(grid, w, s, e, e, e, e, e, e, e, e, e, rho=1.0)
        xc = grid.x0 + dx * (np.arange(n - 1) + 0.5)
        XC, YC = np.meshgrid(xc, grid.y0 + dx * (np.arange(n - 1) + 0.5))
        ue, ve = np.zeros_like(XC), np.zeros_like(XC)
        for x, y, g in zip(X, Y, G):
            r2 = (XC - x) ** 2 + (YC - y) ** 2
            ue += -g * (YC - y) / (2 * np.pi * r2)
            ve += g * (XC - x) / (2 * np.pi * r2)
        U = 1.0 / (2 * np.pi * (yt - yb))                # the pair moves to +x
        exact = U * ue - 0.5 * (ue ** 2 + ve ** 2)
        sel = ((np.hypot(XC - xn, YC - yt) > 0.3) & (np.hypot(XC - xn, YC - yb) > 0.3)
               & (np.hypot(XC, YC) < 0.9))
        errs.append(np.ptp((P - exact)[sel]))
    assert errs[0] <= 2e-3
    assert errs[1] <= 0.6 * errs[0] and errs[2] <= 0.6 * errs[1]


def test_open_plate_jump_operator_is_invertible():
    """A plate (open surface, one-sided normal) has no uniform null
    direction: its operator is inverted as it is."""
    grid = Grid.centered(64, 0.04)
    surf = wl.flat_plate(1.2, 25.0, 20)
    al = np.deg2rad(25.0)
    nx, ny = np.full(20, np.sin(al)), np.full(20, np.cos(al))
    M = pr.jump_operator(grid, surf.xs, surf.ys, surf.ds, nx, ny)
    ev = np.linalg.eigvalsh(0.5 * (M + M.T))
    assert ev[-1] < 0 and abs(ev[-1]) >= 1e-3 * abs(ev[0])


def test_two_cylinders_mirror_potential_jump():
    """Two mirror-image cylinders (several-part body, each part closed) in a
    uniform flow along the mirror line, with mirrored vortices of opposite
    strength: the potential jump is even under the reflection (the sheet,
    its derivative along the surface, is odd), and each part's dS-weighted
    mean is zero."""
    from oracle.multibody import BodySpec, MultiProblem, solve_multi
    grid = Grid.centered(96, 0.04)
    th = 2 * np.pi * (np.arange(40) + 0.5) / 40
    x1 = wl.f32(-0.8 + 0.4 * np.cos(th))
    y1 = wl.f32(0.4 * np.sin(th))
    xs, ys = np.r_[x1, -x1], np.r_[y1, y1]
    ds = np.full(80, 2 * np.pi * 0.4 / 40)
    nx1, ny1 = np.cos(th), np.sin(th)
    nx, ny = np.r_[nx1, -nx1], np.r_[ny1, ny1]
    part = np.r_[np.zeros(40, int), np.ones(40, int)]
    body = body_setup(grid, xs, ys, ds)
    X1 = np.array([-0.2, -1.5]); Y1 = np.array([0.7, -0.3]); G1 = np.array([0.4, -0.2])
    specs = [BodySpec("circulation", gamma_b=0.3), BodySpec("circulation", gamma_b=-0.3)]
    res = solve_multi(MultiProblem(grid, np.r_[X1, -X1], np.r_[Y1, Y1], np.r_[G1, -G1], specs,
                                   u_inf=0.0, v_inf=1.0), body, part)
    dphi = pr.potential_jump(grid, xs, ys, ds, nx, ny, res.f, True, part=part)
    assert np.max(np.abs(dphi[:40] - dphi[40:])) <= 1e-9 * np.max(np.abs(dphi))
    for j in range(2):
        assert abs(np.dot(ds * (part == j), dphi)) <= 1e-10
