"""Pins of the oracle's grid operators (Sec. 2.1-2.2): L^-1 by two routes,
regularization/interpolation adjointness, circulation conservation, exact
point-vortex fields, second-order convergence (Fig. 2) and velocities."""
import numpy as np
import pytest

from oracle.lgf import EULER_GAMMA, lgf_table
from oracle.operators import (Grid, interpolate_surface, interpolate_vortices,
                              inv_laplacian_direct, inv_laplacian_fft, laplacian,
                              regularize_surface, regularize_vortices, vortex_velocity)
from paper_2102_11910_amd import workloads as wl


def test_direct_sum_equals_fft_convolution():
    rng = np.random.default_rng(0)
    n, dx = 24, 0.1
    w = np.zeros((n, n))
    idx = rng.integers(0, n, size=(30, 2))
    w[idx[:, 1], idx[:, 0]] = rng.standard_normal(30)
    a = inv_laplacian_direct(w, dx)
    b = inv_laplacian_fft(w, dx)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(a))


def test_inverse_laplacian_solves_poisson_in_window():
    rng = np.random.default_rng(1)
    n, dx = 64, 0.05
    grid = Grid.centered(n, dx)
    h = (n - 1) * dx / 2 - 4 * dx
    X, Y = rng.uniform(-h, h, 50), rng.uniform(-h, h, 50)
    w = regularize_vortices(grid, X, Y, rng.standard_normal(50))
    s = inv_laplacian_fft(w, dx)
    Ls = laplacian(s, dx)
    assert np.max(np.abs(Ls[1:-1, 1:-1] + w[1:-1, 1:-1])) <= 1e-10 * np.max(np.abs(w))


def test_on_node_vortex_is_scaled_lgf():
    n, dx, gam = 32, 0.07, 0.8
    grid = Grid.centered(n, dx)
    i1, j1 = 10, 13
    w = regularize_vortices(grid, [grid.x0 + i1 * dx], [grid.y0 + j1 * dx], [gam])
    # M4' interpolates: an on-node vortex puts Gamma/dx^2 on one node only
    assert np.count_nonzero(w) == 1 and abs(w[j1, i1] * dx * dx - gam) < 1e-13
    s = inv_laplacian_fft(w, dx)
    T = lgf_table(n)
    J, I = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    exact = -gam * T[np.abs(I - i1), np.abs(J - j1)]
    assert np.max(np.abs(s - exact)) <= 1e-12 * np.max(np.abs(exact))


def test_point_vortex_far_field_log():
    n, dx, gam = 128, 0.01, 1.3
    grid = Grid.centered(n, dx)
    i1 = j1 = 20
    w = regularize_vortices(grid, [grid.x0 + i1 * dx], [grid.y0 + j1 * dx], [gam])
    s = inv_laplacian_fft(w, dx)
    J, I = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    r = np.hypot(I - i1, J - j1) * dx
    far = r >= 10 * dx
    const = gam / (2 * np.pi) * (np.log(dx) - EULER_GAMMA - 1.5 * np.log(2.0))
    resid = s + gam / (2 * np.pi) * np.log(np.where(far, r, 1.0)) - const
    assert np.all(np.abs(resid[far]) <= 0.05 * abs(gam) * (dx / r[far]) ** 2)


def test_circulation_conservation():
    rng = np.random.default_rng(2)
    n, dx = 48, 0.03
    grid = Grid.centered(n, dx)
    h = (n - 1) * dx / 2 - 3 * dx
    X, Y, G = rng.uniform(-h, h, 300), rng.uniform(-h, h, 300), rng.standard_normal(300)
    w = regularize_vortices(grid, X, Y, G)
    assert abs(dx * dx * w.sum() - G.sum()) <= 1e-13 * np.abs(G).sum()
    xs, ys = rng.uniform(-h, h, 40), rng.uniform(-h, h, 40)
    ds, f = rng.uniform(0.01, 0.05, 40), rng.standard_normal(40)
    wr = regularize_surface(grid, xs, ys, ds, f)
    assert abs(dx * dx * wr.sum() - np.dot(ds, f)) <= 1e-13 * np.abs(ds * f).sum()


def test_regularization_is_transpose_of_interpolation():
    rng = np.random.default_rng(3)
    n, dx = 40, 0.05
    grid = Grid.centered(n, dx)
    h = (n - 1) * dx / 2 - 3 * dx
    g = rng.standard_normal((n, n))
    X, Y, G = rng.uniform(-h, h, 25), rng.uniform(-h, h, 25), rng.standard_normal(25)
    lhs = dx * dx * np.sum(regularize_vortices(grid, X, Y, G) * g)
    rhs = np.dot(G, interpolate_vortices(grid, X, Y, g))
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)
    xs, ys, ds, f = (rng.uniform(-h, h, 25), rng.uniform(-h, h, 25),
                     rng.uniform(0.01, 0.1, 25), rng.standard_normal(25))
    lhs = dx * dx * np.sum(regularize_surface(grid, xs, ys, ds, f) * g)
    rhs = np.sum(ds * f * interpolate_surface(grid, xs, ys, g))
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)


def test_surface_interpolation_exact_for_linear_fields():
    rng = np.random.default_rng(4)
    n, dx = 40, 0.05
    grid = Grid.centered(n, dx)
    h = (n - 1) * dx / 2 - 3 * dx
    xs, ys = rng.uniform(-h, h, 30), rng.uniform(-h, h, 30)
    X, Y = np.meshgrid(grid.node_x(), grid.node_y())
    lin = 0.7 * Y - 0.3 * X + 0.2
    assert np.max(np.abs(interpolate_surface(grid, xs, ys, lin) - (0.7 * ys - 0.3 * xs + 0.2))) < 1e-14
    assert np.max(np.abs(interpolate_vortices(grid, xs, ys, lin) - (0.7 * ys - 0.3 * xs + 0.2))) < 1e-14


def test_out_of_window_rejected():
    grid = Grid.centered(16, 0.1)
    with pytest.raises(ValueError):
        regularize_vortices(grid, [grid.x0 + 1.5 * 0.1], [0.0], [1.0])


def test_lone_vortex_no_self_velocity_and_freestream():
    n, dx = 32, 0.05
    grid = Grid.centered(n, dx)
    x, y = grid.x0 + 15 * dx, grid.y0 + 16 * dx
    w = regularize_vortices(grid, [x], [y], [2.0])
    s = inv_laplacian_fft(w, dx)
    u, v = vortex_velocity(grid, s, [x], [y], 0.0, 0.0)
    assert abs(u[0]) < 1e-13 and abs(v[0]) < 1e-13
    u, v = vortex_velocity(grid, np.zeros((n, n)), [0.013], [-0.21], 1.25, -0.5)
    assert u[0] == 1.25 and v[0] == -0.5


def test_second_order_streamfunction_convergence():
    """Fig. 2: random vortices in the lower-left quadrant, error of the
    streamfunction on the upper-right quadrant, second order in dx."""
    rng = np.random.default_rng(5)
    nvort = 20
    Xv = rng.uniform(-0.8, -0.25, nvort)
    Yv = rng.uniform(-0.8, -0.25, nvort)
    Gv = rng.uniform(-1.0, 1.0, nvort)
    errs = []
    for dx in (0.04, 0.02, 0.01):
        n = int(round(2.2 / dx)) + 1
        grid = Grid.centered(n, dx)
        w = regularize_vortices(grid, Xv, Yv, Gv)
        s = inv_laplacian_fft(w, dx)
        XX, YY = np.meshgrid(grid.node_x(), grid.node_y())
        q = (XX >= 0.2) & (YY >= 0.2) & (XX <= 1.0) & (YY <= 1.0)
        exact = np.zeros_like(XX)
        for xq, yq, gq in zip(Xv, Yv, Gv):
            exact -= gq / (2 * np.pi) * np.log(np.hypot(XX - xq, YY - yq))
        # the discrete gauge G(0,0) = 0 fixes the additive constant exactly
        exact += Gv.sum() / (2 * np.pi) * (np.log(dx) - EULER_GAMMA - 1.5 * np.log(2.0))
        errs.append(np.linalg.norm((s - exact)[q]) / np.linalg.norm(exact[q]))
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(order >= 1.8), (errs, order)


def test_workload_surfaces_geometry():
    c = wl.cylinder(0.5, 100)
    assert np.allclose(np.hypot(c.xs, c.ys), 0.5, atol=1e-7)
    p = wl.flat_plate(1.0, 20.0, 256)
    assert abs(p.xs[0] + 0.4698) < 2e-3 and abs(p.ys[0] - 0.1710) < 2e-3
    e = wl.ellipse(0.5, 0.1, 512)
    seg = np.hypot(np.diff(np.r_[e.xs, e.xs[0]]), np.diff(np.r_[e.ys, e.ys[0]]))
    assert seg.max() / seg.min() < 1.01
