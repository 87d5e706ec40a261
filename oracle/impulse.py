"""Impulse, added mass and body geometry (Sec. 2.6.2 impulse-based force and
moment, Sec. 2.6.3 added mass, and the appendix on geometric relations for
discrete surfaces).

Test infrastructure: a plain FP64 statement of the formulas, used only to
check the HIP implementation.

Discrete impulse about the origin (eqs. linimpxd, linimpyd, angimpd), with
w the fluid vorticity on the nodes, <a, b>_N = dx^2 a.b the node inner
product and <a, b>_S = sum_p dS_p a_p b_p the surface one:
    q   = f + n_x v_y - n_y v_x          (sheet plus the body-motion term)
    P_x =  <y, w>_N + <y_s, q>_S
    P_y = -<x, w>_N - <x_s, q>_S
    Pi  = -1/2 <x^2 + y^2, w>_N - 1/2 <x_s^2 + y_s^2, q>_S
Force and moment on a single body are -rho d(P, Pi)/dt (eq. FMimp).

Readings: (n_x, n_y) are unit normals pointing into the fluid; a
zero-thickness body (a plate) has none (its two faces cancel in the motion
term), given as zeros.  The body velocity (v_x, v_y) is taken relative to
the fluid at infinity, (ub - U_inf - Omega y, vb - V_inf + Omega x), the
frame in which the impulse integrals hold; the bound sheet f is the same in
either frame.

Added mass (Sec. 2.6.3): for unit x translation, y translation and unit
rotation about the origin, the sheet of the basic problem without the Kutta
condition f = S^-1 P^Gamma s_b (s_b = y_s, -x_s, -(x_s^2 + y_s^2)/2) and
the motion v = (1, 0), (0, 1), (-y_s, x_s) give the impulses P^(i); then
row i of the 3x3 tensor is rho (P_x^(i), P_y^(i), Pi^(i) - (X_c P_y^(i) - Y_c P_x^(i))).

Geometry (appendix): V = <x_s, n_x>_S = <y_s, n_y>_S (their mean is used),
X_c = <x_s^2 + y_s^2, n_x>_S / (2V), Y_c likewise with n_y (eq. centroid).
For a body without normals (V = 0) the arc-length centroid of the points
stands in for X_c.
"""
from __future__ import annotations

import numpy as np

from .operators import Grid, regularize_vortices


def node_impulse(grid: Grid, w) -> np.ndarray:
    """(<y, w>_N, -<x, w>_N, -1/2 <x^2 + y^2, w>_N) over the nodes; w[j, i]."""
    X, Y = np.meshgrid(grid.node_x(), grid.node_y(), indexing="xy")
    a = grid.dx ** 2
    return np.array([a * np.sum(Y * w), -a * np.sum(X * w),
                     -0.5 * a * np.sum((X * X + Y * Y) * w)])


def surface_impulse(xs, ys, ds, f, nx, ny, vx, vy) -> np.ndarray:
    """(<y_s, q>_S, -<x_s, q>_S, -1/2 <x_s^2 + y_s^2, q>_S), q = f + n_x v_y - n_y v_x."""
    q = np.asarray(f, np.float64) + nx * vy - ny * vx
    return np.array([np.sum(ds * ys * q), -np.sum(ds * xs * q),
                     -0.5 * np.sum(ds * (xs * xs + ys * ys) * q)])


def impulse(grid: Grid, X, Y, G, xs=None, ys=None, ds=None, f=None, nx=None, ny=None,
            vx=0.0, vy=0.0) -> np.ndarray:
    """(P_x, P_y, Pi_O) of vortices (X, Y, G) and, optionally, a body with
    sheet f moving with surface velocity (vx, vy)."""
    P = node_impulse(grid, regularize_vortices(grid, X, Y, G))
    if xs is not None:
        ns = len(xs)
        nx = np.zeros(ns) if nx is None else np.asarray(nx, np.float64)
        ny = np.zeros(ns) if ny is None else np.asarray(ny, np.float64)
        P = P + surface_impulse(np.asarray(xs, np.float64), np.asarray(ys, np.float64),
                                np.asarray(ds, np.float64), f, nx, ny, vx, vy)
    return P


def solution_impulse(p, body, res, nx=None, ny=None) -> np.ndarray:
    """Impulse of a solved problem: all fluid vortices (any new ones with
    their strengths) and the body's sheet and motion relative to the fluid
    at infinity."""
    X, Y, G = np.asarray(p.X, np.float64), np.asarray(p.Y, np.float64), np.asarray(p.G, np.float64)
    if res.gamma_new is not None and len(p.znew):
        X = np.concatenate([X, [z[0] for z in p.znew]])
        Y = np.concatenate([Y, [z[1] for z in p.znew]])
        G = np.concatenate([G, res.gamma_new])
    if body is None:
        return impulse(p.grid, X, Y, G)
    vx = p.ub - p.u_inf - p.omega * body.ys
    vy = p.vb - p.v_inf + p.omega * body.xs
    return impulse(p.grid, X, Y, G, body.xs, body.ys, body.ds, res.f, nx, ny, vx, vy)


def volume_centroid(xs, ys, ds, nx, ny):
    """Enclosed area and centroid from the surface points (eq. centroid)."""
    xs, ys, ds = (np.asarray(a, np.float64) for a in (xs, ys, ds))
    nx, ny = np.asarray(nx, np.float64), np.asarray(ny, np.float64)
    V = 0.5 * (np.sum(ds * xs * nx) + np.sum(ds * ys * ny))
    if V == 0.0:
        L = np.sum(ds)
        return 0.0, float(np.sum(ds * xs) / L), float(np.sum(ds * ys) / L)
    r2 = xs * xs + ys * ys
    return float(V), float(np.sum(ds * r2 * nx) / (2 * V)), float(np.sum(ds * r2 * ny) / (2 * V))


def added_mass(body, nx=None, ny=None, rho=1.0) -> np.ndarray:
    """3x3 added-mass tensor: rows x translation, y translation, rotation
    about the origin; columns force x, force y, moment about the centroid."""
    xs, ys, ds = body.xs, body.ys, body.ds
    ns = len(xs)
    nx = np.zeros(ns) if nx is None else np.asarray(nx, np.float64)
    ny = np.zeros(ns) if ny is None else np.asarray(ny, np.float64)
    _, xc, yc = volume_centroid(xs, ys, ds, nx, ny)
    motions = [(ys, np.ones(ns), np.zeros(ns)),                     # s_b, v_x, v_y
               (-xs, np.zeros(ns), np.ones(ns)),
               (-0.5 * (xs * xs + ys * ys), -ys, xs)]
    M = np.empty((3, 3))
    for i, (sb, vx, vy) in enumerate(motions):
        f = body.solve(body.remove_circulation(sb))
        P = surface_impulse(xs, ys, ds, f, nx, ny, vx, vy)
        M[i] = rho * np.array([P[0], P[1], P[2] - (xc * P[1] - yc * P[0])])
    return M
