"""Pressure (Sec. 2.6.1): the potential jump across the surface, the surface
Bernoulli equation for the pressure jump, and the grid pressure.

Test infrastructure: a plain FP64 statement of the method, used only to
check the HIP implementation.

Staggered layout of the grid (Sec. 2.1): the streamfunction and vorticity
on the n x n nodes (x_i, y_j); the velocity components on the cell faces,
u on the x-faces (x_i, y_j + dx/2) (array [j, i], (n-1) x n) and v on the
y-faces (x_i + dx/2, y_j) ((n) x (n-1)); the pressure on the cell centres
(x_i + dx/2, y_j + dx/2) ((n-1) x (n-1)).

* curl: u = (s[j+1,i] - s[j,i])/dx, v = -(s[j,i+1] - s[j,i])/dx; its matrix
  transpose maps face velocities to the node vorticity dv/dx - du/dy.
* E_f / R_f: the smoothed three-point interpolation of face data to surface
  points and its transpose, R_f = dx^-2 E_f^T diag(dS), per component.
* surface curl C_s s = n . E_f curl s (normal velocity at the points), and
  C_s^T sigma = curl^T R_f (n o sigma).
* potential jump (eq. gamphi and the formula after it):
      dphi = -(C_s L^-1 C_s^T)^+ C_s L^-1 R_s f,
  L^-1 the lattice Green's function solve (here -inv_laplacian_fft).
* surface Bernoulli (eq. surfbernoulli):
      dp = -rho (E_f v - v_s) . (gamma x n) - rho d(dphi)/dt,
  gamma x n = gamma (-n_y, n_x), v the total fluid velocity, v_s the
  surface velocity.
* grid pressure (eq. pgrid):
      p = -1/2 rho |v|^2 - rho L^-1 [ D (w x v) + R_f (n o d(dphi)/dt - v_s x gamma) ],
  w x v = (-w v, w u) on the faces (w averaged from its two nodes, the other
  velocity component from its four faces), D the divergence to the cell
  centres, |v|^2 from the face averages at the centre; v_s x gamma =
  (v_sy gamma, -v_sx gamma).
* p+- = E_c p +- dp/2 on the two sides of the surface (E_c interpolates
  cell data).

Readings: the operator C_s L^-1 C_s^T of a closed surface has the uniform
vector in its null space (the paper; numerically a small eigenvalue), so
dphi, which is defined up to a constant there, is computed with that
direction removed: the dS-weighted mean of dphi is zero (per part for
several closed bodies).  An open surface (a
plate) has no such freedom; its operator is inverted as it is, with the
normal of one side.  d(dphi)/dt is supplied by the caller (a difference of
two time levels).
"""
from __future__ import annotations

import numpy as np

from .kernels import yang3
from .operators import Grid, _gather, _scatter, _stencil, check_inside, inv_laplacian_fft, regularize_surface


def _shifted(grid: Grid, ox: float, oy: float) -> Grid:
    return Grid(grid.n, grid.dx, grid.x0 + ox * grid.dx, grid.y0 + oy * grid.dx)


def curl(s: np.ndarray, dx: float):
    return (s[1:, :] - s[:-1, :]) / dx, -(s[:, 1:] - s[:, :-1]) / dx


def curl_T(u: np.ndarray, v: np.ndarray, dx: float) -> np.ndarray:
    n = u.shape[1]
    w = np.zeros((n, n))
    w[1:, :] += u / dx
    w[:-1, :] -= u / dx
    w[:, :-1] += v / dx
    w[:, 1:] -= v / dx
    return w


def _interp(g: Grid, xs, ys, field) -> np.ndarray:
    i0, j0, wx, wy = _stencil(g, xs, ys, yang3)
    return _gather(i0, j0, wx, wy, field)


def _regularize(g: Grid, xs, ys, amp, shape) -> np.ndarray:
    i0, j0, wx, wy = _stencil(g, xs, ys, yang3)
    full = _scatter(g, i0, j0, wx, wy, amp)      # n x n, then cut to the face array
    return full[:shape[0], :shape[1]] / g.dx ** 2


def face_interp(grid: Grid, xs, ys, u, v):
    """E_f: (u, v) at the surface points."""
    check_inside(grid, xs, ys, halo=1)
    return (_interp(_shifted(grid, 0.0, 0.5), xs, ys, u),
            _interp(_shifted(grid, 0.5, 0.0), xs, ys, v))


def face_regularize(grid: Grid, xs, ys, ds, qx, qy):
    """R_f: surface vector data (qx, qy) onto the x- and y-faces."""
    n = grid.n
    return (_regularize(_shifted(grid, 0.0, 0.5), xs, ys, ds * qx, (n - 1, n)),
            _regularize(_shifted(grid, 0.5, 0.0), xs, ys, ds * qy, (n, n - 1)))


def surface_curl(grid: Grid, xs, ys, nx, ny, s) -> np.ndarray:
    """C_s s = n . E_f curl s."""
    u, v = curl(s, grid.dx)
    eu, ev = face_interp(grid, xs, ys, u, v)
    return nx * eu + ny * ev


def surface_curl_T(grid: Grid, xs, ys, ds, nx, ny, sigma) -> np.ndarray:
    """C_s^T sigma = curl^T R_f (n o sigma)."""
    qx, qy = face_regularize(grid, xs, ys, ds, nx * sigma, ny * sigma)
    return curl_T(qx, qy, grid.dx)


def Linv(q: np.ndarray, dx: float, table=None) -> np.ndarray:
    """L^-1 q (the lattice Green's function solve; -L^-1 is inv_laplacian_fft)."""
    return -inv_laplacian_fft(q, dx, table)


def jump_operator(grid: Grid, xs, ys, ds, nx, ny, table=None) -> np.ndarray:
    """M = C_s L^-1 C_s^T, column by column."""
    ns = len(xs)
    M = np.empty((ns, ns))
    for q in range(ns):
        e = np.zeros(ns)
        e[q] = 1.0
        M[:, q] = surface_curl(grid, xs, ys, nx, ny,
                               Linv(surface_curl_T(grid, xs, ys, ds, nx, ny, e), grid.dx, table))
    return M


def potential_jump(grid: Grid, xs, ys, ds, nx, ny, f, closed: bool, M=None, table=None,
                   part=None):
    """dphi = -M^+ C_s L^-1 R_s f; closed surfaces: dS-weighted mean zero
    (on each part of a several-part body, each part being closed)."""
    xs, ys, ds = (np.asarray(a, np.float64) for a in (xs, ys, ds))
    if M is None:
        M = jump_operator(grid, xs, ys, ds, nx, ny, table)
    b = -surface_curl(grid, xs, ys, nx, ny,
                      Linv(regularize_surface(grid, xs, ys, ds, f), grid.dx, table))
    if not closed:
        return np.linalg.solve(M, b)
    ns = len(xs)
    part = np.zeros(ns, int) if part is None else np.asarray(part)
    nb = int(part.max()) + 1
    A = np.zeros((ns + nb, ns + nb))
    A[:ns, :ns] = M
    for j in range(nb):
        A[:ns, ns + j] = part == j
        A[ns + j, :ns] = ds * (part == j)
    x = np.linalg.solve(A, np.r_[b, np.zeros(nb)])
    return x[:ns]


def fluid_velocity_at_surface(grid: Grid, xs, ys, s, u_inf=0.0, v_inf=0.0):
    """E_f v of the total field (s + s_inf; the uniform flow is exact)."""
    u, v = curl(s, grid.dx)
    eu, ev = face_interp(grid, xs, ys, u, v)
    return eu + u_inf, ev + v_inf


def pressure_jump(grid: Grid, xs, ys, nx, ny, f, s, vsx, vsy, ddphi_dt, rho=1.0,
                  u_inf=0.0, v_inf=0.0):
    """dp = p+ - p- from the surface Bernoulli equation (eq. surfbernoulli)."""
    eu, ev = fluid_velocity_at_surface(grid, xs, ys, s, u_inf, v_inf)
    gx, gy = -f * ny, f * nx                     # gamma x n
    return -rho * ((eu - vsx) * gx + (ev - vsy) * gy) - rho * ddphi_dt


def grid_pressure(grid: Grid, w, s, xs, ys, ds, nx, ny, f, vsx, vsy, ddphi_dt, rho=1.0,
                  u_inf=0.0, v_inf=0.0, table=None) -> np.ndarray:
    """p on the (n-1)^2 cell centres (eq. pgrid), up to a uniform value."""
    dx = grid.dx
    u, v = curl(s, dx)
    u = u + u_inf
    v = v + v_inf
    n = grid.n
    # Lamb vector w x v on the faces
    lx = np.zeros((n - 1, n))                    # x-faces (x_i, y_j+1/2)
    wx_ = 0.5 * (w[:-1, :] + w[1:, :])
    vbar = np.zeros((n - 1, n))
    vbar[:, 1:-1] = 0.25 * (v[:-1, :-1] + v[:-1, 1:] + v[1:, :-1] + v[1:, 1:])
    lx = -wx_ * vbar
    wy_ = 0.5 * (w[:, :-1] + w[:, 1:])           # y-faces (x_i+1/2, y_j)
    ubar = np.zeros((n, n - 1))
    ubar[1:-1, :] = 0.25 * (u[:-1, :-1] + u[:-1, 1:] + u[1:, :-1] + u[1:, 1:])
    ly = wy_ * ubar
    # surface terms onto the faces
    gam = np.asarray(f, np.float64)
    qx = nx * ddphi_dt - vsy * gam
    qy = ny * ddphi_dt + vsx * gam
    rx, ry = face_regularize(grid, xs, ys, ds, qx, qy)
    fx, fy = lx + rx, ly + ry
    div = (fx[:, 1:] - fx[:, :-1]) / dx + (fy[1:, :] - fy[:-1, :]) / dx    # (n-1)^2
    uc = 0.5 * (u[:, :-1] + u[:, 1:])
    vc = 0.5 * (v[:-1, :] + v[1:, :])
    return -0.5 * rho * (uc * uc + vc * vc) - rho * Linv(div, dx, table)


def cell_interp(grid: Grid, xs, ys, p) -> np.ndarray:
    """E_c: cell-centre data at the surface points."""
    cells = Grid(grid.n - 1, grid.dx, grid.x0 + 0.5 * grid.dx, grid.y0 + 0.5 * grid.dx)
    return _interp(cells, xs, ys, p)
