"""Grid operators, regularization and interpolation (Sec. 2.1-2.2).

Conventions (readings of the paper where it is silent):

* The grid is a finite window of the infinite node lattice: n x n nodes,
  node (i, j) at (x0 + i dx, y0 + j dx); arrays are stored [j, i].
* Every kernel stencil must lie inside the window; for vortices a 1-node
  halo is also required because velocities difference the streamfunction.
  Then total circulation is conserved exactly (Sec. 2.1).
* The regularization of eq. (vortexregularization) is
      w_ij = dx^-2 sum_q Gamma_q d((x_i - X_q)/dx) d((y_j - Y_q)/dx),
  and the interpolation E_v is its transpose with respect to the grid inner
  product <a,b> = dx^2 a.b and the plain sum on the vortex points, i.e. a
  weighted sum whose weights add up to one (Sec. 2.1, after Fig. 2).
* Surface regularization R_s is the transpose of the surface interpolation
  E_s with respect to the grid and surface inner products (Sec. 2.2.1):
      R_s f = dx^-2 E_s^T diag(dS) f.
* L = Delta_h / dx^2 and L^-1 w = dx^2 (G * w) over the infinite lattice
  (Sec. 2.1), so the particular solution of L s = -w is s = -dx^2 (G * w).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .kernels import m4prime, yang3
from .lgf import lgf_table


@dataclass(frozen=True)
class Grid:
    n: int          # nodes per direction
    dx: float       # cell size
    x0: float       # x of node i = 0
    y0: float       # y of node j = 0

    @staticmethod
    def centered(n: int, dx: float) -> "Grid":
        """Window centred on the origin: x0 = y0 = -(n-1) dx / 2."""
        h = -(n - 1) * dx / 2.0
        return Grid(int(n), float(dx), h, h)

    def node_x(self) -> np.ndarray:
        return self.x0 + self.dx * np.arange(self.n)

    def node_y(self) -> np.ndarray:
        return self.y0 + self.dx * np.arange(self.n)


# ----------------------------------------------------------------------------
# stencils
# ----------------------------------------------------------------------------

def _stencil(grid: Grid, px, py, kernel):
    """4x4 stencil of a radius-2 kernel at points (px, py).

    Returns (i0, j0, wx, wy): base node indices (lowest node of the stencil)
    and the 1-D weights wx[p, a] = d(xi_p - (i0_p + a)), a = 0..3.
    """
    xi = (np.asarray(px, np.float64) - grid.x0) / grid.dx
    eta = (np.asarray(py, np.float64) - grid.y0) / grid.dx
    i0 = np.floor(xi).astype(np.int64) - 1
    j0 = np.floor(eta).astype(np.int64) - 1
    a = np.arange(4)
    wx = kernel(xi[:, None] - (i0[:, None] + a[None, :]))
    wy = kernel(eta[:, None] - (j0[:, None] + a[None, :]))
    return i0, j0, wx, wy


def check_inside(grid: Grid, px, py, halo: int = 0) -> None:
    """Raise if a radius-2 stencil (plus `halo` nodes) leaves the window."""
    xi = (np.asarray(px, np.float64) - grid.x0) / grid.dx
    eta = (np.asarray(py, np.float64) - grid.y0) / grid.dx
    lo, hi = 1 + halo, grid.n - 2 - halo
    for v in (xi, eta):
        if v.size and (v.min() < lo or v.max() >= hi):
            raise ValueError("stencil leaves the grid window")


def _scatter(grid: Grid, i0, j0, wx, wy, amp) -> np.ndarray:
    out = np.zeros((grid.n, grid.n))
    for a in range(4):
        for b in range(4):
            np.add.at(out, (j0 + b, i0 + a), amp * wx[:, a] * wy[:, b])
    return out


def _gather(i0, j0, wx, wy, field) -> np.ndarray:
    out = np.zeros(len(i0))
    for a in range(4):
        for b in range(4):
            out += wx[:, a] * wy[:, b] * field[j0 + b, i0 + a]
    return out


# ----------------------------------------------------------------------------
# regularization R and interpolation E
# ----------------------------------------------------------------------------

def regularize_vortices(grid: Grid, X, Y, gamma) -> np.ndarray:
    """R_v Gamma: grid vorticity of point vortices (eq. vortexregularization)."""
    check_inside(grid, X, Y, halo=1)
    i0, j0, wx, wy = _stencil(grid, X, Y, m4prime)
    return _scatter(grid, i0, j0, wx, wy, np.asarray(gamma, np.float64)) / grid.dx ** 2


def unit_vortex(grid: Grid, x: float, y: float) -> np.ndarray:
    """d_q: grid vorticity of a unit-strength vortex at (x, y) (Sec. 2.1)."""
    return regularize_vortices(grid, [x], [y], [1.0])


def interpolate_vortices(grid: Grid, X, Y, field) -> np.ndarray:
    """E_v field: M4' interpolation at the vortex points (weights sum to one)."""
    i0, j0, wx, wy = _stencil(grid, X, Y, m4prime)
    return _gather(i0, j0, wx, wy, field)


def interpolate_surface(grid: Grid, xs, ys, field) -> np.ndarray:
    """E_s field: smoothed 3-point interpolation at the surface points."""
    check_inside(grid, xs, ys)
    i0, j0, wx, wy = _stencil(grid, xs, ys, yang3)
    return _gather(i0, j0, wx, wy, field)


def regularize_surface(grid: Grid, xs, ys, ds, f) -> np.ndarray:
    """R_s f = dx^-2 E_s^T diag(dS) f (transpose w.r.t. both inner products)."""
    check_inside(grid, xs, ys)
    i0, j0, wx, wy = _stencil(grid, xs, ys, yang3)
    amp = np.asarray(ds, np.float64) * np.asarray(f, np.float64)
    return _scatter(grid, i0, j0, wx, wy, amp) / grid.dx ** 2


def surface_matrix(grid: Grid, xs, ys):
    """E_s as a dense (Ns x U) matrix over the U distinct stencil nodes.

    Returns (E, nodes) where nodes[u] = (i, j).
    """
    check_inside(grid, xs, ys)
    i0, j0, wx, wy = _stencil(grid, xs, ys, yang3)
    ns = len(i0)
    ii = (i0[:, None, None] + np.arange(4)[None, :, None]) * np.ones((1, 1, 4), np.int64)
    jj = (j0[:, None, None] + np.arange(4)[None, None, :]) * np.ones((1, 4, 1), np.int64)
    ww = wx[:, :, None] * wy[:, None, :]
    keys = (jj * grid.n + ii).reshape(ns, 16)
    uniq, inv = np.unique(keys, return_inverse=True)
    E = np.zeros((ns, len(uniq)))
    np.add.at(E, (np.repeat(np.arange(ns), 16), inv.ravel()), ww.reshape(ns, 16).ravel())
    nodes = np.stack([uniq % grid.n, uniq // grid.n], axis=1)
    return E, nodes


# ----------------------------------------------------------------------------
# L and L^-1
# ----------------------------------------------------------------------------

def laplacian(s: np.ndarray, dx: float) -> np.ndarray:
    """L s = Delta_h s / dx^2 on interior nodes (edges left at zero)."""
    out = np.zeros_like(s)
    out[1:-1, 1:-1] = (s[1:-1, 2:] + s[1:-1, :-2] + s[2:, 1:-1] + s[:-2, 1:-1]
                       - 4.0 * s[1:-1, 1:-1]) / dx ** 2
    return out


def inv_laplacian_direct(w: np.ndarray, dx: float, table=None) -> np.ndarray:
    """-L^-1 w by the direct lattice sum s_ij = -dx^2 sum G(i-i', j-j') w_i'j'.

    Only the nonzero sources are visited; O(n^2 * nnz).
    """
    n = w.shape[0]
    if table is None:
        table = lgf_table(n - 1)
    jj, ii = np.nonzero(w)
    J, I = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    s = np.zeros((n, n))
    for j1, i1 in zip(jj, ii):
        s += table[np.abs(I - i1), np.abs(J - j1)] * w[j1, i1]
    return -dx ** 2 * s


def lgf_kernel_padded(n: int, table=None) -> np.ndarray:
    """K(i, j) = G(min(i, 2n-i), min(j, 2n-j)) on the (2n)^2 periodic box.

    Convolving the zero-padded source with K circularly equals the
    infinite-lattice convolution on the n x n window.
    """
    if table is None:
        table = lgf_table(n)
    k = np.arange(2 * n)
    k = np.minimum(k, 2 * n - k)
    return table[k[None, :], k[:, None]]


def inv_laplacian_fft(w: np.ndarray, dx: float, table=None) -> np.ndarray:
    """-L^-1 w by zero-padded FFT convolution with the LGF (float64)."""
    n = w.shape[0]
    K = lgf_kernel_padded(n, table)
    pad = np.zeros((2 * n, 2 * n))
    pad[:n, :n] = w
    conv = np.fft.irfft2(np.fft.rfft2(pad) * np.fft.rfft2(K), s=(2 * n, 2 * n))
    return -dx ** 2 * conv[:n, :n]


# ----------------------------------------------------------------------------
# velocity
# ----------------------------------------------------------------------------

def node_velocity(s: np.ndarray, dx: float):
    """u = ds/dy, v = -ds/dx at nodes.

    The curl puts velocity components on cell faces by centred differences
    (eq. velsf); averaging the two faces next to a node (Sec. 2.1) gives the
    centred difference across the node.  Edge nodes are left NaN.
    """
    u = np.full_like(s, np.nan)
    v = np.full_like(s, np.nan)
    u[1:-1, :] = (s[2:, :] - s[:-2, :]) / (2.0 * dx)
    v[:, 1:-1] = -(s[:, 2:] - s[:, :-2]) / (2.0 * dx)
    return u, v


def vortex_velocity(grid: Grid, s: np.ndarray, X, Y, u_inf=0.0, v_inf=0.0):
    """Velocity at the vortices: node velocities of s interpolated by E_v.

    s is the streamfunction without the uniform-flow part s_inf =
    U_inf y - V_inf x, whose (exact) velocity (U_inf, V_inf) is added.
    """
    check_inside(grid, X, Y, halo=1)
    u, v = node_velocity(s, grid.dx)
    return (interpolate_vortices(grid, X, Y, u) + u_inf,
            interpolate_vortices(grid, X, Y, v) + v_inf)
