"""Immersed surface: Schur complement and its per-body constants (Sec. 2.2-2.4).

* S = -E_s L^-1 R_s (Schur complement of eq. basicblock), built exactly from
  the LGF table:  S_pq = -dS_q sum_{a in st(p)} sum_{b in st(q)} e_pa e_qb G(a - b)
  (the dx^2 of L^-1 cancels the dx^-2 of R_s).
* f0 = S^-1 1 (eq. f0), Gamma0 = <1, f0>_S (eq. circ0), fhat0 = diag(dS) f0.
* Circulation removal P^Gamma = I - 1 fhat0^T / Gamma0 (eq. circrem).
* Rescaled Schur complement S~ = S diag(f0) (Sec. 2.4), so S~^-1 x = (S^-1 x) / f0.

S is symmetric for uniform dS but indefinite (one negative eigenvalue, the
uniform mode), so it is factored by partially pivoted LU, never Cholesky.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

from .lgf import lgf_table
from .operators import Grid, surface_matrix


def schur_matrix(grid: Grid, xs, ys, ds, table=None) -> np.ndarray:
    """Dense S = -E_s L^-1 R_s for the surface points (float64)."""
    E, nodes = surface_matrix(grid, xs, ys)
    if table is None:
        table = lgf_table(grid.n)
    di = np.abs(nodes[:, None, 0] - nodes[None, :, 0])
    dj = np.abs(nodes[:, None, 1] - nodes[None, :, 1])
    Gnn = table[di, dj]                      # G between stencil nodes
    return -(E @ Gnn @ E.T) * np.asarray(ds, np.float64)[None, :]


@dataclass
class Body:
    xs: np.ndarray
    ys: np.ndarray
    ds: np.ndarray
    S: np.ndarray
    lu: tuple            # scipy LU factors of S
    f0: np.ndarray       # S^-1 1
    gamma0: float        # <1, f0>_S
    fhat0: np.ndarray    # dS * f0

    def solve(self, rhs) -> np.ndarray:
        """S^-1 rhs (rhs may have several columns)."""
        return sla.lu_solve(self.lu, rhs)

    def solve_tilde(self, rhs) -> np.ndarray:
        """S~^-1 rhs = (S^-1 rhs) / f0, with S~ = S diag(f0)."""
        x = self.solve(rhs)
        return x / (self.f0 if np.ndim(x) == 1 else self.f0[:, None])

    def remove_circulation(self, s) -> np.ndarray:
        """P^Gamma s = s - 1 (fhat0 . s) / Gamma0 (eq. circrem)."""
        return s - np.dot(self.fhat0, s) / self.gamma0


def body_setup(grid: Grid, xs, ys, ds, table=None) -> Body:
    xs = np.asarray(xs, np.float64)
    ys = np.asarray(ys, np.float64)
    ds = np.asarray(ds, np.float64)
    S = schur_matrix(grid, xs, ys, ds, table)
    lu = sla.lu_factor(S)
    f0 = sla.lu_solve(lu, np.ones(len(xs)))
    gamma0 = float(np.dot(ds, f0))
    return Body(xs, ys, ds, S, lu, f0, gamma0, ds * f0)
