"""Several bodies in one flow (Sec. 2.7, eq. kuttasystem4).

Test infrastructure: a plain FP64 statement of the method, used only to
check the HIP implementation.

All surface points of all bodies form one Schur complement S (the bodies
see each other through L^-1); the sheet is partitioned by body, and each
body j has its own uniform streamfunction value s0_j.  With the
decomposition f = f0 o f~ (f0 = S^-1 1 over all points, S~ = S diag(f0)):

    f~ = f~* + sum_i Gamma_i f~_i - sum_j s0_j z~_j
    f~* = S~^-1 (s_b' - E_s s*),   f~_i = S~^-1 E_s L^-1 d_i,   z~_j = S~^-1 1_j

(1_j: ones on the points of body j; sum_j z~_j = 1).  The circulation of
body j is fhat0_j . f~ with fhat0_j = dS o f0 o 1_j.  One row per body and
one per new vortex close the system in (s0_1.., Gamma_1..):

* prescribed circulation:  fhat0_j . f~ = Gamma_b,j
* steady Kutta at edge k:  f~_k = 0 (bound circulation free)
* shedding (eq. kuttasystem4, any number of edges):
      Kelvin for the body:  fhat0_j . f~ + sum_{i of body j} Gamma_i = -Gamma_w,j
      each edge i active:   f~_{k_i} = t_i,     inactive: Gamma_i = 0
  with edge bounds as for one body (Sec. 2.5): an edge is active when the
  sheet with nothing shed (every Gamma_i = 0, all rows of the other kinds
  kept) lies outside [fmin_i, fmax_i] at k_i; t_i is the bound it violates.

Readings: Gamma_w,j is the circulation of the vortices released from body j
(the paper's Kelvin row per body); s_b' enters without the circulation
projection, whose uniform shift each s0_j absorbs (for one body the s0
reported differs from the projected form by fhat0 . s_b' / Gamma0, while f
and the strengths are the same).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .body import Body
from .lgf import lgf_table
from .operators import (Grid, interpolate_surface, inv_laplacian_fft, regularize_surface,
                        regularize_vortices, unit_vortex, vortex_velocity)
from .solve import surface_response_to_vortex


@dataclass
class BodySpec:
    mode: str                      # circulation | kutta | shed
    gamma_b: float = 0.0           # circulation
    ub: float = 0.0                # rigid motion of this body (eq. velsurf)
    vb: float = 0.0
    omega: float = 0.0
    edges: tuple = ()              # global surface indices (kutta: one; shed: one per new vortex)
    znew: tuple = ()               # shed: new vortex positions
    gamma_w: float = 0.0           # shed: circulation released from this body so far
    fbounds: tuple = ()            # shed: ((fmin, fmax), ...); () = Kutta


@dataclass
class MultiProblem:
    grid: Grid
    X: np.ndarray
    Y: np.ndarray
    G: np.ndarray
    bodies: list
    u_inf: float = 0.0
    v_inf: float = 0.0


@dataclass
class MultiResult:
    s: np.ndarray
    u: np.ndarray
    v: np.ndarray
    f: np.ndarray
    ftilde: np.ndarray
    s0: np.ndarray                 # per body
    gamma_new: np.ndarray          # new vortices, bodies in order, edges in order
    gamma_b: np.ndarray            # bound circulation per body
    w_total: np.ndarray = field(default=None)


def solve_multi(p: MultiProblem, body: Body, part, table=None) -> MultiResult:
    """body: the Schur data of all points together; part[p] = body of point p."""
    grid = p.grid
    if table is None:
        table = lgf_table(grid.n)
    part = np.asarray(part)
    nb = len(p.bodies)
    w = regularize_vortices(grid, p.X, p.Y, p.G)
    s_star = inv_laplacian_fft(w, grid.dx, table)
    Es_star = interpolate_surface(grid, body.xs, body.ys, s_star)
    # s_b' point by point with the motion of the point's body
    sb = np.empty(len(body.xs))
    for j, b in enumerate(p.bodies):
        on = part == j
        x, y = body.xs[on], body.ys[on]
        sb[on] = (b.ub - p.u_inf) * y - (b.vb - p.v_inf) * x - 0.5 * b.omega * (x * x + y * y)
    ft_star = body.solve_tilde(sb - Es_star)
    Z = np.stack([body.solve_tilde((part == j).astype(float)) for j in range(nb)], axis=1)
    owner, edge_k, znew, bounds = [], [], [], []
    for j, b in enumerate(p.bodies):
        if b.mode == "shed":
            bb = list(b.fbounds) if b.fbounds else [(0.0, 0.0)] * len(b.edges)
            for k, z, lohi in zip(b.edges, b.znew, bb):
                owner.append(j)
                edge_k.append(k)
                znew.append(z)
                bounds.append(lohi)
    m = len(znew)
    F = (np.stack([body.solve_tilde(surface_response_to_vortex(grid, body, z, table))
                   for z in znew], axis=1) if m else np.zeros((len(body.xs), 0)))
    fhat = [body.fhat0 * (part == j) for j in range(nb)]

    def system(active, target):
        """Rows and right-hand side in the unknowns (s0_1..s0_nb, Gamma_1..Gamma_m)."""
        N = nb + m
        A = np.zeros((N, N))
        r = np.zeros(N)
        for j, b in enumerate(p.bodies):
            if b.mode == "kutta":
                (k,) = b.edges
                A[j, :nb] = -Z[k, :]
                A[j, nb:] = F[k, :]
                r[j] = -ft_star[k]
            else:
                A[j, :nb] = -fhat[j] @ Z
                A[j, nb:] = fhat[j] @ F
                if b.mode == "circulation":
                    r[j] = b.gamma_b - fhat[j] @ ft_star
                elif b.mode == "shed":
                    for i in range(m):
                        if owner[i] == j:
                            A[j, nb + i] += 1.0
                    r[j] = -b.gamma_w - fhat[j] @ ft_star
                else:
                    raise ValueError(b.mode)
        for i in range(m):
            row = nb + i
            if active[i]:
                k = edge_k[i]
                A[row, :nb] = -Z[k, :]
                A[row, nb:] = F[k, :]
                r[row] = target[i] - ft_star[k]
            else:
                A[row, nb + i] = 1.0
        return A, r

    # edge activity on the sheet with nothing shed
    sol = np.linalg.solve(*system([False] * m, [0.0] * m))
    ft_keep = ft_star + F @ sol[nb:] - Z @ sol[:nb]
    active, target = [], []
    for i in range(m):
        lo, hi = bounds[i]
        v = ft_keep[edge_k[i]]
        active.append(v < lo or v > hi)
        target.append(lo if v < lo else (hi if v > hi else 0.0))
    if any(active):
        sol = np.linalg.solve(*system(active, target))
    s0 = sol[:nb]
    gamma_new = sol[nb:]
    ftilde = ft_star + F @ gamma_new - Z @ s0
    f = body.f0 * ftilde
    w_total = w + regularize_surface(grid, body.xs, body.ys, body.ds, f)
    for g, z in zip(gamma_new, znew):
        w_total = w_total + g * unit_vortex(grid, z[0], z[1])
    s = inv_laplacian_fft(w_total, grid.dx, table)
    u, v = vortex_velocity(grid, s, p.X, p.Y, p.u_inf, p.v_inf)
    gb = np.array([np.dot(body.ds * (part == j), f) for j in range(nb)])
    return MultiResult(s=s, u=u, v=v, f=f, ftilde=ftilde, s0=s0, gamma_new=gamma_new,
                       gamma_b=gb, w_total=w_total)


@dataclass
class MultiShedState:
    """Vortices of a several-body shedding run, per new-vortex edge the index
    of its last nonzero release (-1 before the first), and per body the
    circulation it has released (its Gamma_w)."""
    X: np.ndarray
    Y: np.ndarray
    G: np.ndarray
    last: list
    gw: list


def shed_step_multi(p: MultiProblem, body: Body, part, st: MultiShedState, dt: float, first,
                    table=None):
    """One forward Euler shedding step of several bodies (Sec. 2.4.2 with the
    rows of Sec. 2.7): every edge of a shedding body places a new vortex as
    for one body (a third of the way to its last release, or at the edge
    point plus first[i] before the first), the solve gives their strengths,
    each body's released circulation grows by the strengths of its new
    vortices, and every vortex moves by x <- x + dt u(x).  Returns the new
    state, the result and the problem solved."""
    import dataclasses
    edges, owners = [], []
    for j, b in enumerate(p.bodies):
        if b.mode == "shed":
            for k in b.edges:
                edges.append(k)
                owners.append(j)
    znew = []
    for i, k in enumerate(edges):
        ex, ey = body.xs[k], body.ys[k]
        l = st.last[i]
        if l >= 0:
            znew.append((ex + (st.X[l] - ex) / 3.0, ey + (st.Y[l] - ey) / 3.0))
        else:
            znew.append((ex + first[i][0], ey + first[i][1]))
    nv = len(st.X)
    m = len(edges)
    X = np.concatenate([st.X, [z[0] for z in znew]])
    Y = np.concatenate([st.Y, [z[1] for z in znew]])
    G = np.concatenate([st.G, np.zeros(m)])
    specs, i0 = [], 0
    for j, b in enumerate(p.bodies):
        nb = dataclasses.replace(b)
        if b.mode == "shed":
            ne = len(b.edges)
            nb.znew = tuple(znew[i0:i0 + ne])
            nb.gamma_w = st.gw[j]
            i0 += ne
        specs.append(nb)
    q = MultiProblem(p.grid, X, Y, G, specs, p.u_inf, p.v_inf)
    res = solve_multi(q, body, part, table)
    G1 = G.copy()
    G1[nv:] = res.gamma_new
    gw = list(st.gw)
    for g, j in zip(res.gamma_new, owners):
        gw[j] += g
    last = [nv + i if res.gamma_new[i] != 0.0 else st.last[i] for i in range(m)]
    return MultiShedState(X + dt * res.u, Y + dt * res.v, G1, last, gw), res, q
