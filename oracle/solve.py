"""The constrained streamfunction solves (Sec. 2.2-2.4, appendix A).

All modes start from the intermediate field of the vortices alone,
s* = -L^-1 w with w = R_v Gamma (eq. poisson, first step of the block-LU
algorithm of eq. basicblock), and end with one more unbounded Poisson solve
for the streamfunction of all vorticity: fluid vortices, any new vortices
and the bound sheet.  Velocities at the vortices difference that field and
add the uniform flow (Sec. 2.1).

Notation: rhs streamfunction s_b' = s_b - E_s s_inf (eq. nopen), with
s_b = U y - V x - Omega (x^2 + y^2)/2 (eq. sfsurf) and s_inf = U_inf y - V_inf x.
Because the smoothed 3-point kernel interpolates linear functions exactly,
E_s s_inf = U_inf y_s - V_inf x_s on the surface points.

Modes
-----
* ``circulation``  prescribed bound circulation Gamma_b (eq. circsystem):
      f_a = S^-1 (s_b' - E_s s*),  s0 = (<1, f_a> - Gamma_b)/Gamma0,
      f = f_a - s0 f0                                    (eq. circs0)
* ``kutta``        steady Kutta condition at edge k (eq. kuttasystem):
      f~* = S~^-1 (P^Gamma s_b' - E_s s*)                (eq. intermedsoln)
      s0 = f~*_k (eq. s0),  f~ = P_k f~* = f~* - s0 1,  f = f0 o f~
* ``shed``         Kutta condition at m edges k_1..k_m, each with a new vortex
                   at z_j, plus Kelvin's theorem (eq. kuttasystem2, kuttasystem3):
      f~_j = S~^-1 E_s L^-1 d_j,
      sum_j (1 + fhat0 . P_{k_i} f~_j) Gamma_j = -(Gamma_w + fhat0 . P_{k_i} f~*)
                                                          (eq. twovortex, any m)
      x = f~* + sum_j Gamma_j f~_j,  s0 = mean_i x_{k_i},  f~ = x - s0 1
      With edge bounds (Sec. 2.5, generalized edge condition; bounds on the
      non-singular sheet f~ at each edge, Kutta = both bounds zero): edge i
      is active when the intermediate sheet lies outside [fmin_i, fmax_i] at
      k_i, with target the violated bound t_i; inactive edges shed nothing
      (Gamma_i = 0).  The intermediate sheet tested is the Kelvin-consistent
      one, f~*_K = f~* - (fhat0 . f~* + Gamma_w)/Gamma0, i.e. the sheet the
      body would carry if nothing were shed: f~* alone moves with the
      Green's function gauge and with the constant removed from s_b, while
      f~*_K does not, and with it a shed strength goes to zero as f~*_K
      reaches its bound.  The active rows read (eq. twovortex-gen)
      sum_j (1 + fhat0 . P_{k_i} f~_j) Gamma_j = -(Gamma_w + fhat0 . P_{k_i} f~* + Gamma0 t_i)
      and s0 = mean over active i of (x_{k_i} - t_i); with no active edge,
      Kelvin's theorem alone gives s0 = (fhat0 . f~* + Gamma_w)/Gamma0.
* ``none``         no body: s = s*.

Time stepping: ``rk2_step`` (explicit midpoint, fixed modes) and
``shed_step`` (forward Euler with one new vortex per edge, Sec. 2.4.2).

E_s s* here equals -E_s L^-1 w of the paper's formulas.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .body import Body
from .lgf import lgf_table
from .operators import (Grid, check_inside, interpolate_surface, inv_laplacian_fft,
                        regularize_surface, regularize_vortices, surface_matrix,
                        unit_vortex, vortex_velocity, _stencil)
from .kernels import m4prime


@dataclass
class Problem:
    grid: Grid
    X: np.ndarray                 # vortex x
    Y: np.ndarray                 # vortex y
    G: np.ndarray                 # vortex strengths Gamma_q
    u_inf: float = 0.0
    v_inf: float = 0.0
    ub: float = 0.0               # rigid body motion (eq. velsurf)
    vb: float = 0.0
    omega: float = 0.0
    mode: str = "none"            # none | circulation | kutta | shed
    gamma_b: float = 0.0          # circulation mode
    edges: tuple = ()             # kutta: (k,), shed: (k_1..k_m)
    znew: tuple = ()              # shed: new vortex positions [(x, y), ...]
    gamma_w: float | None = None  # shed: circulation of existing vorticity
    fbounds: tuple = ()           # shed: ((fmin, fmax), ...) per edge; () = Kutta (0, 0)


@dataclass
class Result:
    s: np.ndarray                              # streamfunction minus s_inf
    u: np.ndarray = field(default_factory=lambda: np.zeros(0))
    v: np.ndarray = field(default_factory=lambda: np.zeros(0))
    f: np.ndarray | None = None                # bound vortex sheet strength
    ftilde: np.ndarray | None = None           # non-singular part f / f0
    s0: float = 0.0
    gamma_new: np.ndarray | None = None        # shed vortex strengths
    gamma_b: float = 0.0                       # <1, f>_S
    s_star: np.ndarray | None = None           # intermediate field -L^-1 R_v Gamma
    w_total: np.ndarray | None = None          # total source of the final solve


def surface_rhs(p: Problem, body: Body) -> np.ndarray:
    """s_b' = s_b - E_s s_inf = (U-U_inf) y - (V-V_inf) x - Omega (x^2+y^2)/2."""
    return ((p.ub - p.u_inf) * body.ys - (p.vb - p.v_inf) * body.xs
            - 0.5 * p.omega * (body.xs ** 2 + body.ys ** 2))


def surface_response_to_vortex(grid: Grid, body: Body, z, table=None) -> np.ndarray:
    """(E_s L^-1 d) for a unit vortex at z, by direct LGF sums.

    L^-1 d = dx^2 G * (dx^-2 M4'(x) M4'(y)) = G * (M4' x M4'): the dx factors
    cancel, so (E_s L^-1 d)_p = sum_a e_pa sum_b m_b G(a - b).
    """
    if table is None:
        table = lgf_table(grid.n)
    E, nodes = surface_matrix(grid, body.xs, body.ys)
    check_inside(grid, [z[0]], [z[1]], halo=1)
    i0, j0, wx, wy = _stencil(grid, [z[0]], [z[1]], m4prime)
    acc = np.zeros(len(nodes))
    for a in range(4):
        for b in range(4):
            di = np.abs(nodes[:, 0] - (i0[0] + a))
            dj = np.abs(nodes[:, 1] - (j0[0] + b))
            acc += wx[0, a] * wy[0, b] * table[di, dj]
    return E @ acc


def solve(p: Problem, body: Body | None = None, table=None) -> Result:
    grid = p.grid
    if table is None:
        table = lgf_table(grid.n)
    w = regularize_vortices(grid, p.X, p.Y, p.G)
    s_star = inv_laplacian_fft(w, grid.dx, table)

    if p.mode == "none":
        u, v = vortex_velocity(grid, s_star, p.X, p.Y, p.u_inf, p.v_inf)
        return Result(s=s_star, u=u, v=v, s_star=s_star, w_total=w)

    assert body is not None
    Es_star = interpolate_surface(grid, body.xs, body.ys, s_star)
    sb = surface_rhs(p, body)
    gamma_new = None
    w_total = w.copy()

    if p.mode == "circulation":
        fa = body.solve(sb - Es_star)
        s0 = (np.dot(body.ds, fa) - p.gamma_b) / body.gamma0
        f = fa - s0 * body.f0
        ftilde = f / body.f0
    elif p.mode == "kutta":
        (k,) = p.edges
        ft_star = body.solve_tilde(body.remove_circulation(sb) - Es_star)
        s0 = ft_star[k]
        ftilde = ft_star - s0
        f = body.f0 * ftilde
    elif p.mode == "shed":
        edges = list(p.edges)
        m = len(edges)
        assert len(p.znew) == m
        gamma_w = float(np.sum(p.G)) if p.gamma_w is None else float(p.gamma_w)
        ft_star = body.solve_tilde(body.remove_circulation(sb) - Es_star)
        ft_j = np.stack([body.solve_tilde(surface_response_to_vortex(grid, body, z, table))
                         for z in p.znew], axis=1)                     # Ns x m
        bounds = list(p.fbounds) if p.fbounds else [(0.0, 0.0)] * m
        assert len(bounds) == m
        # active edges and their targets (the violated bound), tested on
        # the Kelvin-consistent intermediate sheet
        ft_kel = ft_star - (body.fhat0 @ ft_star + gamma_w) / body.gamma0
        active, target = [], []
        for i, k in enumerate(edges):
            lo, hi = bounds[i]
            if ft_kel[k] < lo:
                active.append(i)
                target.append(lo)
            elif ft_kel[k] > hi:
                active.append(i)
                target.append(hi)
        gamma_new = np.zeros(m)
        if active:
            na = len(active)
            A = np.empty((na, na))
            rhs = np.empty(na)
            for r, (i, t) in enumerate(zip(active, target)):
                k = edges[i]
                # fhat0 . P_k x = fhat0 . x - Gamma0 x_k
                A[r, :] = 1.0 + body.fhat0 @ ft_j[:, active] - body.gamma0 * ft_j[k, active]
                rhs[r] = -(gamma_w + body.fhat0 @ ft_star - body.gamma0 * ft_star[k]
                           + body.gamma0 * t)
            gamma_new[active] = np.linalg.solve(A, rhs)
            x = ft_star + ft_j @ gamma_new
            s0 = float(np.mean([x[edges[i]] - t for i, t in zip(active, target)]))
        else:
            x = ft_star
            s0 = float((body.fhat0 @ ft_star + gamma_w) / body.gamma0)
        ftilde = x - s0
        f = body.f0 * ftilde
        for gj, z in zip(gamma_new, p.znew):
            w_total += gj * unit_vortex(grid, z[0], z[1])
    else:
        raise ValueError(p.mode)

    w_total += regularize_surface(grid, body.xs, body.ys, body.ds, f)
    s = inv_laplacian_fft(w_total, grid.dx, table)
    u, v = vortex_velocity(grid, s, p.X, p.Y, p.u_inf, p.v_inf)
    return Result(s=s, u=u, v=v, f=f, ftilde=ftilde, s0=float(s0), gamma_new=gamma_new,
                  gamma_b=float(np.dot(body.ds, f)), s_star=s_star, w_total=w_total)


def rk2_step(p: Problem, body: Body | None, dt: float, table=None):
    """One explicit-midpoint step of vortex advection.

    The paper advances vortices with forward Euler or RK4 (Sec. 2.4, 2.6);
    the midpoint rule uses the same velocity evaluation twice:
    x* = x + dt/2 u(x),  x <- x + dt u(x*).  The prescribed bound
    circulation, if any, is kept fixed over the step.
    Returns (X_new, Y_new, first-stage result, second-stage result).
    """
    r1 = solve(p, body, table)
    Xm = p.X + 0.5 * dt * r1.u
    Ym = p.Y + 0.5 * dt * r1.v
    pm = Problem(**{**p.__dict__, "X": Xm, "Y": Ym})
    r2 = solve(pm, body, table)
    return p.X + dt * r2.u, p.Y + dt * r2.v, r1, r2


@dataclass
class ShedState:
    """Vortices of a shedding run and, per edge, the index of the last vortex
    it released with nonzero strength (-1 before the first)."""
    X: np.ndarray
    Y: np.ndarray
    G: np.ndarray
    last: list


def shed_step(p: Problem, body: Body, st: ShedState, dt: float, first, table=None):
    """One forward Euler step of vortex shedding (Sec. 2.4.2; Sec. 2.5 with
    edge bounds).

    New vortex j goes one third of the way from edge point k_j to the
    current position of the last vortex that edge released, or to the edge
    point plus first[j] before its first release.  The new vortices join the
    set with strength zero, so the solve (shedding mode of p, its bounds
    included, Gamma_w the sum of the strengths) also gives the velocity at
    them; they then take the strengths Gamma_j, and every vortex moves by
    x <- x + dt u(x).  An edge that shed zero keeps its last release.
    Returns the new state, the solve's result and the problem it solved
    (vortices before the move, new ones included with strength zero).
    """
    edges = list(p.edges)
    znew = []
    for j, k in enumerate(edges):
        ex, ey = body.xs[k], body.ys[k]
        l = st.last[j]
        if l >= 0:
            znew.append((ex + (st.X[l] - ex) / 3.0, ey + (st.Y[l] - ey) / 3.0))
        else:
            znew.append((ex + first[j][0], ey + first[j][1]))
    nv = len(st.X)
    X = np.concatenate([st.X, [z[0] for z in znew]])
    Y = np.concatenate([st.Y, [z[1] for z in znew]])
    G = np.concatenate([st.G, np.zeros(len(edges))])
    q = Problem(**{**p.__dict__, "X": X, "Y": Y, "G": G, "znew": tuple(znew), "gamma_w": None})
    res = solve(q, body, table)
    G1 = G.copy()          # q keeps the new vortices at strength zero
    G1[nv:] = res.gamma_new
    last = [nv + j if res.gamma_new[j] != 0.0 else st.last[j] for j in range(len(edges))]
    return ShedState(X + dt * res.u, Y + dt * res.v, G1, last), res, q
