"""Turn a generated workload case into the oracle's problem description."""
import numpy as np

from oracle.body import body_setup
from oracle.operators import Grid
from oracle.solve import Problem


def grid_of(case):
    return Grid.centered(case.n, case.dx)


def problem_of(case, X=None, Y=None):
    return Problem(grid=grid_of(case),
                   X=np.asarray(case.X if X is None else X, np.float64),
                   Y=np.asarray(case.Y if Y is None else Y, np.float64),
                   G=np.asarray(case.G, np.float64),
                   u_inf=case.u_inf, v_inf=case.v_inf, ub=case.ub, vb=case.vb,
                   omega=case.omega, mode=case.mode, gamma_b=case.gamma_b,
                   edges=tuple(case.edges), znew=tuple(case.znew), gamma_w=case.gamma_w,
                   fbounds=tuple(case.fbounds))


def body_of(case, table=None):
    if case.surface is None:
        return None
    s = case.surface
    return body_setup(grid_of(case), s.xs, s.ys, s.ds, table)


def intermediate_sheet(case, body=None):
    """The oracle's intermediate sheet f~* of a shedding case, its
    Kelvin-consistent shift f~*_K (the sheet with nothing shed, which the
    generalized edge conditions of Sec. 2.5 inspect), and the unit-vortex
    responses f~_j."""
    from oracle.operators import interpolate_surface, inv_laplacian_fft, regularize_vortices
    from oracle.solve import surface_response_to_vortex, surface_rhs
    p = problem_of(case)
    body = body or body_of(case)
    grid = p.grid
    w = regularize_vortices(grid, p.X, p.Y, p.G)
    Es_star = interpolate_surface(grid, body.xs, body.ys, inv_laplacian_fft(w, grid.dx))
    ft_star = body.solve_tilde(body.remove_circulation(surface_rhs(p, body)) - Es_star)
    ft_j = [body.solve_tilde(surface_response_to_vortex(grid, body, z)) for z in case.znew]
    gamma_w = float(np.sum(p.G)) if p.gamma_w is None else p.gamma_w
    ft_kel = ft_star - (body.fhat0 @ ft_star + gamma_w) / body.gamma0
    return ft_star, ft_kel, ft_j


def multi_of(mc):
    """A several-body workload case as the oracle's problem, body and parts."""
    from oracle.multibody import BodySpec, MultiProblem
    grid = grid_of(mc)
    specs = []
    fb = list(mc.fbounds)
    zi = 0
    for j, q in enumerate(mc.parts):
        edges = mc.part_edges(j)
        spec = BodySpec(mode=q["mode"], gamma_b=q.get("gamma_b", 0.0), ub=q.get("ub", 0.0),
                        vb=q.get("vb", 0.0), omega=q.get("omega", 0.0),
                        gamma_w=q.get("gamma_w", 0.0))
        if q["mode"] == "kutta":
            spec.edges = edges[:1]
        elif q["mode"] == "shed":
            spec.edges = edges
            spec.znew = tuple(mc.znew[zi:zi + len(edges)])
            if fb:
                spec.fbounds = tuple(fb[zi:zi + len(edges)])
            zi += len(edges)
        specs.append(spec)
    p = MultiProblem(grid, np.asarray(mc.X, np.float64), np.asarray(mc.Y, np.float64),
                     np.asarray(mc.G, np.float64), specs, mc.u_inf, mc.v_inf)
    body = body_setup(grid, mc.xs, mc.ys, mc.ds)
    return p, body, mc.part
