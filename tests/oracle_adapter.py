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
