"""Pins of the oracle's shedding loop (forward Euler, Sec. 2.4.2; edge
bounds of Sec. 2.5).

Every step is one pinned solve in the shedding mode (test_oracle_solve);
these tests pin what the loop adds around it:
* the insertion geometry: a new vortex lies on the segment from its edge
  to that edge's last release, at a third of its length;
* Kelvin's theorem over the run: the bound circulation cancels the total
  vortex circulation after every step, and the Kutta condition holds;
* bookkeeping: m vortices join per step, an edge inside its bounds sheds
  strength zero and keeps its last release;
* reduction: with both edges free nothing is shed, and the existing
  vortices move as forward Euler under the prescribed-circulation solve
  with Gamma_b = -Gamma_w (a different mode's solve).
"""
import numpy as np

from oracle.solve import ShedState, shed_step, solve
from paper_2102_11910_amd import workloads as wl
from tests.oracle_adapter import body_of, problem_of

FREE = (-1e30, 1e30)


def _start(seed=21, nv=12):
    case = wl.random_case(seed, 64, 0.04, nv, surface="plate", mode="shed")
    p = problem_of(case)
    body = body_of(case)
    first = [(z[0] - body.xs[k], z[1] - body.ys[k]) for z, k in zip(case.znew, case.edges)]
    st = ShedState(p.X.copy(), p.Y.copy(), p.G.copy(), [-1] * len(case.edges))
    return case, p, body, first, st


def test_insertion_geometry_and_kelvin_over_a_run():
    case, p, body, first, st = _start()
    m = len(case.edges)
    dt = 0.02
    for step in range(4):
        prev = st
        st, res, _ = shed_step(p, body, prev, dt, first)
        nv = len(prev.X)
        assert len(st.X) == nv + m
        for j, k in enumerate(case.edges):
            e = np.array([body.xs[k], body.ys[k]])
            zj = np.array([st.X[nv + j] - dt * res.u[nv + j], st.Y[nv + j] - dt * res.v[nv + j]])
            if prev.last[j] < 0:
                ref = e + np.array(first[j])
            else:
                zl = np.array([prev.X[prev.last[j]], prev.Y[prev.last[j]]])
                # on the segment e -> z_last, at a third of its length
                a, b = zj - e, zl - e
                assert abs(a[0] * b[1] - a[1] * b[0]) <= 1e-12 * (b @ b)
                assert abs(np.linalg.norm(a) * 3.0 - np.linalg.norm(b)) <= 1e-12 * np.linalg.norm(b)
                assert a @ b > 0
                ref = e + b / 3.0
            assert np.max(np.abs(zj - ref)) <= 1e-12
            assert st.G[nv + j] == res.gamma_new[j] != 0.0
            assert st.last[j] == nv + j
            assert abs(res.ftilde[k]) <= 1e-12
        # Kelvin: bound circulation cancels all vortex circulation
        assert abs(np.dot(body.ds, res.f) + st.G.sum()) <= 1e-12 * max(1.0, np.abs(st.G).sum())
        # forward Euler for the vortices that existed before the step
        assert np.array_equal(st.X[:nv], prev.X + dt * res.u[:nv])


def test_free_edges_shed_nothing_and_reduce_to_prescribed_circulation():
    case, p, body, first, st = _start(seed=22)
    p.fbounds = (FREE, FREE)
    dt = 0.02
    nv = len(st.X)
    st1, res, _ = shed_step(p, body, st, dt, first)
    assert np.all(res.gamma_new == 0.0) and st1.last == [-1, -1]
    assert np.all(st1.G[nv:] == 0.0)
    circ = wl.random_case(22, 64, 0.04, 12, surface="plate", mode="circulation")
    circ.gamma_b = -float(np.sum(case.G))
    rc = solve(problem_of(circ), body)
    scale = np.max(np.abs(rc.u)) + np.max(np.abs(rc.v))
    assert np.max(np.abs(st1.X[:nv] - (st.X + dt * rc.u))) <= 1e-10 * dt * scale
    assert np.max(np.abs(st1.Y[:nv] - (st.Y + dt * rc.v))) <= 1e-10 * dt * scale
    # the next step again places at the first-release offsets
    st2, res2, _ = shed_step(p, body, st1, dt, first)
    for j, k in enumerate(case.edges):
        x0 = st2.X[nv + 2 + j] - dt * res2.u[nv + 2 + j]
        assert abs(x0 - (body.xs[k] + first[j][0])) <= 1e-12


def test_one_free_edge_keeps_its_last_release():
    """Leading edge held by Kutta, trailing edge with bounds wide enough to
    be inside: only the leading edge releases, and its second vortex goes a
    third of the way to its first."""
    case, p, body, first, st = _start(seed=23)
    p.fbounds = ((0.0, 0.0), FREE)
    dt = 0.02
    nv = len(st.X)
    st1, r1, _ = shed_step(p, body, st, dt, first)
    st2, r2, _ = shed_step(p, body, st1, dt, first)
    assert r1.gamma_new[1] == 0.0 and r2.gamma_new[1] == 0.0
    assert st2.last == [nv + 2, -1]
    k = case.edges[0]
    zx = st2.X[nv + 2] - dt * r2.u[nv + 2]
    assert abs(zx - (body.xs[k] + (st1.X[nv] - body.xs[k]) / 3.0)) <= 1e-12


def test_impulse_and_lift_of_an_impulsive_start():
    """A plate nose up in a uniform flow, started from rest, shedding at its
    trailing edge only: Kelvin holds after every step (total circulation
    zero), and the lift from the impulse rate, -rho dP_y/dt (eq. FMimp),
    follows Wagner's classical result for an impulsive start: about half the
    steady lift pi rho c U^2 sin(alpha) at first, changing slowly.  (The first
    difference spans the jump from the first release, placed at the given
    offset, to the one-third rule, and is left out.)"""
    from oracle.impulse import solution_impulse
    case, p, body, first, st = _start(seed=24, nv=0)
    p.v_inf = 0.0
    p.fbounds = (FREE, (0.0, 0.0))
    P = []
    dt = 0.02
    for _ in range(6):
        st, res, q = shed_step(p, body, st, dt, first)
        assert abs(st.G.sum() + np.dot(body.ds, res.f)) <= 1e-12
        assert res.gamma_new[0] == 0.0 and res.gamma_new[1] > 0.0
        P.append(solution_impulse(q, body, res))
    lift = -np.diff(np.array(P)[:, 1]) / dt
    sf = case.surface
    steady = np.pi * sf.params["chord"] * np.sin(np.deg2rad(sf.params["alpha_deg"]))
    ratio = lift[1:] / steady
    assert np.all((ratio > 0.45) & (ratio < 0.65)), ratio
    assert ratio.max() / ratio.min() < 1.05, ratio
