"""Pressure on the GPU (gpf_pressure, Sec. 2.6.1) against the oracle: the
potential jump, the pressure jump of the surface Bernoulli equation (with
a time derivative from a previous level), the grid pressure on the cell
centres and the two side pressures, for a closed cylinder, an open plate
and a several-part body; FP64 plans to 1e-9, FP32 fields to 1e-4."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2102_11910_amd import gpf  # noqa: E402
from paper_2102_11910_amd import workloads as wl  # noqa: E402
from oracle import pressure as pr  # noqa: E402
from oracle.solve import solve as oracle_solve  # noqa: E402
from tests.conftest import rell2  # noqa: E402
from tests.oracle_adapter import body_of, problem_of  # noqa: E402

DEV = torch.device("cuda", 0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    return gpf.Context(0)


def _normals(case):
    sf = case.surface
    if sf.nx is not None:
        return sf.nx, sf.ny, True
    al = np.deg2rad(sf.params["alpha_deg"])       # plate: one side's normal
    return np.full(sf.ns, np.sin(al)), np.full(sf.ns, np.cos(al)), False


def _oracle_pressure(case, res, nx, ny, closed, dphi_prev=None, dt=1.0, rho=1.0, part=None):
    p, body = problem_of(case), body_of(case)
    dphi = pr.potential_jump(p.grid, body.xs, body.ys, body.ds, nx, ny, res.f, closed, part=part)
    ddt = np.zeros_like(dphi) if dphi_prev is None else (dphi - dphi_prev) / dt
    vsx = p.ub - p.omega * body.ys
    vsy = p.vb + p.omega * body.xs
    dp = pr.pressure_jump(p.grid, body.xs, body.ys, nx, ny, res.f, res.s, vsx, vsy, ddt, rho,
                          p.u_inf, p.v_inf)
    from oracle.operators import regularize_vortices
    X = np.r_[p.X, [z[0] for z in p.znew]] if res.gamma_new is not None else p.X
    Y = np.r_[p.Y, [z[1] for z in p.znew]] if res.gamma_new is not None else p.Y
    G = np.r_[p.G, res.gamma_new] if res.gamma_new is not None else p.G
    w = regularize_vortices(p.grid, X, Y, G)
    P = pr.grid_pressure(p.grid, w, res.s, body.xs, body.ys, body.ds, nx, ny, res.f, vsx, vsy,
                         ddt, rho, p.u_inf, p.v_inf)
    pc = pr.cell_interp(p.grid, body.xs, body.ys, P)
    return dphi, dp, P, pc + 0.5 * dp, pc - 0.5 * dp


def _gpu(ctx, case, flags, nx, ny, closed, prev_case=None, dt=1.0, rho=1.0):
    edges = tuple(case.edges) if case.mode in ("kutta", "shed") else None
    s = gpf.Solver(ctx, case.n, case.dx, case.surface, flags=flags, edges=edges)
    s.body.set_normals(nx, ny, closed)
    ns, n = case.surface.ns, case.n
    z = lambda k: torch.zeros(k, dtype=torch.float64, device=DEV)
    dphi_prev = None
    if prev_case is not None:
        X, Y, G = s.upload(prev_case)
        s.solve(s.inputs_for(prev_case, X, Y, G), X)
        gpf.gpf_sync(s.status)
        dphi_prev, dp0 = z(ns), z(ns)
        gpf.gpf_pressure(s.plan, s.body, s.inputs_for(prev_case, X, Y, G), s.psi, s.f,
                         dphi_prev, dp0, rho=rho)
    X, Y, G = s.upload(case)
    inp = s.inputs_for(case, X, Y, G)
    s.solve(inp, X)
    gpf.gpf_sync(s.status)
    dphi, dp, P, side = z(ns), z(ns), z(n * n), z(2 * ns)
    gpf.gpf_pressure(s.plan, s.body, inp, s.psi, s.f, dphi, dp, P, side, dphi_prev=dphi_prev,
                     dt=dt, rho=rho)
    gpf.gpf_sync(s.status)
    h = lambda t: t.cpu().numpy()
    return h(dphi), h(dp), h(P).reshape(n, n)[:n - 1, :n - 1], h(side)


def _check(label, got, ref, tol):
    names = ("dphi", "dp", "p", "p+", "p-")
    gd, gdp, gP, gs = got
    vals = (gd, gdp, gP - gP.mean(), gs[:len(gd)], gs[len(gd):])
    refs = (ref[0], ref[1], ref[2] - ref[2].mean(), ref[3], ref[4])
    # the side pressures carry the grid pressure's free constant: compare
    # them after removing the cell field's mean on each side
    shift = gP.mean() - ref[2].mean()
    vals = vals[:3] + (vals[3] - shift, vals[4] - shift)
    errs = [rell2(v, r) for v, r in zip(vals, refs)]
    say(f"   {label}: " + ", ".join(f"{k} {e:.2e}" for k, e in zip(names, errs)))
    for k, e in zip(names, errs):
        assert e <= tol, (label, k, e)


@pytest.mark.parametrize("flags", [gpf.GPF_FP64, gpf.GPF_FP32])
def test_cylinder_pressure(ctx, flags):
    say(f"[pressure] moving cylinder, vortices, circulation, flags={flags}")
    case = wl.random_case(171, 128, 2.0 / 128, 300, surface="cylinder", mode="circulation")
    nx, ny, closed = _normals(case)
    got = _gpu(ctx, case, flags, nx, ny, closed)
    ref = _oracle_pressure(case, oracle_solve(problem_of(case), body_of(case)), nx, ny, closed)
    _check(f"cylinder flags={flags}", got, ref, 1e-9 if flags == gpf.GPF_FP64 else 1e-4)


@pytest.mark.parametrize("flags", [gpf.GPF_FP64, gpf.GPF_POLICY_AUTO])
def test_plate_pressure_with_time_derivative(ctx, flags):
    """An open plate (Kutta at its trailing edge, moving, with vortices);
    the previous level has the vortices moved a little."""
    say(f"[pressure] plate with d(dphi)/dt, flags={flags}")
    case = wl.random_case(172, 128, 2.0 / 128, 300, surface="plate", mode="kutta")
    prev = wl.random_case(172, 128, 2.0 / 128, 300, surface="plate", mode="kutta")
    prev.X = wl.f32(prev.X - 0.01)
    nx, ny, closed = _normals(case)
    dt, rho = 0.01, 1.2
    got = _gpu(ctx, case, flags, nx, ny, closed, prev_case=prev, dt=dt, rho=rho)
    r0 = oracle_solve(problem_of(prev), body_of(prev))
    p0 = problem_of(prev)
    b0 = body_of(prev)
    dphi0 = pr.potential_jump(p0.grid, b0.xs, b0.ys, b0.ds, nx, ny, r0.f, closed)
    ref = _oracle_pressure(case, oracle_solve(problem_of(case), body_of(case)), nx, ny, closed,
                           dphi_prev=dphi0, dt=dt, rho=rho)
    _check(f"plate flags={flags}", got, ref, 1e-9 if flags == gpf.GPF_FP64 else 1e-4)


def test_pressure_needs_normals(ctx):
    case = wl.random_case(173, 64, 2.0 / 64, 20, surface="cylinder", mode="circulation")
    s = gpf.Solver(ctx, case.n, case.dx, case.surface, flags=gpf.GPF_FP64)
    X, Y, G = s.upload(case)
    inp = s.inputs_for(case, X, Y, G)
    z = torch.zeros(case.surface.ns, dtype=torch.float64, device=DEV)
    with pytest.raises(gpf.GpfError) as e:
        gpf.gpf_pressure(s.plan, s.body, inp, s.psi, s.f, z, z)
    assert e.value.status == gpf.GPF_E_INVALID


def test_two_cylinder_parts_pressure(ctx):
    """A body of two closed parts (one uniform direction removed per part),
    each with its own circulation, in a uniform flow with vortices."""
    say("[pressure] two cylinders as parts")
    from oracle.multibody import solve_multi
    from oracle.operators import regularize_vortices
    from tests.oracle_adapter import multi_of
    rng = np.random.default_rng(174)
    n, dx = 128, 2.0 / 128
    c1 = wl.cylinder(0.3, 75, center=(-0.45, 0.05))
    c2 = wl.cylinder(0.25, 63, center=(0.45, -0.1))
    pts = rng.uniform(-0.9, 0.9, size=(600, 2))
    keep = wl.outside_surface(c1, pts, 3 * dx) & wl.outside_surface(c2, pts, 3 * dx)
    pts = pts[keep][:300]
    mc = wl.MultiCase("two cylinders", n, dx, wl.f32(pts[:, 0]), wl.f32(pts[:, 1]),
                      wl.f32(rng.normal(0, 1e-2, len(pts))), [c1, c2],
                      [{"mode": "circulation", "gamma_b": 0.2},
                       {"mode": "circulation", "gamma_b": -0.1}], (), (), u_inf=1.0, v_inf=0.1)
    plan = gpf.Plan(ctx, n, dx, flags=gpf.GPF_FP64)
    body = gpf.Body(plan, mc.xs, mc.ys, mc.ds)
    body.set_parts(mc.part)
    nx, ny = np.r_[c1.nx, c2.nx], np.r_[c1.ny, c2.ny]
    body.set_normals(nx, ny, True)
    t = lambda a: torch.as_tensor(np.asarray(a), dtype=torch.float64).to(DEV)
    X, Y, G = t(mc.X), t(mc.Y), t(mc.G)
    ns = len(mc.xs)
    z = lambda k: torch.zeros(k, dtype=torch.float64, device=DEV)
    psi = torch.empty((n, n), dtype=torch.float64, device=DEV)
    f, sc, status = z(ns), z(gpf.N_SCALARS), torch.zeros(1, dtype=torch.int32, device=DEV)
    inp = gpf.make_parts_inputs(X, Y, G, mc.parts, u_inf=mc.u_inf, v_inf=mc.v_inf)
    out = gpf.make_outputs(psi, None, None, f, None, sc, status)
    gpf.gpf_solve(plan, body, inp, out)
    dphi, dp, P, side = z(ns), z(ns), z(n * n), z(2 * ns)
    gpf.gpf_pressure(plan, body, inp, psi, f, dphi, dp, P, side)
    gpf.gpf_sync(status)
    got = (dphi.cpu().numpy(), dp.cpu().numpy(), P.cpu().numpy().reshape(n, n)[:n - 1, :n - 1],
           side.cpu().numpy())
    p, ob, part = multi_of(mc)
    res = solve_multi(p, ob, part)
    odphi = pr.potential_jump(p.grid, ob.xs, ob.ys, ob.ds, nx, ny, res.f, True, part=part)
    zz = np.zeros(ns)
    odp = pr.pressure_jump(p.grid, ob.xs, ob.ys, nx, ny, res.f, res.s, zz, zz, zz, 1.0,
                           mc.u_inf, mc.v_inf)
    w = regularize_vortices(p.grid, p.X, p.Y, p.G)
    oP = pr.grid_pressure(p.grid, w, res.s, ob.xs, ob.ys, ob.ds, nx, ny, res.f, zz, zz, zz, 1.0,
                          mc.u_inf, mc.v_inf)
    pc = pr.cell_interp(p.grid, ob.xs, ob.ys, oP)
    _check("two cylinders", got, (odphi, odp, oP, pc + 0.5 * odp, pc - 0.5 * odp), 1e-9)
