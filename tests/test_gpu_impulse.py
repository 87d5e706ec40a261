"""Impulse, added mass and body geometry on the GPU against the oracle
(eqs. linimpxd, linimpyd, angimpd; Sec. 2.6.3; eq. centroid)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2102_11910_amd import gpf  # noqa: E402
from paper_2102_11910_amd import workloads as wl  # noqa: E402
from oracle.impulse import added_mass, solution_impulse, volume_centroid  # noqa: E402
from oracle.solve import solve as oracle_solve  # noqa: E402
from tests.oracle_adapter import body_of, problem_of  # noqa: E402

DEV = torch.device("cuda", 0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    return gpf.Context(0)


def _solve_with_impulse(ctx, case, flags):
    edges = tuple(case.edges) if case.mode in ("kutta", "shed") else None
    s = gpf.Solver(ctx, case.n, case.dx, case.surface, flags=flags, edges=edges)
    if s.body is not None and case.surface.nx is not None:
        s.body.set_normals(case.surface.nx, case.surface.ny)
    X, Y, G = s.upload(case)
    inp = s.inputs_for(case, X, Y, G)
    imp = torch.zeros(3, dtype=torch.float64, device=DEV)
    out = gpf.make_outputs(s.psi, None, None, s.f if s.body else None,
                           s.ftilde if s.body else None, s.scalars, s.status, imp)
    gpf.gpf_solve(s.plan, s.body, inp, out)
    gpf.gpf_sync(s.status)
    return imp.cpu().numpy()


@pytest.mark.parametrize("mode,surface", [("circulation", "cylinder"), ("circulation", "ellipse"),
                                          ("shed", "plate"), ("kutta", "plate"), ("none", None)])
@pytest.mark.parametrize("flags", [gpf.GPF_FP64, gpf.GPF_POLICY_AUTO])
def test_impulse_matches_oracle(ctx, mode, surface, flags):
    """Moving bodies in a uniform flow (relative motion term), new vortices
    of the shedding mode, and vortices alone."""
    say(f"[impulse] {mode}/{surface} flags={flags}")
    case = wl.random_case(150, 128, 2.0 / 128, 400, surface=surface, mode=mode)
    got = _solve_with_impulse(ctx, case, flags)
    p, body = problem_of(case), body_of(case)
    res = oracle_solve(p, body)
    sf = case.surface
    ref = solution_impulse(p, body, res, None if sf is None else sf.nx,
                           None if sf is None else sf.ny)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    say(f"   impulse {got} vs {ref}: {err:.2e}")
    assert err <= (1e-9 if flags == gpf.GPF_FP64 else 1e-5)


@pytest.mark.parametrize("surface", ["cylinder", "ellipse", "plate"])
def test_added_mass_and_geometry_match_oracle(ctx, surface):
    say(f"[added mass] {surface}")
    case = wl.random_case(151, 128, 2.0 / 128, 10, surface=surface)
    sf = case.surface
    plan = gpf.Plan(ctx, case.n, case.dx, flags=gpf.GPF_FP64)
    body = gpf.Body(plan, sf.xs, sf.ys, sf.ds)
    ob = body_of(case)
    if sf.nx is not None:
        body.set_normals(sf.nx, sf.ny)
        V, xc, yc = body.geometry()
        rV, rxc, ryc = volume_centroid(sf.xs, sf.ys, sf.ds, sf.nx, sf.ny)
        assert abs(V - rV) <= 1e-12 * abs(rV) and abs(xc - rxc) <= 1e-12 and abs(yc - ryc) <= 1e-12
    M = body.added_mass(1.3)
    ref = added_mass(ob, sf.nx, sf.ny, rho=1.3)
    err = np.max(np.abs(M - ref)) / np.max(np.abs(ref))
    say(f"   added mass err {err:.2e}\n{M}")
    assert err <= 1e-9


def test_impulse_needs_the_sheet(ctx):
    case = wl.random_case(152, 64, 2.0 / 64, 10, surface="cylinder")
    s = gpf.Solver(ctx, case.n, case.dx, case.surface, flags=gpf.GPF_FP64)
    X, Y, G = s.upload(case)
    inp = s.inputs_for(case, X, Y, G)
    imp = torch.zeros(3, dtype=torch.float64, device=DEV)
    out = gpf.make_outputs(s.psi, None, None, None, None, s.scalars, s.status, imp)
    with pytest.raises(gpf.GpfError) as e:
        gpf.gpf_solve(s.plan, s.body, inp, out)
    assert e.value.status == gpf.GPF_E_INVALID
