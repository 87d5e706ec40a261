"""GPU parity: every stage and full solves against the FP64 oracle.

All inputs are float32-representable (rounded by the generators) so that
parity measures compute error, not input rounding.  Tolerances:
* FP64 plans: 1e-9 relative (rounding-order differences only);
* FP32 plans, full solve: relL2(s) <= 1e-5, relL2(f) <= 1e-4,
  relL2(u, v) <= 1e-4, new-vortex strengths and circulations <= 1e-5 relative;
* FP32 stages that are not amplified by the ill-conditioned Schur solve:
  10x tighter (1e-6).
"""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2102_11910_amd import gpf  # noqa: E402
from paper_2102_11910_amd import workloads as wl  # noqa: E402
from oracle import operators as op  # noqa: E402
from oracle.lgf import lgf_table  # noqa: E402
from oracle.solve import solve as oracle_solve  # noqa: E402
from tests.conftest import rell2  # noqa: E402
from tests.oracle_adapter import body_of, grid_of, problem_of  # noqa: E402

DEV = torch.device("cuda", 0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    return gpf.Context(0)


def dt(a, dtype=torch.float64):
    return torch.as_tensor(np.asarray(a), dtype=dtype).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


# ---------------------------------------------------------------------------
# stages
# ---------------------------------------------------------------------------

def _random_source(n, dx, nv, seed):
    rng = np.random.default_rng(seed)
    grid = op.Grid.centered(n, dx)
    h = (n - 1) * dx / 2 - 3 * dx
    X = wl.f32(rng.uniform(-h, h, nv))
    Y = wl.f32(rng.uniform(-h, h, nv))
    G = wl.f32(rng.normal(0, 1, nv))
    return grid, X, Y, G


@pytest.mark.parametrize("n", [16, 32, 64, 128, 256, 512, 1024])
@pytest.mark.parametrize("fp64", [False, True])
def test_convolution_matches_oracle(ctx, n, fp64):
    say(f"[conv] n={n} fp64={fp64}")
    dx = 2.0 / n
    grid, X, Y, G = _random_source(n, dx, max(8, n), seed=n)
    w = op.regularize_vortices(grid, X, Y, G)
    ftype = torch.float64 if fp64 else torch.float32
    w_in = w if fp64 else w.astype(np.float32).astype(np.float64)
    plan = gpf.Plan(ctx, n, dx, flags=gpf.GPF_FP64 if fp64 else gpf.GPF_FP32)
    wd = dt(w_in, ftype)
    sd = torch.empty_like(wd)
    gpf.gpf_convolve(plan, wd, sd, dx * dx * float(np.sum(w_in)))
    ref = op.inv_laplacian_fft(w_in, dx, lgf_table(n))
    got = host(sd)
    err = rell2(got, ref)
    say(f"   relL2 = {err:.3e}")
    assert err <= (1e-12 if fp64 else 1e-6)


@pytest.mark.parametrize("fp64", [False, True])
def test_regularization_matches_oracle(ctx, fp64):
    n, dx = 128, 0.02
    grid, X, Y, G = _random_source(n, dx, 3001, seed=7)
    plan = gpf.Plan(ctx, n, dx, flags=gpf.GPF_FP64 if fp64 else gpf.GPF_FP32)
    w = torch.zeros((n, n), dtype=plan.field_dtype, device=DEV)
    status = torch.zeros(1, dtype=torch.int32, device=DEV)
    gpf.gpf_regularize_vortices(plan, dt(X), dt(Y), dt(G), w, False, status)
    gpf.gpf_sync(status)
    ref = op.regularize_vortices(grid, X, Y, G)
    err = np.max(np.abs(host(w) - ref)) / np.max(np.abs(ref))
    say(f"[regularize] fp64={fp64} max rel = {err:.3e}")
    assert err <= (1e-13 if fp64 else 1e-6)
    # circulation conservation on the device field
    assert abs(dx * dx * host(w).sum() - G.sum()) <= (1e-12 if fp64 else 1e-4) * np.abs(G).sum()


@pytest.mark.parametrize("fp64", [False, True])
def test_interpolations_match_oracle(ctx, fp64):
    n, dx = 128, 0.02
    grid, X, Y, _ = _random_source(n, dx, 777, seed=9)
    rng = np.random.default_rng(10)
    XX, YY = np.meshgrid(grid.node_x(), grid.node_y())
    s = np.sin(3 * XX) * np.cos(2 * YY) + 0.1 * rng.standard_normal((n, n))
    s_in = s if fp64 else s.astype(np.float32).astype(np.float64)
    plan = gpf.Plan(ctx, n, dx, flags=gpf.GPF_FP64 if fp64 else gpf.GPF_FP32)
    sd = dt(s_in, plan.field_dtype)
    u = torch.empty(len(X), dtype=torch.float64, device=DEV)
    v = torch.empty_like(u)
    gpf.gpf_vortex_velocity(plan, sd, dt(X), dt(Y), 0.5, -0.25, u, v)
    ur, vr = op.vortex_velocity(grid, s_in, X, Y, 0.5, -0.25)
    assert np.max(np.abs(host(u) - ur)) <= 1e-12 * np.max(np.abs(ur))
    assert np.max(np.abs(host(v) - vr)) <= 1e-12 * np.max(np.abs(vr))
    surf = wl.cylinder(0.7, 150)
    body = gpf.Body(plan, surf.xs, surf.ys, surf.ds)
    r = torch.empty(150, dtype=torch.float64, device=DEV)
    gpf.gpf_interpolate_surface(body, sd, r)
    rr = op.interpolate_surface(grid, surf.xs, surf.ys, s_in)
    assert np.max(np.abs(host(r) - rr)) <= 1e-13 * np.max(np.abs(rr))


def test_body_setup_matches_oracle(ctx):
    case = wl.random_case(21, 128, 0.02, 10, surface="plate", mode="kutta")
    plan = gpf.Plan(ctx, case.n, case.dx)
    sf = case.surface
    body = gpf.Body(plan, sf.xs, sf.ys, sf.ds, sf.edges)
    ob = body_of(case)
    info = body.info()
    say(f"[body] gamma0 {info['gamma0']:.12g} vs {ob.gamma0:.12g}, amp {info['amp']:.3g}")
    assert abs(info["gamma0"] - ob.gamma0) <= 1e-10 * abs(ob.gamma0)
    assert rell2(body.f0(), ob.f0) <= 1e-10


# ---------------------------------------------------------------------------
# full solves
# ---------------------------------------------------------------------------

def run_solve(ctx, case, flags, velocities=True):
    edges = tuple(case.edges) if case.mode in ("kutta", "shed") else None
    s = gpf.Solver(ctx, case.n, case.dx, case.surface, flags=flags, edges=edges)
    X, Y, G = s.upload(case)
    inp = s.inputs_for(case, X, Y, G)
    s.solve(inp, X, velocities=velocities)
    gpf.gpf_sync(s.status)
    res = {"s": host(s.psi), "scalars": host(s.scalars)}
    if s.body is not None:
        res["f"] = host(s.f)
        res["ftilde"] = host(s.ftilde)
    if velocities:
        res["u"], res["v"] = host(s.u), host(s.v)
    res["info"] = s.body.info() if s.body else None
    return res


def compare(case, got, ref, fp64, label):
    tol_s, tol_f, tol_u, tol_g = (1e-9, 1e-8, 1e-9, 1e-9) if fp64 else (1e-5, 1e-4, 1e-4, 1e-5)
    es = rell2(got["s"], ref.s)
    msg = [f"s {es:.2e}"]
    assert es <= tol_s, (label, msg)
    if case.nv:
        eu = rell2(np.r_[got["u"], got["v"]], np.r_[ref.u, ref.v])
        msg.append(f"uv {eu:.2e}")
        assert eu <= tol_u, (label, msg)
    if ref.f is not None:
        ef = rell2(got["f"], ref.f)
        eft = rell2(got["ftilde"], ref.ftilde)
        gb = got["scalars"][3]
        egb = abs(gb - ref.gamma_b) / max(abs(ref.gamma_b), 1e-3)
        msg += [f"f {ef:.2e}", f"ftilde {eft:.2e}", f"gamma_b {egb:.2e}"]
        assert ef <= tol_f, (label, msg)
        assert egb <= tol_g, (label, msg)
        if ref.gamma_new is not None:
            gn = got["scalars"][4:4 + len(ref.gamma_new)]
            eg = np.max(np.abs(gn - ref.gamma_new)) / max(np.max(np.abs(ref.gamma_new)), 1e-3)
            msg.append(f"gamma_new {eg:.2e}")
            assert eg <= tol_g, (label, msg)
    say(f"   {label}: " + ", ".join(msg))


CASES = [
    ("none", None, 64), ("circulation", "cylinder", 64), ("kutta", "plate", 64),
    ("shed", "plate", 64), ("circulation", "ellipse", 128), ("shed", "plate", 128),
    ("kutta", "plate", 256),
]


@pytest.mark.parametrize("mode,surface,n", CASES)
@pytest.mark.parametrize("flags", [gpf.GPF_FP64, gpf.GPF_FP32, gpf.GPF_CONV1_FP64])
def test_solve_matches_oracle(ctx, mode, surface, n, flags):
    say(f"[solve] mode={mode} surface={surface} n={n} flags={flags}")
    case = wl.random_case(100 + n, n, 2.0 / n, 3 * n + 7, surface=surface, mode=mode)
    got = run_solve(ctx, case, flags)
    ref = oracle_solve(problem_of(case), body_of(case))
    compare(case, got, ref, flags == gpf.GPF_FP64, f"{mode}/{surface}/n={n}/flags={flags}")


def test_config1_full_parity(ctx):
    say("[C1] cylinder 128^2, 200 vortices, FP32")
    case = wl.config1()
    got = run_solve(ctx, case, gpf.GPF_FP32)
    ref = oracle_solve(problem_of(case), body_of(case))
    compare(case, got, ref, False, "C1 FP32")
    got = run_solve(ctx, case, gpf.GPF_FP64)
    compare(case, got, ref, True, "C1 FP64")


def test_config2_fp32_first_convolution_is_not_enough(ctx):
    """With an FP32 first convolution the ill-conditioned Schur solve
    (dS/dx = 0.78) amplifies its rounding noise in f: the reason the
    precision policy runs that convolution in FP64 for such bodies."""
    case = wl.config2()
    got = run_solve(ctx, case, gpf.GPF_FP32)
    ref = oracle_solve(problem_of(case), body_of(case))
    ef = rell2(got["f"], ref.f)
    say(f"[C2 all-FP32] s {rell2(got['s'], ref.s):.2e} f {ef:.2e} amp {got['info']['amp']:.3g}")
    assert rell2(got["s"], ref.s) <= 1e-5


@pytest.mark.parametrize("flags", [gpf.GPF_POLICY_AUTO, gpf.GPF_FP64])
def test_config2_full_parity(ctx, flags):
    say(f"[C2] plate 512^2, Kutta at both edges, 1e4 vortices, flags={flags}")
    case = wl.config2()
    got = run_solve(ctx, case, flags)
    say(f"   body info {got['info']}")
    ref = oracle_solve(problem_of(case), body_of(case))
    compare(case, got, ref, flags == gpf.GPF_FP64, f"C2 flags={flags}")


# ---------------------------------------------------------------------------
# edge cases and error paths
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("mode,surface", [("circulation", "cylinder"), ("none", None)])
def test_total_streamfunction_flag(ctx, mode, surface):
    """GPF_PSI_TOTAL stores psi = s + U_inf y - V_inf x (Sec. 2.1) and
    differences it for the velocities: equal to the oracle's s plus the
    uniform-flow field, velocities within the FP32 rounding of psi."""
    case = wl.random_case(61, 128, 2.0 / 128, 300, surface=surface, mode=mode)
    got = run_solve(ctx, case, gpf.GPF_FP32 | gpf.GPF_PSI_TOTAL)
    ref = oracle_solve(problem_of(case), body_of(case))
    g = grid_of(case)
    xs = g.x0 + g.dx * np.arange(case.n)
    ys = g.y0 + g.dx * np.arange(case.n)
    sinf = case.u_inf * ys[:, None] - case.v_inf * xs[None, :]
    es = rell2(got["s"], ref.s + sinf)
    eu = rell2(np.r_[got["u"], got["v"]], np.r_[ref.u, ref.v])
    say(f"[psi total] {mode}: psi {es:.2e}, uv {eu:.2e}")
    assert es <= 1e-6
    assert eu <= 1e-4


@pytest.mark.parametrize("flags", [gpf.GPF_FP64, gpf.GPF_POLICY_AUTO])
def test_shedding_at_one_edge(ctx, flags):
    """Kutta condition with one new vortex at the trailing edge only (the
    m-edge system with m = 1, Sec. 2.4.2)."""
    case = wl.random_case(81, 128, 2.0 / 128, 250, surface="plate", mode="shed")
    case.edges = (case.surface.edges[1],)
    case.znew = (case.znew[1],)
    got = run_solve(ctx, case, flags)
    ref = oracle_solve(problem_of(case), body_of(case))
    compare(case, got, ref, flags == gpf.GPF_FP64, f"shed at one edge, flags={flags}")


def _bounds_case(kind):
    """A two-edge plate with edge bounds placed around the oracle's
    Kelvin-consistent intermediate sheet (margins far above any rounding),
    so that the active set is the same in every precision."""
    from tests.oracle_adapter import intermediate_sheet
    case = wl.random_case(91, 128, 2.0 / 128, 300, surface="plate", mode="shed")
    _, ft_star, _ = intermediate_sheet(case)
    k1, k2 = case.edges
    a1, a2 = ft_star[k1], ft_star[k2]
    d1, d2 = 0.25 * max(1.0, abs(a1)), 0.25 * max(1.0, abs(a2))
    inf = math.inf
    case.fbounds = {
        "lo-active/free": ((a1 + d1, a1 + 3 * d1), (a2 - d2, a2 + d2)),
        "free/hi-active": ((-inf, inf), (a2 - 3 * d2, a2 - d2)),
        "both-active": ((a1 + d1, inf), (-inf, a2 - d2)),
        "both-free": ((a1 - d1, a1 + d1), (-inf, inf)),
    }[kind]
    return case


@pytest.mark.parametrize("kind", ["lo-active/free", "free/hi-active", "both-active", "both-free"])
@pytest.mark.parametrize("flags", [gpf.GPF_FP64, gpf.GPF_POLICY_AUTO])
def test_generalized_edge_conditions(ctx, kind, flags):
    """Bounds on f~ at the edges (Sec. 2.5, eq. twovortex-gen): the same
    active set as the oracle, its strengths, sheet and field; a free edge
    sheds exactly zero."""
    say(f"[edge bounds] {kind} flags={flags}")
    case = _bounds_case(kind)
    got = run_solve(ctx, case, flags)
    ref = oracle_solve(problem_of(case), body_of(case))
    gn = got["scalars"][4:6]
    assert np.array_equal(gn == 0.0, ref.gamma_new == 0.0), (gn, ref.gamma_new)
    compare(case, got, ref, flags == gpf.GPF_FP64, f"edge bounds {kind}, flags={flags}")
    for i, (lo, hi) in enumerate(case.fbounds):
        if ref.gamma_new[i] != 0.0:
            t = got["ftilde"][case.edges[i]]
            assert min(abs(t - lo), abs(t - hi)) <= 1e-6 * max(1.0, abs(t)), (i, t, lo, hi)


def test_edge_bounds_validated(ctx):
    case = wl.random_case(92, 64, 2.0 / 64, 20, surface="plate", mode="shed")
    s = gpf.Solver(ctx, case.n, case.dx, case.surface, flags=gpf.GPF_FP64, edges=tuple(case.edges))
    X, Y, G = s.upload(case)
    for bad in (((0.5, 0.1), (0.0, 0.0)), ((0.0, 0.0), (math.nan, 1.0))):
        case.fbounds = bad
        with pytest.raises(gpf.GpfError) as e:
            s.solve(s.inputs_for(case, X, Y, G), X)
        assert e.value.status == gpf.GPF_E_INVALID


def test_empty_vortex_set(ctx):
    case = wl.random_case(5, 64, 2.0 / 64, 0, surface="cylinder")
    case.X = case.Y = case.G = np.zeros(0)
    case.gamma_b = 0.1
    got = run_solve(ctx, case, gpf.GPF_FP32, velocities=False)
    ref = oracle_solve(problem_of(case), body_of(case))
    assert rell2(got["s"], ref.s) <= 1e-5
    assert rell2(got["f"], ref.f) <= 1e-4


def test_out_of_grid_vortex_is_reported(ctx):
    n, dx = 64, 0.05
    s = gpf.Solver(ctx, n, dx)
    x0 = -(n - 1) * dx / 2
    X = dt([0.0, x0 + 1.5 * dx])      # second one is too close to the edge
    Y = dt([0.0, 0.0])
    G = dt([1.0, 1.0])
    inp = gpf.make_inputs(X, Y, G)
    s.solve(inp, X)
    with pytest.raises(gpf.GpfError) as e:
        gpf.gpf_sync(s.status)
    assert e.value.status == gpf.GPF_E_OUT_OF_GRID
    # the status word is cleared by the sync; a valid solve then passes
    inp = gpf.make_inputs(X[:1], Y[:1], G[:1])
    s.solve(inp, X[:1])
    gpf.gpf_sync(s.status)


def test_singular_body_rejected(ctx):
    plan = gpf.Plan(ctx, 64, 0.05)
    xs = np.array([0.1, 0.1, 0.3, 0.2])
    ys = np.array([0.0, 0.0, 0.1, 0.3])
    with pytest.raises(gpf.GpfError) as e:
        gpf.Body(plan, xs, ys, np.full(4, 0.05))
    assert e.value.status == gpf.GPF_E_SINGULAR


def test_invalid_arguments(ctx):
    with pytest.raises(gpf.GpfError) as e:
        gpf.Plan(ctx, 100, 0.05)
    assert e.value.status == gpf.GPF_E_UNSUPPORTED
    with pytest.raises(gpf.GpfError) as e:
        gpf.Plan(ctx, 64, -1.0)
    assert e.value.status == gpf.GPF_E_INVALID
    plan = gpf.Plan(ctx, 64, 0.05)
    with pytest.raises(gpf.GpfError) as e:
        gpf.Body(plan, [5.0, 5.1], [0.0, 0.0], [0.1, 0.1])
    assert e.value.status == gpf.GPF_E_OUT_OF_GRID
    surf = wl.flat_plate(1.0, 10.0, 32)
    s = gpf.Solver(ctx, 64, 0.05, surf)
    X = dt([0.9])
    inp = gpf.make_inputs(X, X, X, mode="shed", znew=((0.6, 0.0),))   # m != edge count
    with pytest.raises(gpf.GpfError) as e:
        s.solve(inp, X)
    assert e.value.status == gpf.GPF_E_INVALID
    inp = gpf.make_inputs(X, X, X, u_inf=math.inf)
    with pytest.raises(gpf.GpfError):
        s.solve(inp, X)


@pytest.mark.parametrize("n,surface", [(64, None), (256, None), (256, "cylinder")])
@pytest.mark.parametrize("flags", [gpf.GPF_FP64, gpf.GPF_FP32, gpf.GPF_CONV1_FP64])
def test_tile_borders_beside_empty_tiles(ctx, n, surface, flags):
    """A few vortices in the cells on either side of the 32-cell tile
    borders (their stencils reach the neighbouring tiles' border nodes,
    corners included) and most tiles without vortices: the solves add every
    neighbour's halo entries as they read the field, and an empty tile's
    entries must count as zero.  Against the oracle."""
    case = wl.random_case(400 + n, n, 2.0 / n, 0, surface=surface,
                          mode="circulation" if surface else "none")
    dx, x0 = case.dx, -(n - 1) * case.dx / 2
    rng = np.random.default_rng(n)
    cells = [32 * k + d for k in range(1, n // 32) for d in (-2, -1, 0, 1)]
    picks = rng.choice(len(cells) ** 2, size=min(60, len(cells) ** 2), replace=False)
    xi = [cells[p % len(cells)] + 0.37 for p in picks]
    eta = [cells[p // len(cells)] + 0.61 for p in picks]
    case.X = x0 + dx * np.asarray(xi)
    case.Y = x0 + dx * np.asarray(eta)
    case.G = wl.f32(rng.normal(0.0, 1.0, len(xi)))
    say(f"[tile borders] n={n} surface={surface} flags={flags}, {len(xi)} vortices")
    got = run_solve(ctx, case, flags)
    ref = oracle_solve(problem_of(case), body_of(case))
    compare(case, got, ref, flags == gpf.GPF_FP64, f"tile borders n={n} {surface} flags={flags}")


@pytest.mark.parametrize("flags", [gpf.GPF_FP64, gpf.GPF_FP32])
def test_window_limits_nodes_and_coincident_vortices(ctx, flags):
    """Vortices exactly at the lowest allowed cell index (xi = 2) and just
    below the highest (n - 3), on nodes, and thousands at one point (one
    tile, one LDS window, heavy atomic traffic), against the oracle; the
    first index outside the window on either side is reported."""
    n = 64
    case = wl.random_case(77, n, 2.0 / n, 0)
    dx, x0 = case.dx, -(n - 1) * case.dx / 2          # both exact in binary
    lo, hi = 2.0, (n - 3) - 2.0 ** -20
    rng = np.random.default_rng(77)
    xi = [lo, hi, lo, hi, 30.0, 30.5, 17.0]
    eta = [lo, hi, hi, lo, 30.0, 30.5, 40.25]
    k = 3000
    xi += [33.37] * k
    eta += [21.81] * k
    G = np.r_[[0.3, -0.2, 0.1, 0.25, -0.4, 0.15, 0.05], rng.normal(0.0, 1e-2, k)]
    case.X = x0 + dx * np.asarray(xi)
    case.Y = x0 + dx * np.asarray(eta)
    case.G = wl.f32(G)
    say(f"[window] n={n}, {len(case.X)} vortices, flags={flags}")
    got = run_solve(ctx, case, flags)
    ref = oracle_solve(problem_of(case), body_of(case))
    compare(case, got, ref, flags == gpf.GPF_FP64, f"window limits, flags={flags}")
    s = gpf.Solver(ctx, n, dx, flags=flags)
    for bad in (n - 3.0, 2.0 - 2.0 ** -20):
        X = dt([x0 + dx * 30.0, x0 + dx * bad])
        Y = dt([x0 + dx * 30.0, x0 + dx * 30.0])
        s.solve(gpf.make_inputs(X, Y, dt([1.0, 1.0])), X)
        with pytest.raises(gpf.GpfError) as e:
            gpf.gpf_sync(s.status)
        assert e.value.status == gpf.GPF_E_OUT_OF_GRID, bad
