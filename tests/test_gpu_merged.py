"""Batches of several grid sizes run merged: every stage of the solve is one
launch per precision of the first convolution over all grid sizes, and the
FP32 transform passes take their blocks from one work list (largest grids
first).  Each problem must equal the same problem solved in the grouped
path (one launch sequence per configuration) and alone, within the FP32
reordering of atomic additions, and meet the oracle tolerances."""
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


def _edge_case(seed, n, top):
    """A small cylinder whose surface stencils reach the first (top=False)
    or last (top=True) rows a body may use: the band of the first
    convolution then sits at the window's edge, where the workgroups of
    small grids (32 or 64 rows) reach past it."""
    dx = 2.0 / n
    rng = np.random.default_rng(seed)
    half = (n - 1) * dx / 2.0
    r = 4.0 * dx
    cy = (half - 3.5 * dx - r) * (1.0 if top else -1.0)
    surf = wl.cylinder(r, 16, center=(0.1 * half, cy))
    cloud = wl._uniform_cloud(rng, 80, half - 4.0 * dx, surf, 2.0 * dx)
    X, Y = wl.f32(cloud[:, 0]), wl.f32(cloud[:, 1])
    G = wl.f32(rng.normal(0.0, 1e-2, size=80))
    return wl.Case(f"edge band n={n} {'top' if top else 'bottom'}", n, dx, X, Y, G, surf,
                   u_inf=1.0, v_inf=0.1, mode="circulation", gamma_b=float(-np.sum(G)))


def mixed_sizes():
    """Every grid size of the merged passes, every one-part mode, both first
    convolution precisions (the 512^2 plate's noise amplification takes its
    first convolution to FP64 under GPF_POLICY_AUTO) and repeated sizes."""
    return [
        wl.random_case(201, 2048, 2.56 / 2048, 4000, surface="cylinder", ns=700),
        wl.random_case(202, 1024, 2.56 / 1024, 3000, surface="plate", mode="shed"),
        wl.config2(seed=203, nv=2500),
        wl.random_case(204, 512, 2.56 / 512, 1500, surface="ellipse"),
        wl.random_case(205, 256, 2.56 / 256, 900, surface="plate", mode="kutta"),
        wl.random_case(206, 128, 2.0 / 128, 400, surface="cylinder"),
        wl.random_case(207, 128, 2.0 / 128, 333, surface="ellipse"),
        wl.random_case(208, 64, 2.0 / 64, 90, surface="plate", mode="shed"),
        _edge_case(209, 64, True),
        _edge_case(210, 128, False),
        _edge_case(211, 128, True),
    ]


class Setup:
    def __init__(self, ctx, cases, total_psi_for=()):
        self.cases = cases
        self.plans, self.bodies, self.ins, self.keep = [], [], [], []
        plans = {}
        for i, c in enumerate(cases):
            flags = gpf.GPF_POLICY_AUTO | (gpf.GPF_PSI_TOTAL if i in total_psi_for else 0)
            key = (c.n, c.dx, flags)
            if key not in plans:
                plans[key] = gpf.Plan(ctx, c.n, c.dx, flags=flags)
            p = plans[key]
            sf = c.surface
            edges = tuple(c.edges) if c.mode in ("kutta", "shed") else ()
            self.plans.append(p)
            self.bodies.append(gpf.Body(p, sf.xs, sf.ys, sf.ds, edges))
            X, Y, G = (torch.as_tensor(a, dtype=torch.float64).to(DEV) for a in (c.X, c.Y, c.G))
            self.keep.append((X, Y, G))
            self.ins.append(gpf.make_inputs(X, Y, G, c.u_inf, c.v_inf, c.ub, c.vb, c.omega, c.mode,
                                            c.gamma_b, c.znew))
        self._plans = plans

    def outputs(self):
        return [gpf.Outputs(c.n, c.nv, c.surface.ns) for c in self.cases]


def _host(o):
    torch.cuda.synchronize()
    return {"s": o.psi.double().cpu().numpy(), "f": o.f.cpu().numpy(),
            "uv": np.r_[o.u.cpu().numpy(), o.v.cpu().numpy()]}


def _compare(a, b, tag):
    es, ef, eu = rell2(a["s"], b["s"]), rell2(a["f"], b["f"]), rell2(a["uv"], b["uv"])
    msg = f"{tag}: s {es:.1e} f {ef:.1e} uv {eu:.1e}"
    say(msg)
    assert es <= 1e-6 and ef <= 1e-5 and eu <= 1e-5, msg


def test_merged_equals_grouped_alone_and_oracle(ctx):
    cases = mixed_sizes()
    st = Setup(ctx, cases, total_psi_for=(3,))
    say(f"[merged] sizes {[c.n for c in cases]}, FP64 first convolution: "
        f"{[i for i, b in enumerate(st.bodies) if b.info()['conv1_fp64']]}")
    assert any(b.info()["conv1_fp64"] for b in st.bodies)
    merged = gpf.Batch(ctx, len(cases))
    grouped = gpf.Batch(ctx, len(cases), merge=False)
    om, og = st.outputs(), st.outputs()
    for rep in range(2):   # the second call reuses the zeroed workspaces
        for o in om:
            o.psi.fill_(float("nan"))
        merged.solve(st.plans, st.bodies, st.ins, [o.struct for o in om])
        for o in om:
            gpf.gpf_sync(o.status)
    grouped.solve(st.plans, st.bodies, st.ins, [o.struct for o in og])
    for o in og:
        gpf.gpf_sync(o.status)
    for i, c in enumerate(cases):
        oa = gpf.Outputs(c.n, c.nv, c.surface.ns)
        gpf.gpf_solve(st.plans[i], st.bodies[i], st.ins[i], oa.struct)
        gpf.gpf_sync(oa.status)
        hm = _host(om[i])
        _compare(hm, _host(og[i]), f"[merged vs grouped] {c.name}")
        _compare(hm, _host(oa), f"[merged vs alone] {c.name}")
        if c.n <= 512:
            ref = oracle_solve(problem_of(c), body_of(c))
            s_ref = ref.s
            if i == 3:   # total streamfunction stored: psi = s + U_inf y - V_inf x
                grid_x = -(c.n - 1) * c.dx / 2 + c.dx * np.arange(c.n)
                s_ref = ref.s + c.u_inf * grid_x[:, None] - c.v_inf * grid_x[None, :]
            es, ef = rell2(hm["s"], s_ref), rell2(hm["f"], ref.f)
            eu = rell2(hm["uv"], np.r_[ref.u, ref.v])
            say(f"   oracle: s {es:.2e} f {ef:.2e} uv {eu:.2e}")
            assert es <= 1e-5 and ef <= 1e-4 and eu <= 1e-4


def test_merged_batch_graph_replays(ctx):
    """A merged batch captured into a graph replays the eager result, with
    eager work and synchronizations between replays."""
    cases = [wl.random_case(221, 512, 2.56 / 512, 700, surface="cylinder"),
             wl.random_case(222, 256, 2.56 / 256, 500, surface="plate", mode="shed"),
             wl.random_case(223, 128, 2.0 / 128, 300, surface="ellipse"),
             wl.random_case(224, 128, 2.0 / 128, 200, surface="plate", mode="kutta")]
    st = Setup(ctx, cases)
    batch = gpf.Batch(ctx, len(cases))
    outs = st.outputs()
    structs = [o.struct for o in outs]
    batch.solve(st.plans, st.bodies, st.ins, structs)
    for o in outs:
        gpf.gpf_sync(o.status)
    eager = [_host(o) for o in outs]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        batch.solve(st.plans, st.bodies, st.ins, structs, stream=stream)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        batch.solve(st.plans, st.bodies, st.ins, structs, stream=stream)
    for rep in range(3):
        for o in outs:
            o.psi.fill_(0.0)
        g.replay()
        torch.cuda.synchronize()
        for i, o in enumerate(outs):
            _compare(_host(o), eager[i], f"[merged graph replay {rep}] {cases[i].name}")
        batch.solve(st.plans, st.bodies, st.ins, structs)
        for o in outs:
            gpf.gpf_sync(o.status)


def test_side_stream_same_bits_and_graph(ctx):
    """A merged batch with both first-convolution precisions: the FP64 class
    on the batch's side stream (merge 1, the default) gives the same bits as
    every kernel on the caller's stream (merge 2), and the grouped path
    (merge 0) agrees within tolerance; a graph captured with the side stream
    forked and joined replays the eager bits, with eager work and
    synchronizations between replays; merge values outside 0..2 are refused."""
    cases = [wl.config2(seed=271, nv=2500),
             wl.random_case(272, 256, 2.56 / 256, 900, surface="plate", mode="kutta"),
             wl.random_case(273, 128, 2.0 / 128, 400, surface="cylinder"),
             _with_dense_cluster(wl.random_case(274, 128, 2.0 / 128, 500, surface="ellipse"), 2000, 274)]
    st = Setup(ctx, cases)
    fp64 = [b.info()["conv1_fp64"] for b in st.bodies]
    say(f"[side stream] FP64 first convolution: {fp64}")
    assert any(fp64) and not all(fp64)
    res = {}
    for m in (1, 2, 0):
        batch = gpf.Batch(ctx, len(cases), merge=m)
        outs = st.outputs()
        batch.solve(st.plans, st.bodies, st.ins, [o.struct for o in outs])
        for o in outs:
            gpf.gpf_sync(o.status)
        res[m] = [_host(o) for o in outs]
        batch.close()
    for i, c in enumerate(cases):
        same = all(np.array_equal(res[1][i][k], res[2][i][k]) for k in res[1][i])
        say(f"[side stream vs one stream] {c.name}: bit-identical {same}")
        assert same, c.name
        _compare(res[1][i], res[0][i], f"[side stream vs grouped] {c.name}")
    batch = gpf.Batch(ctx, len(cases))
    outs = st.outputs()
    structs = [o.struct for o in outs]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        batch.solve(st.plans, st.bodies, st.ins, structs, stream=stream)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        batch.solve(st.plans, st.bodies, st.ins, structs, stream=stream)
    for rep in range(3):
        for o in outs:
            o.psi.fill_(0.0)
        g.replay()
        torch.cuda.synchronize()
        for i, o in enumerate(outs):
            h = _host(o)
            same = all(np.array_equal(h[k], res[1][i][k]) for k in h)
            say(f"[side stream graph replay {rep}] {cases[i].name}: bit-identical {same}")
            assert same, cases[i].name
        batch.solve(st.plans, st.bodies, st.ins, structs)
        for o in outs:
            gpf.gpf_sync(o.status)
    for bad in (-1, 3):
        with pytest.raises(gpf.GpfError):
            batch.set_merge(bad)


def test_dense_clouds_velocity_tiles(ctx):
    """Clouds of at least one vortex per four nodes take the tile-by-tile
    velocity kernel (the field window of a tile through LDS): alone, in a
    merged batch with sparse problems, and against the oracle."""
    cases = [wl.random_case(231, 128, 2.0 / 128, 6000, surface="cylinder"),
             wl.random_case(232, 64, 2.0 / 64, 2500, surface="plate", mode="shed"),
             wl.random_case(233, 256, 2.56 / 256, 300, surface="ellipse")]
    st = Setup(ctx, cases)
    batch = gpf.Batch(ctx, len(cases))
    outs = st.outputs()
    batch.solve(st.plans, st.bodies, st.ins, [o.struct for o in outs])
    for o in outs:
        gpf.gpf_sync(o.status)
    for i, c in enumerate(cases):
        oa = gpf.Outputs(c.n, c.nv, c.surface.ns)
        gpf.gpf_solve(st.plans[i], st.bodies[i], st.ins[i], oa.struct)
        gpf.gpf_sync(oa.status)
        hm = _host(outs[i])
        _compare(hm, _host(oa), f"[dense batch vs alone] {c.name} nv={c.nv}")
        ref = oracle_solve(problem_of(c), body_of(c))
        eu = rell2(hm["uv"], np.r_[ref.u, ref.v])
        es = rell2(hm["s"], ref.s)
        say(f"   oracle: s {es:.2e} uv {eu:.2e} (vortices per node {c.nv / c.n ** 2:.2f})")
        assert es <= 1e-5 and eu <= 1e-4


def _cluster_case(seed, n, nv, center, radius):
    """All vortices in a disc a few cells across: one or a few tiles hold
    thousands of records, which their R_v workgroups take 512 at a time."""
    dx = 2.56 / n
    rng = np.random.default_rng(seed)
    r = radius * np.sqrt(rng.uniform(0.0, 1.0, nv))
    th = rng.uniform(0.0, 2.0 * np.pi, nv)
    X, Y = wl.f32(center[0] + r * np.cos(th)), wl.f32(center[1] + r * np.sin(th))
    G = wl.f32(rng.normal(0.0, 1e-3, size=nv))
    surf = wl.cylinder(0.2, 64)
    return wl.Case(f"cluster n={n} nv={nv}", n, dx, X, Y, G, surf, u_inf=1.0, v_inf=0.0,
                   mode="circulation", gamma_b=float(-np.sum(G)))


def test_dense_tiles_in_chunks(ctx):
    """Tiles of more than 512 vortices, whose workgroups take their records
    in several chunks: a uniform cloud of about 1200 per tile, one of
    exactly 512 and 513 per tile on average, and a tight cluster inside one
    tile (thousands of records); alone, merged, and against the oracle."""
    cases = [wl.random_case(241, 128, 2.0 / 128, 20000, surface="cylinder"),
             _cluster_case(242, 256, 4000, (0.6, -0.55), 6.0 * 2.56 / 256),
             _cluster_case(243, 256, 513, (-0.4, 0.5), 3.0 * 2.56 / 256),
             wl.random_case(244, 64, 2.0 / 64, 2100, surface="plate", mode="shed")]
    st = Setup(ctx, cases)
    batch = gpf.Batch(ctx, len(cases))
    outs = st.outputs()
    for rep in range(2):   # the second call reuses the cleared tile counts
        batch.solve(st.plans, st.bodies, st.ins, [o.struct for o in outs])
        for o in outs:
            gpf.gpf_sync(o.status)
    for i, c in enumerate(cases):
        oa = gpf.Outputs(c.n, c.nv, c.surface.ns)
        gpf.gpf_solve(st.plans[i], st.bodies[i], st.ins[i], oa.struct)
        gpf.gpf_sync(oa.status)
        hm = _host(outs[i])
        _compare(hm, _host(oa), f"[dense tiles batch vs alone] {c.name}")
        ref = oracle_solve(problem_of(c), body_of(c))
        es, ef = rell2(hm["s"], ref.s), rell2(hm["f"], ref.f)
        eu = rell2(hm["uv"], np.r_[ref.u, ref.v])
        say(f"   oracle: s {es:.2e} f {ef:.2e} uv {eu:.2e}")
        assert es <= 1e-5 and ef <= 1e-4 and eu <= 1e-4


def _with_dense_cluster(c, k, seed):
    """c plus k vortices within a few cells of a tile corner: that tile and
    its neighbours hold more than 512 vortices each (several chunks)."""
    rng = np.random.default_rng(seed)
    cx = c.x0 + c.dx * 64.0
    c.X = np.r_[c.X, wl.f32(cx + c.dx * rng.uniform(-3.0, 3.0, k))]
    c.Y = np.r_[c.Y, wl.f32(cx + c.dx * rng.uniform(-3.0, 3.0, k))]
    c.G = np.r_[c.G, wl.f32(rng.normal(0.0, 1e-2, k))]
    return c


def test_scattered_field_repeats_bit_for_bit(ctx):
    """R_v: the source field is the same bits on every call, whatever order
    the workgroups run in (sparse and dense clouds, one and several tiles per
    grid, tiles of several chunks of records, overwrite and accumulate), and
    for the vortices given in another order."""
    cases = [wl.random_case(251, 512, 2.56 / 512, 20000, surface="ellipse"),
             wl.random_case(252, 256, 2.56 / 256, 3000, surface="plate", mode="shed"),
             wl.random_case(253, 1024, 2.56 / 1024, 4000, surface="cylinder"),
             wl.random_case(254, 128, 2.0 / 128, 6000, surface="cylinder"),
             _with_dense_cluster(wl.random_case(256, 128, 2.0 / 128, 4000, surface=None), 6000, 256),
             wl.random_case(255, 32, 2.0 / 32, 300, surface=None)]
    for c in cases:
        plan = gpf.Plan(ctx, c.n, c.dx)
        X, Y, G = (torch.as_tensor(a, dtype=torch.float64).to(DEV) for a in (c.X, c.Y, c.G))
        fields = []
        for rep in range(3):
            w = torch.full((c.n, c.n), float("nan"), dtype=plan.field_dtype, device=DEV)
            gpf.gpf_regularize_vortices(plan, X, Y, G, w)
            gpf.gpf_regularize_vortices(plan, X, Y, G, w, accumulate=True)   # 2 R_v
            torch.cuda.synchronize()
            fields.append(w.cpu().numpy())
        perm = np.random.default_rng(7).permutation(c.nv)
        Xp, Yp, Gp = (torch.as_tensor(a[perm], dtype=torch.float64).to(DEV) for a in (c.X, c.Y, c.G))
        w = torch.full((c.n, c.n), float("nan"), dtype=plan.field_dtype, device=DEV)
        gpf.gpf_regularize_vortices(plan, Xp, Yp, Gp, w)
        gpf.gpf_regularize_vortices(plan, Xp, Yp, Gp, w, accumulate=True)
        torch.cuda.synchronize()
        fields.append(w.cpu().numpy())
        same = all(np.array_equal(fields[0], f) for f in fields[1:])
        ok = np.isfinite(fields[0]).all() and np.abs(fields[0]).max() > 0
        ref = 2.0 * op.regularize_vortices(op.Grid.centered(c.n, c.dx), c.X, c.Y, c.G)
        err = rell2(fields[0].astype(np.float64), ref)
        say(f"[R_v repeat] {c.name} nv={c.nv}: bit-identical {same}, finite {ok}, relL2 {err:.1e}")
        assert same and ok, c.name
        assert err <= 1e-6, (c.name, err)


def test_solves_repeat_bit_for_bit(ctx):
    """No step of a solve adds with float atomics (R_v in integers, R_s f
    and the new vortices node by node): streamfunction, f and velocities
    are the same bits on every call, alone and in a merged batch, for a
    cylinder with prescribed circulation, a plate shedding at both edges,
    an FP64 first convolution, and tiles of several items."""
    cases = [wl.random_case(261, 128, 2.0 / 128, 3000, surface="cylinder"),
             wl.random_case(262, 256, 2.0 / 256, 2000, surface="plate", mode="shed"),
             _with_dense_cluster(wl.random_case(263, 128, 2.0 / 128, 1000, surface="ellipse"), 3000, 263)]
    flags = [gpf.GPF_FP32, gpf.GPF_FP32, gpf.GPF_CONV1_FP64]
    for c, fl in zip(cases, flags):
        outs = []
        for rep in range(3):
            r = run_solve_case(ctx, c, fl)
            outs.append(r)
        same = all(np.array_equal(outs[0][k], o[k]) for o in outs[1:] for k in outs[0])
        say(f"[solve repeat] {c.name} flags={fl}: bit-identical {same}")
        assert same, c.name
    st = Setup(ctx, cases)
    batch = gpf.Batch(ctx, len(cases))
    runs = []
    for rep in range(3):
        outs = st.outputs()
        batch.solve(st.plans, st.bodies, st.ins, [o.struct for o in outs])
        for o in outs:
            gpf.gpf_sync(o.status)
        runs.append([_host(o) for o in outs])
    same = all(np.array_equal(runs[0][i][k], r[i][k]) for r in runs[1:] for i in range(len(cases))
               for k in runs[0][i])
    say(f"[merged repeat] {len(cases)} problems: bit-identical {same}")
    assert same


def run_solve_case(ctx, c, flags):
    edges = tuple(c.edges) if c.mode in ("kutta", "shed") else None
    s = gpf.Solver(ctx, c.n, c.dx, c.surface, flags=flags, edges=edges)
    X, Y, G = s.upload(c)
    s.solve(s.inputs_for(c, X, Y, G), X, velocities=True)
    gpf.gpf_sync(s.status)
    torch.cuda.synchronize()
    return {"s": s.psi.cpu().numpy(), "u": s.u.cpu().numpy(), "v": s.v.cpu().numpy(),
            "f": s.f.cpu().numpy(), "sc": s.scalars.cpu().numpy()}


def test_solve_without_body_repeats_bit_for_bit(ctx):
    """Without a body no step of a solve adds with atomics: the
    streamfunction and the velocities are the same bits on every call, with
    tiles of several chunks of records."""
    c = _with_dense_cluster(wl.random_case(257, 128, 2.0 / 128, 4000, surface=None), 6000, 257)
    outs = []
    for rep in range(3):
        s = gpf.Solver(ctx, c.n, c.dx, None, flags=gpf.GPF_FP32)
        X, Y, G = s.upload(c)
        s.solve(s.inputs_for(c, X, Y, G), X, velocities=True)
        gpf.gpf_sync(s.status)
        torch.cuda.synchronize()
        outs.append([t.cpu().numpy() for t in (s.psi, s.u, s.v)])
    same = all(np.array_equal(a, b) for o in outs[1:] for a, b in zip(outs[0], o))
    say(f"[solve repeat] n={c.n} nv={c.nv}: bit-identical {same}")
    assert same
