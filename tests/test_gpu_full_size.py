"""Parity at the benchmark's launch configuration and at the largest sizes.

* The timed configuration itself: 32 plate problems (512^2, Kutta at both
  edges with new vortices, 1e4 vortices each, different seeds) in one batched
  launch sequence, every problem against the oracle.
* The largest grid, 2048^2: a cylinder with 1024 surface points and 1e6
  vortices (prescribed circulation), and a plate with Kutta at both edges,
  against the oracle (full fields; the oracle's FFT route handles 2048^2).
"""
import functools
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2102_11910_amd import gpf  # noqa: E402
from paper_2102_11910_amd import workloads as wl  # noqa: E402
from oracle.lgf import lgf_table  # noqa: E402
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


def upload(c):
    return [torch.as_tensor(a, dtype=torch.float64).to(DEV) for a in (c.X, c.Y, c.G)]


def check(c, o, ref, tol_s=1e-5, tol_f=1e-4, tol_u=1e-4, label=""):
    es = rell2(o.psi.double().cpu().numpy(), ref.s)
    eu = rell2(np.r_[o.u.cpu().numpy(), o.v.cpu().numpy()], np.r_[ref.u, ref.v])
    ef = rell2(o.f.cpu().numpy(), ref.f)
    msg = f"{label}: s {es:.2e} uv {eu:.2e} f {ef:.2e}"
    if ref.gamma_new is not None:
        gn = o.scalars.cpu().numpy()[4:4 + len(ref.gamma_new)]
        eg = float(np.max(np.abs(gn - ref.gamma_new)) / np.max(np.abs(ref.gamma_new)))
        msg += f" gamma_new {eg:.2e}"
        assert eg <= 1e-5, msg
    say("   " + msg)
    assert es <= tol_s and eu <= tol_u and ef <= tol_f, msg
    return es, eu, ef


def test_benchmark_batch_of_32_plates_matches_oracle(ctx):
    B = 32
    cases = [wl.config2(seed=2 + i) for i in range(B)]
    c0 = cases[0]
    plan = gpf.Plan(ctx, c0.n, c0.dx, flags=gpf.GPF_POLICY_AUTO)
    sf = c0.surface
    body = gpf.Body(plan, sf.xs, sf.ys, sf.ds, tuple(c0.edges))
    assert body.info()["conv1_fp64"]
    ins, outs, keep = [], [], []
    for c in cases:
        X, Y, G = upload(c)
        keep.append((X, Y, G))
        ins.append(gpf.make_inputs(X, Y, G, c.u_inf, c.v_inf, mode=c.mode, znew=c.znew))
        outs.append(gpf.Outputs(c.n, c.nv, sf.ns))
    batch = gpf.Batch(ctx, B)
    batch.solve([plan] * B, [body] * B, ins, [o.struct for o in outs])
    for o in outs:
        gpf.gpf_sync(o.status)
    torch.cuda.synchronize()
    say(f"[bench configuration] {B} x {c0.name}, nv={c0.nv}")
    table = lgf_table(c0.n)
    ob = body_of(c0, table)
    worst = np.zeros(3)
    for i, (c, o) in enumerate(zip(cases, outs)):
        ref = oracle_solve(problem_of(c), ob, table)
        worst = np.maximum(worst, check(c, o, ref, label=f"problem {i}") )
    say(f"   worst over the batch: s {worst[0]:.2e} uv {worst[1]:.2e} f {worst[2]:.2e}")


@functools.lru_cache(maxsize=1)
def largest_cases():
    rng = np.random.default_rng(2048)
    n, dx = 2048, 2.56 / 2048
    cyl = wl.cylinder(0.5, 1024)
    pts = wl._uniform_cloud(rng, 1000000, 1.2, cyl, 2.0 * dx)
    G = rng.normal(0.0, 1e-3, size=len(pts))
    X, Y, G = wl.f32(pts[:, 0]), wl.f32(pts[:, 1]), wl.f32(G)
    c1 = wl.Case("cylinder 2048^2, 1e6 vortices", n, dx, X, Y, G, cyl, u_inf=1.0,
                 mode="circulation", gamma_b=float(-np.sum(G)))
    plate = wl.flat_plate(1.0, 15.0, 1024)
    pts = wl._uniform_cloud(rng, 100000, 1.2, plate, 2.0 * dx)
    G = rng.normal(0.0, 1e-3, size=len(pts))
    X, Y, G = wl.f32(pts[:, 0]), wl.f32(pts[:, 1]), wl.f32(G)
    c2 = wl.Case("plate 2048^2, Kutta x2, 1e5 vortices", n, dx, X, Y, G, plate, u_inf=1.0,
                 mode="shed")
    c2.edges = plate.edges
    c2.znew = wl.plate_new_vortices(plate, 4.0 * dx)
    return [c1, c2]


@functools.lru_cache(maxsize=2)
def oracle_ref(which):
    c = largest_cases()[which]
    return oracle_solve(problem_of(c), body_of(c))


@pytest.mark.parametrize("which", [0, 1])
@pytest.mark.parametrize("flags", [gpf.GPF_POLICY_AUTO, gpf.GPF_FP64])
def test_largest_grid_matches_oracle(ctx, which, flags):
    c = largest_cases()[which]
    say(f"[largest] {c.name}, ns={c.surface.ns}, flags={flags}")
    plan = gpf.Plan(ctx, c.n, c.dx, flags=flags)
    sf = c.surface
    edges = tuple(c.edges) if c.mode == "shed" else ()
    body = gpf.Body(plan, sf.xs, sf.ys, sf.ds, edges)
    X, Y, G = upload(c)
    inp = gpf.make_inputs(X, Y, G, c.u_inf, c.v_inf, mode=c.mode, gamma_b=c.gamma_b, znew=c.znew)
    o = gpf.Outputs(c.n, c.nv, sf.ns, fp64=bool(flags & gpf.GPF_FP64))
    gpf.gpf_solve(plan, body, inp, o.struct)
    gpf.gpf_sync(o.status)
    torch.cuda.synchronize()
    say(f"   body {body.info()}")
    ref = oracle_ref(which)
    if flags & gpf.GPF_FP64:
        check(c, o, ref, tol_s=1e-9, tol_f=1e-8, tol_u=1e-9, label="FP64")
    else:
        check(c, o, ref, label="FP32 + policy")
