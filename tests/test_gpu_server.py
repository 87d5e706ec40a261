"""The request server: mixed requests submitted from the host thread, solved
in batches by the server's worker, each equal to the same request solved
alone on the same plan and body; admission and argument errors."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2102_11910_amd import gpf  # noqa: E402
from paper_2102_11910_amd import workloads as wl  # noqa: E402
from tests.conftest import rell2  # noqa: E402

DEV = torch.device("cuda", 0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    return gpf.Context(0)


def requests():
    cases = []
    for k in range(14):
        n = (64, 128, 256)[k % 3]
        kind = ("cylinder", "plate", None, "ellipse")[k % 4]
        mode = "shed" if kind == "plate" else None
        cases.append(wl.random_case(200 + k, n, 2.0 / n, 50 + 37 * k, surface=kind, mode=mode))
    return cases


def test_server_matches_plain_solves(ctx):
    srv = gpf.Server(ctx, 4 << 30, max_slots=4)
    cases = requests()
    bodies, ins, keep, plans = [], [], [], []
    for c in cases:
        plan = srv.plan(c.n, c.dx)
        plans.append(plan)
        sf = c.surface
        edges = tuple(c.edges) if c.mode == "shed" else ()
        bodies.append(gpf.Body(plan, sf.xs, sf.ys, sf.ds, edges) if sf is not None else None)
        X, Y, G = (torch.as_tensor(a, dtype=torch.float64).to(DEV) for a in (c.X, c.Y, c.G))
        keep.append((X, Y, G))
        ins.append(gpf.make_inputs(X, Y, G, c.u_inf, c.v_inf, c.ub, c.vb, c.omega, c.mode,
                                   c.gamma_b, znew=c.znew))
    outs = [gpf.Outputs(c.n, c.nv, c.surface.ns if c.surface else 0) for c in cases]
    say(f"[server] {len(cases)} requests, n in {sorted(set(c.n for c in cases))}")
    ids = [srv.submit(p, b, i, o.struct) for p, b, i, o in zip(plans, bodies, ins, outs)]
    lat = [srv.wait(r) for r in ids]
    for o in outs:
        gpf.gpf_sync(o.status)
    assert all(x > 0.0 for x in lat)
    say(f"   latency ms: min {1e3 * min(lat):.3f} max {1e3 * max(lat):.3f}")
    worst = 0.0
    for c, p, b, i, o in zip(cases, plans, bodies, ins, outs):
        ref = gpf.Outputs(c.n, c.nv, c.surface.ns if c.surface else 0)
        gpf.gpf_solve(p, b, i, ref.struct)
        gpf.gpf_sync(ref.status)
        es = rell2(o.psi.double().cpu().numpy(), ref.psi.double().cpu().numpy())
        eu = rell2(np.r_[o.u.cpu().numpy(), o.v.cpu().numpy()], np.r_[ref.u.cpu().numpy(), ref.v.cpu().numpy()])
        ef = rell2(o.f.cpu().numpy(), ref.f.cpu().numpy()) if c.surface else 0.0
        worst = max(worst, es, eu, ef / 10.0)
        assert es <= 1e-5 and eu <= 1e-5 and ef <= 1e-4, (c.name, es, eu, ef)
    say(f"   server vs alone: worst {worst:.2e}")
    # a done request is forgotten once reported
    with pytest.raises(gpf.GpfError) as e:
        srv.poll(ids[0])
    assert e.value.status == gpf.GPF_E_INVALID
    srv.close()


def test_server_errors(ctx):
    srv = gpf.Server(ctx, 4 << 30, max_slots=2)
    c = wl.random_case(300, 64, 2.0 / 64, 40, surface="cylinder")
    other = srv.plan(128, 2.0 / 128)
    body = gpf.Body(other, c.surface.xs * 0.5, c.surface.ys * 0.5, c.surface.ds * 0.5)
    plan = srv.plan(c.n, c.dx)
    X, Y, G = (torch.as_tensor(a, dtype=torch.float64).to(DEV) for a in (c.X, c.Y, c.G))
    inp = gpf.make_inputs(X, Y, G, c.u_inf, mode="circulation", gamma_b=c.gamma_b)
    o = gpf.Outputs(c.n, c.nv, c.surface.ns)
    with pytest.raises(gpf.GpfError) as e:          # body of another grid's plan
        srv.submit(plan, body, inp, o.struct)
    assert e.value.status == gpf.GPF_E_INVALID
    with pytest.raises(gpf.GpfError) as e:          # circulation mode without a body
        srv.submit(plan, None, inp, o.struct)
    assert e.value.status == gpf.GPF_E_INVALID
    srv.close()
    tiny = gpf.Server(ctx, 1 << 20, max_slots=2)   # 1 MiB: no plan fits
    with pytest.raises(gpf.GpfError) as e:
        tiny.plan(256, 0.01)
    assert e.value.status == gpf.GPF_E_NOMEM
    tiny.close()


def test_batches_overlap_on_the_device(ctx):
    """One request per batch, a dozen large requests queued at once: the
    worker puts consecutive batches on different workspace sets and streams
    before the earlier ones finish, and every result still equals the same
    request solved alone."""
    srv = gpf.Server(ctx, 16 << 30, max_slots=1)
    cases = [wl.random_case(300 + k, 1024, 2.56 / 1024, 20000 + 3000 * k,
                            surface=("cylinder", "ellipse", "plate")[k % 3],
                            mode="shed" if k % 3 == 2 else None) for k in range(12)]
    plan = srv.plan(1024, 2.56 / 1024)
    bodies, ins, keep = [], [], []
    for c in cases:
        sf = c.surface
        edges = tuple(c.edges) if c.mode == "shed" else ()
        bodies.append(gpf.Body(plan, sf.xs, sf.ys, sf.ds, edges))
        X, Y, G = (torch.as_tensor(a, dtype=torch.float64).to(DEV) for a in (c.X, c.Y, c.G))
        keep.append((X, Y, G))
        ins.append(gpf.make_inputs(X, Y, G, c.u_inf, c.v_inf, c.ub, c.vb, c.omega, c.mode,
                                   c.gamma_b, znew=c.znew))
    outs = [gpf.Outputs(c.n, c.nv, c.surface.ns) for c in cases]
    say(f"[server overlap] {len(cases)} requests on 1024^2, one per batch")
    ids = [srv.submit(plan, b, i, o.struct) for b, i, o in zip(bodies, ins, outs)]
    for r in ids:
        srv.wait(r)
    for o in outs:
        gpf.gpf_sync(o.status)
    nbatch, most = srv.stats()
    say(f"   batches {nbatch}, most in flight at once {most}")
    assert nbatch == len(cases) and 2 <= most <= 3
    for c, b, i, o in zip(cases, bodies, ins, outs):
        ref = gpf.Outputs(c.n, c.nv, c.surface.ns)
        gpf.gpf_solve(plan, b, i, ref.struct)
        gpf.gpf_sync(ref.status)
        es = rell2(o.psi.double().cpu().numpy(), ref.psi.double().cpu().numpy())
        eu = rell2(np.r_[o.u.cpu().numpy(), o.v.cpu().numpy()], np.r_[ref.u.cpu().numpy(), ref.v.cpu().numpy()])
        ef = rell2(o.f.cpu().numpy(), ref.f.cpu().numpy())
        assert es <= 1e-5 and eu <= 1e-5 and ef <= 1e-4, (c.name, es, eu, ef)
    srv.close()
