"""Convolution schedules and the autotuner on the GPU.

Every schedule the autotuner can choose performs the same transforms, so
the batched solves of the benchmark's plate workload under each of them
agree with the default schedule to rounding and with the oracle to the
standard tolerances.  The autotuner picks one of them, stores it in the
context, and reuses a cached result without timing."""
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
from oracle.lgf import lgf_table  # noqa: E402
from oracle.solve import solve as oracle_solve  # noqa: E402
from tests.conftest import rell2  # noqa: E402
from tests.oracle_adapter import body_of, problem_of  # noqa: E402

DEV = torch.device("cuda", 0)
B = 4


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    return gpf.Context(0)


def schedules(fp64, n):
    cols = (1, 2) if fp64 and n >= 512 else (0,)
    return [{"rows": r, "order": o, "cols": c} for r in (1, 2) for o in (1, 2) for c in cols]


class PlateBatch:
    def __init__(self, ctx):
        self.cases = [wl.config2(seed=2 + i) for i in range(B)]
        c0 = self.cases[0]
        sf = c0.surface
        self.plan = gpf.Plan(ctx, c0.n, c0.dx, flags=gpf.GPF_POLICY_AUTO)
        self.body = gpf.Body(self.plan, sf.xs, sf.ys, sf.ds, tuple(c0.edges))
        assert self.body.info()["conv1_fp64"]
        self.keep, self.ins, self.outs = [], [], []
        for c in self.cases:
            X, Y, G = (torch.as_tensor(a, dtype=torch.float64).to(DEV) for a in (c.X, c.Y, c.G))
            self.keep.append((X, Y, G))
            self.ins.append(gpf.make_inputs(X, Y, G, c.u_inf, c.v_inf, mode=c.mode, znew=c.znew))
            self.outs.append(gpf.Outputs(c.n, c.nv, sf.ns))
        self.batch = gpf.Batch(ctx, B)

    def solve(self):
        self.batch.solve([self.plan] * B, [self.body] * B, self.ins, [o.struct for o in self.outs])
        for o in self.outs:
            gpf.gpf_sync(o.status)
        torch.cuda.synchronize()
        h = lambda t: t.double().cpu().numpy().copy()
        return [{"s": h(o.psi), "u": h(o.u), "v": h(o.v), "f": h(o.f)} for o in self.outs]


def test_every_schedule_gives_the_same_solves(ctx):
    pb = PlateBatch(ctx)
    n = pb.cases[0].n
    for fp64 in (False, True):
        gpf.schedule_set(ctx, n, fp64, B, None)
    base = pb.solve()
    table = lgf_table(n)
    ref = oracle_solve(problem_of(pb.cases[0]), body_of(pb.cases[0], table), table)
    for s64 in schedules(True, n):
        for s32 in schedules(False, n):
            gpf.schedule_set(ctx, n, True, B, s64)
            gpf.schedule_set(ctx, n, False, B, s32)
            got = pb.solve()
            worst = [0.0, 0.0, 0.0]
            for g, b in zip(got, base):
                worst[0] = max(worst[0], rell2(g["s"], b["s"]))
                worst[1] = max(worst[1], rell2(np.r_[g["u"], g["v"]], np.r_[b["u"], b["v"]]))
                worst[2] = max(worst[2], rell2(g["f"], b["f"]))
            es = rell2(got[0]["s"], ref.s)
            ef = rell2(got[0]["f"], ref.f)
            say(f"[schedule] FP64 {s64} FP32 {s32}: vs default s {worst[0]:.1e} uv {worst[1]:.1e} "
                f"f {worst[2]:.1e}; vs oracle s {es:.1e} f {ef:.1e}")
            assert worst[0] <= 1e-6 and worst[1] <= 1e-6 and worst[2] <= 1e-8
            assert es <= 1e-5 and ef <= 1e-4
    for fp64 in (False, True):
        gpf.schedule_set(ctx, n, fp64, B, None)
        assert gpf.schedule_get(ctx, n, fp64, B) == {"rows": 0, "order": 0, "cols": 0}


@pytest.mark.parametrize("fp64", [False, True])
def test_autotune_picks_a_schedule_and_caches_it(ctx, tmp_path, fp64):
    c = wl.config2()
    plan = gpf.Plan(ctx, c.n, c.dx)
    cache = tmp_path / "tune.txt"
    chosen, us = gpf.autotune(plan, fp64, B, cache)
    say(f"[autotune] n={c.n} fp64={fp64} nb={B}: {chosen}, {us:.1f} us per batched convolution")
    assert chosen in [{"rows": 0, "order": 0, "cols": 0}] + schedules(fp64, c.n)
    assert us > 0.0 and math.isfinite(us)
    assert gpf.schedule_get(ctx, c.n, fp64, B) == chosen
    # batch sizes of the same class share the entry; other classes do not
    assert gpf.schedule_get(ctx, c.n, fp64, 7) == chosen
    assert gpf.schedule_get(ctx, c.n, fp64, 1) == {"rows": 0, "order": 0, "cols": 0}
    lines = cache.read_text().splitlines()
    assert len(lines) == 1
    f = lines[0].split()
    assert len(f) == 8 and f[0].startswith("gfx")
    assert [int(v) for v in f[1:7]] == [c.n, int(fp64), 1, chosen["rows"], chosen["order"],
                                         chosen["cols"]]
    # a second call reads the cache: same answer, nothing appended
    gpf.schedule_set(ctx, c.n, fp64, B, None)
    again, us2 = gpf.autotune(plan, fp64, B, cache)
    assert again == chosen and abs(us2 - float(f[7])) <= 1e-3
    assert len(cache.read_text().splitlines()) == 1
    gpf.schedule_set(ctx, c.n, fp64, B, None)


def test_schedule_arguments_checked(ctx):
    c = wl.config1()
    plan = gpf.Plan(ctx, c.n, c.dx)
    with pytest.raises(gpf.GpfError) as e:
        gpf.schedule_set(ctx, c.n, False, 1, {"rows": 3, "order": 0, "cols": 0})
    assert e.value.status == gpf.GPF_E_INVALID
    with pytest.raises(gpf.GpfError) as e:
        gpf.autotune(plan, False, 0)
    assert e.value.status == gpf.GPF_E_INVALID
    with pytest.raises(gpf.GpfError) as e:
        gpf.autotune(plan, False, 2000)
    assert e.value.status == gpf.GPF_E_INVALID


def test_batched_autotuner_tunes_the_entries_the_batch_uses(ctx):
    """On the plate batch the tuner chooses a lane count (read back with
    gpf_batch_get_lanes), then the FP64 entry (first convolution) and the
    FP32 entry (second) of the class its launches fall in, and the solves
    that follow, on those lanes, still match the oracle."""
    pb = PlateBatch(ctx)
    n = pb.cases[0].n
    for fp64 in (False, True):
        gpf.schedule_set(ctx, n, fp64, B, None)
    pb.batch.autotune([pb.plan] * B, [pb.body] * B, pb.ins, [o.struct for o in pb.outs])
    # the lane count comes first; a batch of one group is dealt out over the
    # lanes, so its launches (and the schedule class) hold ceil(B / lanes)
    lanes = pb.batch.lanes
    assert 1 <= lanes <= 4 and lanes == gpf.lib.gpf_batch_get_lanes(pb.batch.h)
    nb = -(-B // lanes)
    s64, s32 = gpf.schedule_get(ctx, n, True, nb), gpf.schedule_get(ctx, n, False, nb)
    say(f"[autotune batched] lanes {lanes}, FP64 {s64}, FP32 {s32}")
    assert s64 in [{"rows": 0, "order": 0, "cols": 0}] + schedules(True, n)
    assert s32 in [{"rows": 0, "order": 0, "cols": 0}] + schedules(False, n)
    # classes the batch does not use are untouched
    assert gpf.schedule_get(ctx, n, True, 32) == {"rows": 0, "order": 0, "cols": 0}
    got = pb.solve()
    table = lgf_table(n)
    for i in (0, B - 1):
        ref = oracle_solve(problem_of(pb.cases[i]), body_of(pb.cases[i], table), table)
        es, ef = rell2(got[i]["s"], ref.s), rell2(got[i]["f"], ref.f)
        say(f"   problem {i}: s {es:.1e} f {ef:.1e}")
        assert es <= 1e-5 and ef <= 1e-4
    for fp64 in (False, True):
        gpf.schedule_set(ctx, n, fp64, nb, None)
