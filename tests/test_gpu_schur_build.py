"""The Schur complement built column by column from batched unit sheets
(R_s, the convolution, E_s) against the exact S from the LGF table: two
independent routes to the same matrix.  In FP64 they agree to rounding; in
FP32 the column build carries the convolution's rounding, which the
ill-conditioned plate amplifies beyond the sheet tolerance (the reason the
library builds S exactly in FP64)."""
import sys

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2102_11910_amd import gpf  # noqa: E402
from paper_2102_11910_amd import workloads as wl  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    return gpf.Context(0)


def body_for(ctx, case):
    plan = gpf.Plan(ctx, case.n, case.dx)
    sf = case.surface
    edges = tuple(case.edges) if case.mode in ("kutta", "shed") else ()
    return plan, gpf.Body(plan, sf.xs, sf.ys, sf.ds, edges)


def test_cylinder_columns_match_the_exact_schur_complement(ctx):
    plan, body = body_for(ctx, wl.config1())
    s64, f64, ms64 = body.schur_by_convolution(fp64=True, batch=16)
    s32, f32, ms32 = body.schur_by_convolution(fp64=False, batch=16)
    say(f"[schur columns] cylinder 128^2 ns={body.ns}: FP64 S {s64:.1e} f {f64:.1e} ({ms64:.2f} ms); "
        f"FP32 S {s32:.1e} f {f32:.1e} ({ms32:.2f} ms)")
    assert s64 <= 1e-12 and f64 <= 1e-10
    assert s32 <= 1e-6 and f32 <= 1e-4     # well conditioned: FP32 columns suffice


def test_plate_columns_fp32_amplified(ctx):
    plan, body = body_for(ctx, wl.config2())
    s64, f64, ms64 = body.schur_by_convolution(fp64=True, batch=32)
    s32, f32, ms32 = body.schur_by_convolution(fp64=False, batch=32)
    amp = body.info()["amp"]
    say(f"[schur columns] plate 512^2 ns={body.ns} amp={amp:.3g}: FP64 S {s64:.1e} f {f64:.1e} "
        f"({ms64:.2f} ms); FP32 S {s32:.1e} f {f32:.1e} ({ms32:.2f} ms)")
    assert s64 <= 1e-12 and f64 <= 1e-8
    assert s32 <= 1e-6
    assert f32 <= 1e-4 and f32 >= 100.0 * s32     # amplified, still inside the tolerance


def test_schur_columns_arguments_checked(ctx):
    plan, body = body_for(ctx, wl.config1())
    with pytest.raises(gpf.GpfError) as e:
        body.schur_by_convolution(batch=0)
    assert e.value.status == gpf.GPF_E_INVALID
