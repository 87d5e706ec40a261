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


def test_amplification_probe_on_the_oracle_schur(ctx):
    """The precision policy's probe `amp`: how much more S^-1 amplifies the
    alternating vector (+-max|y_s|, the finest pattern the surface carries)
    than the smooth freestream right-hand side -y_s, relative to their
    sizes.  The device value (from its FP64 inverse) equals the same
    quantity formed with the oracle's LU factors of S, for the well
    conditioned cylinder and the amplifying plate."""
    import numpy as np
    import scipy.linalg as sla
    from tests.oracle_adapter import body_of
    # the cylinder stays under the policy threshold (500), the plate exceeds it
    for case, lo, hi in ((wl.config1(), 0.0, 500.0), (wl.config2(), 500.0, np.inf)):
        _, body = body_for(ctx, case)
        ob = body_of(case)
        ys = np.asarray(case.surface.ys, np.float64)
        r = -ys
        a = np.where(np.arange(len(ys)) % 2 == 1, -1.0, 1.0) * np.abs(ys).max()
        fr, fa = sla.lu_solve(ob.lu, r), sla.lu_solve(ob.lu, a)
        ref = (np.linalg.norm(fa) / np.linalg.norm(fr)) * (np.linalg.norm(r) / np.linalg.norm(a))
        amp = body.info()["amp"]
        say(f"[amp] {case.name}: device {amp:.6g} oracle {ref:.6g}")
        assert abs(amp - ref) <= 1e-8 * ref
        assert lo <= amp <= hi
