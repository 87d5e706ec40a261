"""The allocation-free convolution entry point against gpf_convolve (same
kernels, so the same bits) and against the oracle's FP64 convolution
(Sec. 2.1, eq. poisson), on two calls in a row, the second on a smaller
grid, and its refusal of grids beyond its fixed scratch."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2102_11910_amd import gpf  # noqa: E402
from oracle.operators import Grid, inv_laplacian_fft, regularize_vortices  # noqa: E402
from tests.conftest import rell2  # noqa: E402

DEV = torch.device("cuda", 0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _source(n, dx, nv, seed):
    """Grid vorticity of a seeded vortex cloud (the oracle's R_v), rounded to
    the plan's field type by the caller."""
    rng = np.random.default_rng(seed)
    grid = Grid.centered(n, dx)
    h = (n - 1) * dx / 2 - 4 * dx
    X, Y = rng.uniform(-h, h, nv), rng.uniform(-h, h, nv)
    G = rng.normal(0.0, 1e-2, nv)
    return regularize_vortices(grid, X, Y, G)


@pytest.fixture(scope="module")
def ctx():
    return gpf.Context(0)


def _one(ctx, n, fp64, seed):
    dx = 2.4 / n
    flags = gpf.GPF_FP64 if fp64 else gpf.GPF_FP32
    plan = gpf.Plan(ctx, n, dx, flags=flags)
    dt = torch.float64 if fp64 else torch.float32
    w64 = _source(n, dx, 3 * n, seed)
    w = torch.as_tensor(w64).to(dt).to(DEV)
    wd = w.double().cpu().numpy()        # the values the GPU sees
    gamma = float(dx * dx * wd.sum())
    s_ref = torch.empty_like(w)
    s_na = torch.full_like(w, float("nan"))
    say(f"[no-alloc] n={n} fp64={fp64}: gpf_convolve, then gpf_convolve_noalloc")
    gpf.gpf_convolve(plan, w, s_ref, gamma)
    gpf.gpf_convolve_noalloc(plan, w, s_na, gamma)
    torch.cuda.synchronize()
    a, b = s_na.double().cpu().numpy(), s_ref.double().cpu().numpy()
    assert np.array_equal(a, b), float(np.max(np.abs(a - b)))
    oracle = inv_laplacian_fft(wd, dx)
    err = rell2(a, oracle)
    say(f"   bit-equal to gpf_convolve; relL2 against the oracle {err:.2e}")
    assert err <= (1e-12 if fp64 else 1e-5)


def test_noalloc_two_calls_second_smaller(ctx):
    # largest FP64 grid the scratch holds, then a smaller FP32 grid
    _one(ctx, 1024, True, 101)
    _one(ctx, 256, False, 102)


def test_noalloc_largest_fp32_then_smaller(ctx):
    _one(ctx, 2048, False, 103)
    _one(ctx, 64, False, 104)


def test_noalloc_rejects_grids_beyond_scratch(ctx):
    plan = gpf.Plan(ctx, 2048, 2.4 / 2048, flags=gpf.GPF_FP64)
    w = torch.zeros((2048, 2048), dtype=torch.float64, device=DEV)
    with pytest.raises(gpf.GpfError) as e:
        gpf.gpf_convolve_noalloc(plan, w, w, 0.0)
    assert e.value.status == gpf.GPF_E_UNSUPPORTED
