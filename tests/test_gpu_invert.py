"""FP64 inverse of the Schur complement's solver (Sec. 2.2.2, App. A):
blocked Gauss-Jordan with partial pivoting (16-column panels, updates on
FP64 matrix cores) for n <= 2048 and the column-by-column elimination
above.  Compared with LAPACK's inverse (numpy) on seeded matrices whose
sizes cross panel (16) and tile (64) edges, on matrices that need row
exchanges, and on a singular one."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2102_11910_amd import gpf  # noqa: E402

DEV = torch.device("cuda", 0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    return gpf.Context(0)


def _inverse(ctx, a):
    da = torch.as_tensor(a, dtype=torch.float64).to(DEV).contiguous()
    di = torch.full_like(da, float("nan"))
    mp = gpf.gpf_invert_fp64(ctx, da, di)
    torch.cuda.synchronize()
    return di.cpu().numpy(), mp


@pytest.mark.parametrize("n", [1, 2, 3, 15, 16, 17, 63, 64, 65, 100, 513, 1024, 1100, 2048])
def test_random_matrices(ctx, n):
    rng = np.random.default_rng(1000 + n)
    a = rng.standard_normal((n, n)) + 4.0 * np.sqrt(n) * np.eye(n) * rng.choice([-1.0, 1.0], n)
    say(f"[invert] random n={n}")
    x, mp = _inverse(ctx, a)
    ref = np.linalg.inv(a)
    err = np.abs(x - ref).max() / np.abs(ref).max()
    res = np.abs(x @ a - np.eye(n)).max()
    say(f"   rel err {err:.2e}, residual {res:.2e}, min pivot rel {mp:.2e}")
    assert err <= 1e-12 and res <= 1e-12 and mp > 1e-3


@pytest.mark.parametrize("n", [40, 300])
def test_row_exchanges(ctx, n):
    """A permuted matrix with tiny diagonal entries: every column step must
    take its pivot from another row."""
    rng = np.random.default_rng(7 + n)
    perm = rng.permutation(n)
    a = 1e-9 * rng.standard_normal((n, n))
    a[np.arange(n), perm] = rng.uniform(1.0, 2.0, n) * rng.choice([-1.0, 1.0], n)
    say(f"[invert] permuted n={n}")
    x, mp = _inverse(ctx, a)
    ref = np.linalg.inv(a)
    err = np.abs(x - ref).max() / np.abs(ref).max()
    say(f"   rel err {err:.2e}, min pivot rel {mp:.2e}")
    assert err <= 1e-12


def test_column_by_column_path_above_2048(ctx):
    n = 2100
    rng = np.random.default_rng(5)
    a = rng.standard_normal((n, n)) + 4.0 * np.sqrt(n) * np.eye(n)
    say(f"[invert] random n={n} (column by column)")
    x, mp = _inverse(ctx, a)
    err = np.abs(x - np.linalg.inv(a)).max() / np.abs(x).max()
    say(f"   rel err {err:.2e}")
    assert err <= 1e-12


def test_singular_matrix_reports_a_tiny_pivot(ctx):
    rng = np.random.default_rng(9)
    b = rng.standard_normal((50, 49))
    a = b @ rng.standard_normal((49, 50))     # rank 49
    say("[invert] singular n=50")
    _, mp = _inverse(ctx, a)
    say(f"   min pivot rel {mp:.2e}")
    assert mp < 1e-12


def test_arguments_checked(ctx):
    a = torch.eye(4, dtype=torch.float64, device=DEV)
    with pytest.raises(gpf.GpfError) as e:
        gpf.gpf_invert_fp64(ctx, a, a)
    assert e.value.status == gpf.GPF_E_INVALID
