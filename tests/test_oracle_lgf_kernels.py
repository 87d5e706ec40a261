"""Pins of the oracle's lattice Green's function and discrete delta functions.

The LGF is fixed by its defining equation Delta_h G = delta with G(0,0) = 0
(Sec. 2.1), by exact lattice values that follow from that equation and the
lattice symmetry, and by the continuous Green's function far away.  The two
delta functions are fixed by the moment conditions that define them (Fig. 1).
"""
import json
import os

import numpy as np
import pytest

from oracle.kernels import m4prime, yang3
from oracle.lgf import QUAD_RADIUS, lgf_far_field, lgf_quadrature, lgf_table

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def lap5(T, m, n):
    """Delta_h G at offset (m, n) using the symmetric table."""
    g = lambda a, b: T[abs(a), abs(b)]
    return g(m + 1, n) + g(m - 1, n) + g(m, n + 1) + g(m, n - 1) - 4 * g(m, n)


def test_lgf_closed_values():
    with open(os.path.join(GOLDEN, "lgf_closed_values.json")) as fh:
        gold = json.load(fh)
    T = lgf_table(12)
    for item in gold["values"]:
        m, n = item["offset"]
        assert abs(T[m, n] - item["value"]) <= 1e-13, item
    # diagonal: G(k,k) = (1/pi) sum_{l=1..k} 1/(2l-1)
    for k in range(1, 13):
        exact = sum(1.0 / (2 * l - 1) for l in range(1, k + 1)) / np.pi
        assert abs(T[k, k] - exact) <= 1e-13


def test_lgf_discrete_laplacian_is_delta():
    nmax = QUAD_RADIUS + 24
    T = lgf_table(nmax)
    worst_near = worst_far = 0.0
    for m in range(0, nmax - 1):
        for n in range(0, m + 1):
            res = lap5(T, m, n) - (1.0 if (m, n) == (0, 0) else 0.0)
            if m * m + n * n <= (QUAD_RADIUS - 1) ** 2:
                worst_near = max(worst_near, abs(res))
            else:
                worst_far = max(worst_far, abs(res))
    assert worst_near <= 1e-12
    assert worst_far <= 1e-9


def test_lgf_far_field_matches_quadrature_at_switch():
    pts = [(QUAD_RADIUS, 0), (100, 90), (127, 20), (140, 3), (96, 96)]
    q = lgf_quadrature(pts)
    f = lgf_far_field([p[0] for p in pts], [p[1] for p in pts])
    assert np.max(np.abs(q - f)) <= 2e-13


def test_lgf_leading_term_is_continuous_greens_function():
    # G(r) - ln(r)/(2 pi) -> (gamma + 3/2 ln 2)/(2 pi) as r -> infinity
    q = lgf_quadrature([(60, 0), (120, 0)])
    c = (0.57721566490153286 + 1.5 * np.log(2.0)) / (2 * np.pi)
    err = np.abs(q - np.log([60.0, 120.0]) / (2 * np.pi) - c)
    assert err[1] < err[0] / 3.5          # decays like r^-2
    assert err[1] < 1e-5


def test_lgf_symmetry():
    T = lgf_table(40)
    assert np.array_equal(T, T.T)
    assert T[0, 0] == 0.0


@pytest.mark.parametrize("kernel", [m4prime, yang3])
@pytest.mark.parametrize("x", [0.0, 0.13, 0.5, 0.77, 0.999])
def test_kernel_partition_of_unity_and_first_moment(kernel, x):
    shifts = np.arange(-3, 4)
    w = kernel(x - shifts)
    assert abs(w.sum() - 1.0) <= 1e-14
    assert abs(np.sum((x - shifts) * w)) <= 1e-14


@pytest.mark.parametrize("x", [0.0, 0.13, 0.5, 0.77])
def test_m4prime_second_moment_and_interpolation(x):
    shifts = np.arange(-3, 4)
    w = m4prime(x - shifts)
    assert abs(np.sum((x - shifts) ** 2 * w)) <= 1e-14
    assert m4prime(0.0) == 1.0 and m4prime(1.0) == 0.0 and m4prime(2.0) == 0.0


def test_kernel_continuity_and_support():
    for k in (m4prime, yang3):
        for b in (1.0, 2.0):
            assert abs(k(b - 1e-12) - k(b + 1e-12)) < 1e-9
        assert k(2.0) == 0.0 and k(2.5) == 0.0
    # the smoothed 3-point function is non-negative; M4' has negative lobes
    assert np.all(yang3(np.linspace(-2, 2, 101)) >= 0.0)
    assert m4prime(1.5) < 0.0
    # values at the nodes of the smoothed 3-point function
    assert abs(yang3(0.0) - 0.6182) < 1e-4
    assert abs(yang3(1.0) - 0.1909) < 1e-4
