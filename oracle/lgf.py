"""Lattice Green's function (LGF) of the unscaled 5-point Laplacian.

Sec. 2.1 writes the particular solution of the discrete Poisson equation
L s = -w (eq. poisson) with the inverse operator L^-1 given by the lattice
Green's function of L.  The paper only cites the function, so this module
takes it from its definition:

    Delta_h G = delta,   Delta_h g(m,n) = g(m+1,n)+g(m-1,n)+g(m,n+1)+g(m,n-1)-4g(m,n)

with the additive gauge fixed by G(0,0) = 0.  Writing G as the Fourier
integral over the Brillouin zone and integrating one angle in closed form
(int_{-pi}^{pi} cos(n a)/(cosh t - cos a) da = 2 pi e^{-|n| t}/sinh t) gives
the one-dimensional integral

    G(m,n) = 1/(2 pi) int_0^pi [1 - cos(m th) exp(-|n| t(th))] / sinh t(th) dth,
    cosh t = 2 - cos th,

which is used here with |n| >= |m| so that the oscillating factor is damped.
Far from the origin the classical asymptotic expansion of this lattice
function (terms r^0, r^-2, r^-4) is used; its truncation error is below
1e-13 beyond r = 128, where the quadrature is switched off.

The scaled operator of the paper is L = Delta_h / dx^2, so L^-1 w = dx^2 (G * w).
"""
from __future__ import annotations

import functools

import numpy as np
from scipy import integrate

EULER_GAMMA = 0.57721566490153286061

#: radius (in cells) inside which G is integrated numerically
QUAD_RADIUS = 128


def _integrand(m: np.ndarray, n: np.ndarray):
    """Integrand of the 1-D LGF integral for arrays of offsets (|n| >= |m|).

    The numerator 1 - cos(m th) e^{-n t} is rewritten as
    2 sin^2(m th / 2) - cos(m th) expm1(-n t) so that it keeps full relative
    accuracy as th -> 0; cosh t - 1 = 1 - cos th = 2 sin^2(th/2).
    """

    def f(th):
        x = 2.0 * np.sin(0.5 * th) ** 2          # cosh t - 1
        sinh_t = np.sqrt(x * (x + 2.0))
        t = np.log1p(x + sinh_t)                 # acosh(1 + x)
        num = 2.0 * np.sin(0.5 * m * th) ** 2 - np.cos(m * th) * np.expm1(-n * t)
        return num / sinh_t

    return f


def lgf_quadrature(offsets) -> np.ndarray:
    """G at the given integer offsets [(m, n), ...] by adaptive quadrature."""
    off = np.abs(np.asarray(offsets, dtype=np.int64)).reshape(-1, 2)
    lo = np.minimum(off[:, 0], off[:, 1]).astype(np.float64)
    hi = np.maximum(off[:, 0], off[:, 1]).astype(np.float64)
    out = np.zeros(len(off))
    nz = (lo + hi) > 0
    if nz.any():
        val, _ = integrate.quad_vec(_integrand(lo[nz], hi[nz]), 0.0, np.pi,
                                    epsabs=1e-14, epsrel=1e-13, norm="max",
                                    limit=20000)
        out[nz] = val / (2.0 * np.pi)
    return out


def lgf_far_field(m, n) -> np.ndarray:
    """Asymptotic expansion of G for large r = sqrt(m^2 + n^2).

    G ~ (ln r + gamma + 3/2 ln 2)/(2 pi) - cos(4 th)/(24 pi r^2)
        - (43 c^8 - 772 c^6 s^2 + 1570 c^4 s^4 - 772 c^2 s^6 + 43 s^8)/(480 pi r^4)
    with c = m/r, s = n/r.  The leading term is the continuous Green's
    function of the Laplacian, -1/(2 pi) ln r for the operator -Delta.
    """
    m = np.asarray(m, dtype=np.float64)
    n = np.asarray(n, dtype=np.float64)
    r = np.hypot(m, n)
    c = m / r
    s = n / r
    c2, s2 = c * c, s * s
    cos4 = c2 * c2 - 6.0 * c2 * s2 + s2 * s2
    p8 = (43.0 * c2 ** 4 - 772.0 * c2 ** 3 * s2 + 1570.0 * c2 ** 2 * s2 ** 2
          - 772.0 * c2 * s2 ** 3 + 43.0 * s2 ** 4)
    return ((np.log(r) + EULER_GAMMA + 1.5 * np.log(2.0)) / (2.0 * np.pi)
            - cos4 / (24.0 * np.pi * r ** 2)
            - p8 / (480.0 * np.pi * r ** 4))


@functools.lru_cache(maxsize=8)
def lgf_table(nmax: int) -> np.ndarray:
    """Table T[a, b] = G(a, b) for 0 <= a, b <= nmax (symmetric in a, b).

    Quadrature inside r <= QUAD_RADIUS, asymptotic expansion outside.
    The returned array is read-only (it is cached).
    """
    nmax = int(nmax)
    a, b = np.meshgrid(np.arange(nmax + 1), np.arange(nmax + 1), indexing="ij")
    T = np.zeros((nmax + 1, nmax + 1))
    upper = a >= b                     # compute one octant, mirror after
    near = upper & (a * a + b * b <= QUAD_RADIUS * QUAD_RADIUS)
    far = upper & ~near
    if near.any():
        T[near] = lgf_quadrature(np.stack([a[near], b[near]], axis=1))
    if far.any():
        T[far] = lgf_far_field(a[far], b[far])
    T = np.where(upper, T, T.T)
    T.setflags(write=False)
    return T


def lgf(m, n, table: np.ndarray | None = None) -> np.ndarray:
    """G(m, n) for integer arrays m, n (any sign), from a table if given."""
    m = np.abs(np.asarray(m, dtype=np.int64))
    n = np.abs(np.asarray(n, dtype=np.int64))
    if table is None:
        table = lgf_table(int(max(m.max(initial=0), n.max(initial=0))))
    return table[m, n]
