"""The two discrete Dirac delta functions of radius two (Fig. 1(b), Sec. 2.1-2.2).

* Vortices are regularized with the M4' function of Monaghan (1985), cited
  in Sec. 2.1 (eq. vortexregularization).
* Surface data use the smoothed three-point function of Yang et al. (2009),
  cited in Sec. 2.2.1.

The paper prints neither formula, so both are written from the cited
definitions.  Their defining properties (sum to one over integer shifts,
vanishing first moment, M4' also vanishing second moment and interpolating,
continuity at the branch points) are checked in tests/test_oracle_kernels.py.
"""
from __future__ import annotations

import numpy as np


def m4prime(r) -> np.ndarray:
    """M4'(r): 1 - 5/2 r^2 + 3/2 |r|^3 on |r|<=1, (2-|r|)^2 (1-|r|)/2 on 1<=|r|<=2."""
    r = np.abs(np.asarray(r, dtype=np.float64))
    inner = 1.0 - 2.5 * r ** 2 + 1.5 * r ** 3
    outer = 0.5 * (2.0 - r) ** 2 * (1.0 - r)
    return np.where(r <= 1.0, inner, np.where(r <= 2.0, outer, 0.0))


def yang3(r) -> np.ndarray:
    """Smoothed three-point delta function (Yang et al. 2009), radius 2."""
    r = np.abs(np.asarray(r, dtype=np.float64))
    s3 = np.sqrt(3.0)
    with np.errstate(invalid="ignore"):
        inner = (17.0 / 48.0 + s3 * np.pi / 108.0 + r / 4.0 - r ** 2 / 4.0
                 + (1.0 - 2.0 * r) / 16.0 * np.sqrt(np.maximum(-12.0 * r ** 2 + 12.0 * r + 1.0, 0.0))
                 - s3 / 12.0 * np.arcsin(np.clip(s3 / 2.0 * (2.0 * r - 1.0), -1.0, 1.0)))
        outer = (55.0 / 48.0 - s3 * np.pi / 108.0 - 13.0 * r / 12.0 + r ** 2 / 4.0
                 + (2.0 * r - 3.0) / 48.0 * np.sqrt(np.maximum(-12.0 * r ** 2 + 36.0 * r - 23.0, 0.0))
                 + s3 / 36.0 * np.arcsin(np.clip(s3 / 2.0 * (2.0 * r - 3.0), -1.0, 1.0)))
    return np.where(r <= 1.0, inner, np.where(r <= 2.0, outer, 0.0))
