"""Plain FP64 CPU oracle for the grid-based potential-flow solve of
Beckers & Eldredge, "Planar potential flow on Cartesian grids" (arXiv 2102.11910).

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) imports, calls or links anything in this package; only the
test suite, the smoke check and the CPU-baseline leg of the benchmark do.
It shares no code with the GPU path: no kernels, tables, constants or
helpers.  Inputs come from the seeded generators, which hold none of the
method's arithmetic.

Everything is float64 NumPy/SciPy, written for a reader to check against the
paper by eye:

* ``lgf``       lattice Green's function of the 5-point Laplacian (Sec. 2.1)
* ``kernels``   the M4' and smoothed 3-point discrete delta functions (Fig. 1)
* ``operators`` regularization / interpolation, L and L^-1, velocities (Sec. 2.1-2.2)
* ``body``      Schur complement S, f0, Gamma0, circulation removal (Sec. 2.2-2.3)
* ``solve``     the constrained solves: prescribed circulation, steady Kutta,
                Kutta with shed vortices at m edges (Sec. 2.3-2.4), and one
                explicit-midpoint step of vortex advection

Every function is pinned by a CPU test against values the mathematics or the
paper fixes (closed forms, invariants, brute force on tiny inputs); see
``tests/test_oracle_*.py``.  Parity of the two derived far-field checks of the
time-stepping trajectory is unpinned (chaotic), only single steps are gated.
"""

from . import lgf, kernels, operators, body, solve  # noqa: F401
