"""FP64 CPU oracle for the SCVT hot path.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg may import it.  The product path (the HIP library and its
Python binding) never imports, links or calls anything here, and nothing here
imports the product package.

    voronoi  -- Delaunay triangulation as the convex hull, Voronoi cells
    scvt     -- cell integrals (C, scvt_oracle.c), energy, gradient, Lloyd
                preconditioner and step, two-loop recursion, P-LBFGS loop
                (and the compared methods: Lloyd, plain LBFGS)
    mesh     -- bisection, Delaunay triangle list, cellQ and triQ

Parity notes: every function here is pinned by the `-m "not gpu"` tests
(closed forms, brute force, invariants); see tests/test_oracle_*.py.
Parity unpinned: the line-search constants (alpha0 = 1, factor 1/2,
c1 = 1e-4, ten evaluations) and the curvature-skip threshold
(y.s > 1e-10 |y||s|) are conventions of this reading, not values the paper
fixes; both sides implement the same ones.  Converged meshes beyond the
energy statistics are unpinned too (the energy has many local minima).
"""
from ._clib import build  # noqa: F401
from .scvt import (Evaluation, LineSearchError, Solver, cell_integrals, dot, evaluate, local_cell,  # noqa: F401
                   normalize_rows, two_loop)
from .voronoi import cells, circumcentres, delaunay, neighbour_sets  # noqa: F401
from . import mesh  # noqa: F401
