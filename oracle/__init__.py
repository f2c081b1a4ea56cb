"""FP64 CPU oracle for the NeuRLP-PDE least-squares solve (Mechanistic PDE
Networks, arXiv 2502.18377).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, the smoke check in
``__graft_entry__.py`` and the ``cpu_baseline`` leg of ``bench.py`` use it.
It shares no code with the HIP path (no kernels, headers, helpers, tables or
constant generators); both sides only consume the seeded inputs produced by
the ``workloads`` package.

What it computes (the plain definitions, in the paper's order):

* ``stencil``  -- 5-point finite-difference weights of the central-difference
  constraints (Sec. "Linear PDE Solving With Differentiable Optimization",
  Eq. 5 and the sentence after it), obtained by solving the moment system
  in exact rational arithmetic.
* ``system``   -- assembly of the sparse constraint matrix ``A`` and vector
  ``d`` of Eq. 8 from the equation rows (Eq. 3), initial/boundary rows
  (Eq. 4), central-difference rows (Eq. 5) and forward/backward Taylor
  smoothness rows (Eqs. 6-7).
* ``solve``    -- the least-squares solution of Eq. 8: the saddle-point
  (KKT) system of Eq. 10 factored by a sparse direct LU, cross-checked by a
  sparse LU of the normal equations (Eq. 9) and by a dense least-squares
  solve; the dual ``lambda* = d - A z*``; the normal-equation residual.
* ``adjoint``  -- the backward saddle-point system of Eq. 11 and the
  gradient formulas that follow it (d_A l = d_lambda z*^T + lambda* d_z^T,
  d_d l = -d_lambda), chained to the coefficient fields, the source and the
  boundary data; central finite differences of the same loss.

Readings of the paper that the canonical system fixes (all pinned by tests
under ``tests/``): a grid of "32x32" has 32 points per axis; each point
carries u and the first and second derivative along every axis (V = 1+2D
variables); equation rows exist at every grid point, boundary rows once per
constrained point, Taylor rows wherever the neighbour exists (everywhere on a
periodic axis) and both central-difference rows at every point, with
one-sided 5-point windows at the edges of non-periodic axes.  These are the
only choices that reproduce the variable and constraint counts the paper
prints for 32x32 and 32x32x32 grids (Sec. "Scaling PDE Solving").

Parity status: every function here is pinned by at least one test that does
not re-type its formula (printed counts, textbook stencil tables, exactness on
quadratics, translation invariance, dense brute force, LS optimality,
manufactured-solution convergence, finite differences).
"""

from .stencil import fd_weights, window_offsets  # noqa: F401
from .system import OracleProblem, assemble, variable_count  # noqa: F401
from .solve import (  # noqa: F401
    solve_kkt, solve_normal_lu, solve_dense_lstsq, normal_residual,
    cg_normal, dual,
)
from .adjoint import adjoint_kkt, grad_A_entries, chain_gradients, fd_gradient  # noqa: F401
