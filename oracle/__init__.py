"""CPU FP64 oracle for the P0 Galerkin capacity computation.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the tests, the smoke check of the entry module and
the CPU-baseline leg of the benchmark use it.  It shares no code with the HIP
library; both sides only share the seeded mesh generators in ``synth``.

It is a plain, slow, obviously correct NumPy implementation of what the GPU
path computes:

* the Galerkin matrix of the single-layer operator on piecewise constants of
  the primal mesh (Appendix A, eq. "discreteform:residual"; the operator is
  eq. "strongform" with kernel 1/(4 pi |x-y|)), using
    - a collapsed (Duffy) tensor Gauss-Legendre rule on each triangle for
      pairs that share no vertex, and
    - Sauter-Schwab-type regularising transformations of the 4-D reference
      integral for pairs that share a vertex, an edge, or are identical;
* the right-hand side b_i = |T_i| (the load <1, chi_i>) and the direct
  (Cholesky) solution of V x = b (Section 2.5, dense direct solve of small
  systems);
* the discrete capacity Cap = (1/4 pi) sum_i x_i |T_i| (eq. "cap:ell" and
  the proof of the capacity proposition);
* ZZ-type indicators for the primal P0 solution (eq. "zz:T", Section 2.4)
  and Doerfler marking (eq. "doerfler");
* the dual-mesh system of the paper's Algorithm 1 (``dual``): barycentric
  V, the projections P and Q_m, the hypersingular matrix, the mass matrix,
  the direct dual solve, its capacity and ZZ indicators (Section 2.6);
* the weighted-residual estimator of the primal solution (``residual``;
  Appendix A, eq. "residual:indicator") with the residual evaluated in the
  discontinuous piecewise linears.

Parity pins are in tests/test_oracle_*.py.  Functions without an independent
pin say "parity unpinned" in their docstring.
"""

from .quadrature import gauss_legendre01, triangle_rule, ss_rule, radon7  # noqa: F401
from .operator import (  # noqa: F401
    element_geometry,
    quad_points,
    classify_pairs,
    near_pairs,
    regular_entry,
    singular_entry,
    entry,
    assemble,
    assemble_rows,
    SSOrders,
)
from .capacity import (  # noqa: F401
    rhs,
    solve_direct,
    solve_cg,
    capacity,
    zz_indicators,
    doerfler,
    mesh_check,
)
from . import dual  # noqa: F401
from . import residual  # noqa: F401
