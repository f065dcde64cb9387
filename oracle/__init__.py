"""FP64 CPU oracle for the SymX element-derivative / BSR-assembly / Newton path.

TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  The HIP library never calls it, and
the two share no code: the oracle's derivatives are derived by hand from the
paper's energy definitions, while the library's come from its own symbolic
differentiator.

Contents (each module cites the passage it follows):
  elements.py    per-element energy, gradient and Hessian (Stable Neo-Hookean
                 tet4, StVK triangle membrane, quadratic bending hinge, inertia)
  rest.py        Lame parameters, rest-shape quantities, lumped masses
  assembly.py    brute-force sparsity pattern, scatter map, assembly into 3x3
                 BSR in element-id order, Dirichlet treatment
  projection.py  per-element projection of Hessians onto the PSD cone
  newton.py      block-Jacobi PCG and the Newton step with backtracking line
                 search and time-step halving

Parity status: every function here is pinned by tests/test_oracle_pins.py
(complex-step derivatives, closed forms at rest, invariants, brute force).
No function is "parity unpinned".
"""
from . import elements, rest, assembly, projection, newton  # noqa: F401
