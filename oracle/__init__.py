"""CPU oracle for the structured-NLP derivative evaluator -- TEST INFRASTRUCTURE.

This package is a plain, slow, deliberately unoptimised reference that the
tests, the smoke check and the benchmark's CPU-baseline leg compare the GPU
library against.  Nothing in the product path may import or call it; the
GPU library fails loudly when its native extension is missing instead of
falling back to anything here.

What it computes (paper Sec. 2.1 callbacks on the SIMD form of Sec. 2.2):
objective, gradient, constraints, COO Jacobian and COO Lagrangian Hessian in
the partially compressed layout of Sec. 5.2, plus the Jacobian/Hessian-vector
products and the parameter adjoint.  How:

* ``rules``   -- the build-time simplification table of Sec. 7.1.2 and the
  sparsity probe of Sec. 5.2 (first-order visit order, second-order pair
  emission, compressor maps, o1step/o2step), written from the paper's
  description;
* ``taylor``  -- second-order forward mode: every node carries its value,
  gradient and Hessian with respect to the pattern's local independents,
  propagated with the textbook chain rule; it shares no code with the GPU
  path;
* ``nlp``     -- the callbacks, assembled from the definitions (sums over
  data points, COO layout, library matvecs for the products).
* ``csc``     -- full compression of the COO output into compressed
  sparse columns (duplicates summed), the solver-side step of Sec. 5.2.

All arithmetic is IEEE float64 (numpy), vectorised over data points.

Parity status: values are pinned by the paper's printed examples, complex
step, finite differences and closed forms (tests/test_oracle_pins.py).  The
slot order of the ACOPF and PDE patterns is not printed in the paper: it is
pinned only through the Rosenbrock probe example, coverage of the dense
Hessian and symmetry ("parity unpinned" for that order beyond the rule).
"""
from .nlp import OracleModel  # noqa: F401
from . import csc, rules, taylor  # noqa: F401
