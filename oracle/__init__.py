"""CPU FP64 oracle for K-GRAPE (Larocca & Wisniacki, arXiv 2010.03598).

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
GPU library is checked against.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product path (the HIP
library and its Python binding) never does, and this package imports nothing
from the product path.

Modules
-------
model     the open XXZ chain and its control operators (Sec. III.A, Eqs. 6 and 10),
          built three independent ways: Kronecker products of spin matrices,
          bit operations into a sparse matrix, and a matrix-free bit apply.
krylov    the Lanczos basis (App. A, Algorithm 2) and the Krylov propagator
          (Eqs. A1-A3), FP64 throughout.
grape     the GRAPE sweeps of Algorithm 1 with Krylov propagation: forward
          states, overlap and fidelity (Eq. 2), backward costates and the
          zeroth-order gradient (Eq. 5); the plain gradient-ascent update.
exact     plain definitions the method approximates: dense propagators by
          diagonalisation (Eq. B2, B12), the exact piecewise-constant gradient
          (Eqs. B3-B5) by Daleckii-Krein divided differences and by Van Loan's
          block exponential, quadrature of the natural gradient (Eqs. B7-B8),
          and central finite differences.
dimension the Krylov dimension of the batched form: the smallest m whose a-priori
          error bound (Hochbruck-Lubich) meets a requested accuracy per slice.

Every function is pinned by tests marked ``not gpu`` against closed forms,
invariants, brute force and library routines (see tests/test_oracle_*.py).
"""

from . import model, krylov, grape, exact, dimension  # noqa: F401
