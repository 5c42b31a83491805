"""CPU oracle for the coupled-channel R-matrix internal-region solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, link or run anything in this package; only
the tests, the smoke check and the benchmark's CPU-baseline leg do.

It is a plain, slow, FP64 implementation of what the paper computes, written
from the paper's statement of the method (Sec. 2 and Sec. 3.1) plus the
standard Lagrange-mesh / R-matrix relations the paper defers to its
references, each one pinned by tests against values that do not come from
this package:

* ``mesh``     -- Lagrange-Legendre mesh on (0, a), basis functions f_i(r),
                  kinetic + Bloch matrix by quadrature of its definition,
                  surface values q_i = f_i(a).
* ``system``   -- block matrix M (Eq. block_structure) and surface
                  right-hand sides B (Sec. 3.1, step 2).
* ``ge``       -- plain Gaussian elimination with partial pivoting (C).
* ``rmatrix``  -- R-matrix extraction (Sec. 3.1, step 4, with the
                  hbar^2/2mu a factor), Coulomb functions (mpmath), collision
                  matrix by matching, channel cross sections.
* ``pipeline`` -- one energy end to end.
"""
