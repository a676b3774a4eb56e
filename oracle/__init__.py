"""Plain CPU FP64 oracle of the closest point method (CPM) with interior
boundary conditions (King, Su, Aanjaneya, Ruuth, Batty, "A Closest Point
Method for PDEs on Manifolds with Interior Boundary Conditions for Geometry
Processing", ACM TOG 2024, arXiv 2305.04711).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, constant or
helper with the HIP library under ``paper_2305_04711_amd/``.

The oracle is slow on purpose: it builds the band by a bounding-box scan (and,
for checking, by the breadth-first search of Algorithm 1), stores the
closest-point extension E and the Laplacian L explicitly as CSR matrices as the
paper does (Sec. 5.3), and applies the operator by the paper's four-step
matrix-vector product (Sec. 5.4).  All arithmetic is IEEE FP64 in the order
written (numpy never contracts a*b+c into an FMA).

Modules
  geometry  closest-point functions cp_S, cp_C and orientation vectors (App. A)
  band      Omega(S) (eq. bandwidth, Alg. 1), Omega(C) and the check region
            (Sec. 4.1, 4.6), side vectors (eq. cpdiff, Sec. 4.2)
  operator  stencils, swaps, BC-DOF rows (Sec. 4.3), E and L (Sec. 5.3), the
            system A = mI + n[diag L + (L - diag L)E] (Sec. 5.4), the RHS
  krylov    dense LU, BiCGSTAB (van der Vorst), GMRES(k)
  adjoint   transposed operator and gradients of a quadratic loss
  local     the operator evaluated row by row (sampled rows of large bands)
  timestep  Crank-Nicolson steps of the heat equation (Sec. 6.2)

Parity status: every function is pinned by the CPU tests in
``tests/test_oracle_*.py`` (closed forms, invariants, brute force); none is
"parity unpinned".
"""

from . import geometry, band, operator, krylov, adjoint, local, timestep  # noqa: F401
