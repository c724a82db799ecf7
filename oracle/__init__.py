"""Plain FP64 CPU oracle for one IPCS time step on Taylor-Hood simplices
(P2-P1 on triangles and tetrahedra, P3-P2 on triangles).

THIS PACKAGE IS TEST INFRASTRUCTURE. Only the test suite, the smoke check and
the CPU-baseline leg of the benchmark may import it. The product library never
calls it, links it or falls back to it.

It is a slow, obviously correct NumPy/SciPy implementation of what the paper
(arXiv 2605.25403, FEALPy.CFD) computes for the incremental pressure-correction
scheme (IPCS, Section 2.2.1, eq. (9)) with the Taylor-Hood pair P2-P1
(Section 2.2.1, the spaces V_h and Q_h of eqs. (4)-(5); Section 4.2 selects
Lagrange p=2 for velocity and p=1 for pressure; its higher-order study, table
"convergence_p3_p2", takes p=3 and p=2 on triangles). It shares no code,
tables or constants with the HIP library.

Modules
  quadrature  - cell rules (degree 5; degree 8 for P3-P2) and error rules
  mesh        - structured unit-square / unit-cube simplex meshes
  fem         - P1/P2/P3 spaces, local matrices, COO->CSR assembly, Dirichlet
  krylov      - Jacobi-PCG and Jacobi-BiCGStab (textbook definitions)
  problems    - manufactured solutions (Taylor-Green, John, Beltrami, polynomial)
  ipcs        - the IPCS time step in the paper's order
  steady      - steady Navier-Stokes by Newton's method (monolithic, P2-P1)
  errors      - L2 errors against exact fields

Every function is pinned by a test in tests/ (tests/test_oracle_*.py) against
closed forms, hand-derived matrices, invariants or dense direct solves. The
mixed-precision comparison has no closed-form pin of its own and is reported
as a measured difference ("parity unpinned" for that form only).
"""
