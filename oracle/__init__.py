"""Plain FP64 CPU oracle for the enriched Taylor-Hood (Q2 velocity, Q1 + P0
pressure frame) Stokes and Oseen systems of Pestana & Silvester,
"Fast solution of incompressible flow problems with two-level pressure
approximation" (arXiv 2303.10233).

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and
the CPU-baseline leg of the benchmark may import it.  The GPU library never
calls it, and it shares no code with the GPU path: element matrices here are
computed by Gauss quadrature from the basis-function definitions, assembled
element by element into SciPy sparse matrices, and solved with SuperLU or with
Krylov methods written out from the paper.

Module map
----------
fem       basis functions, quadrature, element matrices (Sec. 2.1, eq:stokes_fe)
assemble  global sparse matrices, Dirichlet data and the lifted RHS
          (eq:saddle_point, eq:oseen-system)
direct    bordered sparse direct solve, canonicalisation, adjoint gradients
krylov    preconditioned MINRES (alg:minres) and flexible GMRES (Sec. 3)
precond   block preconditioners P1, diagonal / Chebyshev-SGS pressure-mass
          solves (Sec. 2.2-2.3), geometric multigrid, PCD (Sec. 3.1) and the
          two-stage driver (Sec. 3.1, full-system / reduced-system), the
          P0-elimination multigrid for M_Q (Sec. 2.3)
infsup    inf-sup constant (Sec. 2.4) and its EST-MINRES estimate
picard    fixed-point (Picard) steps of the steady Navier-Stokes equations
          that produce the Oseen systems of Sec. 3, and their residual

Every function is pinned by a test in ``tests/test_oracle_*.py`` against a
closed form, a brute-force computation or an identity the paper states; the
functions without such a pin say "parity unpinned" in their docstring.
"""
