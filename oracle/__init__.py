"""FP64 CPU oracle for the space-time heat-conduction solve (Alexandersen & Appel,
arXiv 2508.09589).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or link
anything in this package; only the test-suite, the smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code with the HIP library:
it assembles the system matrix from element matrices with scipy.sparse and
solves it directly, so that every GPU result can be checked against the exact
discrete solution.

Modules
  grid       -- node/element numbering, Dirichlet set                 (§3.1.2, §2.3)
  element    -- element matrices: Kronecker form and brute-force quadrature (§3.1.1)
  assemble   -- SIMP coefficients, global matrix, load, Dirichlet elimination
  solve      -- sparse LU + refinement, block Gauss-Seidel in time, adjoint
  hierarchy  -- semi-coarsening level choice (Algorithm 1)
  multigrid  -- trilinear prolongation, masks, Galerkin operators (§3.2)
  krylov     -- Jacobi-GMRES, V-cycle and FGMRES written from their definitions
  design     -- PDE filter, objective, adjoint sensitivities (§3.3)
  residual   -- matrix-free residual at sampled nodes for full-size checks

Every function states the passage of the paper it follows.  Where the paper is
silent the reading taken is stated in the docstring.  Parity unpinned: none of
the functions here is unpinned -- each has a check in tests/test_oracle_*.py
against a closed form, an invariant, a brute-force construction or a printed
value of the paper.
"""
