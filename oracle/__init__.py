"""CPU oracle: a plain, slow, FP64 definition of every step of the solver.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the library and its Python
binding never do.  It shares no code with the GPU path: every table, stencil,
domain solve and Krylov step is written here again from the paper
(Nakamura et al., "Modified Block BiCGSTAB for Lattice QCD"):

* gamma     -- Euclidean chiral gamma basis (the paper leaves the basis open).
* geometry  -- site, neighbour, parity/even-odd and SAP-domain tables.
* dirac     -- Wilson-Dirac operator A = 1 - kappa*H (Sec. 2.1, hopping-term
               equation) with boundary phases; per-site and dense forms;
               domain-restricted (Dirichlet) operator of Sec. 2.2.
* sap       -- minimal-residual domain solver, SAP cycles
               M = K sum_j (1 - A K)^j (Sec. 2.2), exact-inverse variants.
* ssor      -- SSOR domain inverse in Eisenstat form (Sec. 2.2).
* clover    -- clover term and Jacobi (site-diagonal) preconditioning.
* krylov    -- modified Gram-Schmidt QR, modified block BiCGSTAB (Alg. 1),
               its memory-saving form (Alg. 2), textbook right-preconditioned
               BiCGSTAB (van der Vorst 1992) for the L = 1 pin.

Fields are complex128 arrays of shape (V, 4, 3, L) (site, spin, colour,
right-hand side), i.e. the N x L block with row n = 12*site + 3*spin + colour.
"""
