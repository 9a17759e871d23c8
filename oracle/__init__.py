"""Plain FP64 CPU oracle for the Fast-Diagonalization (FD) preconditioner apply.

This package is TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import or call it. The product
path (the HIP library and its Python binding) never imports it, and it never
imports the product path. The two share no code; only the seeded input
generators in ``paper_1712_00403_amd.workloads`` (random draws and problem
descriptors, no arithmetic of the method) serve both.

Every function is written from the paper (Montardini, Sangalli, Tani,
"Robust isogeometric preconditioners for the Stokes system based on the Fast
Diagonalization method", 2018) and cites the passage it follows:

* ``bspline``   -- open knot vectors and the Cox-de Boor recursion (Sec. 2.1),
                   Gauss-Legendre quadrature.
* ``assemble``  -- univariate stiffness/mass factors of the simple P_V and P_Q
                   (Sec. 5, factors below eq. prec3D_TH and eq. precQ) and
                   their weighted versions (Appendix).
* ``geneig``    -- generalized eigendecomposition K U = M U D, U^T M U = I
                   (Sec. 5.2, eq. eig_dec), by Cholesky reduction and cyclic
                   Jacobi.
* ``fd``        -- Algorithm 1 (Sec. 5.2) with m-mode products (Sec. 2.3), the
                   pressure-mass solve by banded per-mode solves (Sec. 5.2,
                   first paragraph) and the block-diagonal P_D (eq. P_D).
* ``brute``     -- the same operators assembled as explicit Kronecker sums and
                   solved directly (tiny grids only).
* ``geometry``  -- the coefficient-aware variant (Sec. 6 and Appendix).

Readings where the paper is silent or garbled (direction ordering of the
Kronecker products, quadrature order, the separable-approximation iteration)
are stated in the docstrings of the functions that take them.
"""
