"""FP64 CPU oracle for the condensed spectral-element p-multigrid solver.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
re-statement of what the method computes (Huismann, Stiller & Froehlich,
"Scaling to the stars -- a linearly scaling elliptic solver for p-multigrid",
arXiv 1808.03595).  Only the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import it.  The GPU product path never calls it and
shares no code with it; the two meet only through the seeded input
generators in the separate ``synth`` package, which hold none of the
method's arithmetic.

Layout of the package:

* ``sem1d``   -- GLL basis, 1D mass/stiffness, generalized eigenpairs,
                 Lagrange interpolation, the degree-7 weight polynomial
                 (Sec. 2.1, eq. (helmholtzop); Sec. 3.2 weight functions).
* ``mesh``    -- Cartesian element meshes, node grids, skeleton index sets,
                 boundary kinds per side: Dirichlet, Neumann, periodic
                 (Sec. 3.3).
* ``dense``   -- dense assembly of H, its Schur complement and the star
                 operators on tiny meshes (plain definitions, Sec. 2.2/2.3).
* ``matfree`` -- matrix-free condensed operator, the star inverse (Alg. 1),
                 the Schwarz smoother (Alg. 2), grid transfers, static
                 condensation and interior recovery.
* ``solver``  -- V-cycle (Alg. 3), MG solver (Alg. 4), ipCG (Alg. 5), the
                 coarse CG, the mixed-precision preconditioner form.
* ``blocks``  -- the element-centred block smoother (Sec. 3.4).
* ``coarse_fd`` -- exact coarse solve by fast diagonalization of the whole
                 coarse mesh.
* ``mlp``     -- the damping-weight MLP: forward, analytic backward, Adam.
* ``dirichlet`` -- inhomogeneous Dirichlet data by lifting (Sec. 3.3
                 boundary treatment, Sec. 5.2 test problem) and its dense
                 brute-force solve.

Every array in this package is float64 unless a function says otherwise.
Global node grids are numpy arrays of shape (N3, N2, N1), x1 fastest,
with N_d = n_d * p + 1; in a periodic direction the last layer mirrors the
first and holds no unknown of its own.
"""
