"""FP64 CPU oracle for the multi-shift twisted-mass solver.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The product path (the
HIP library and its Python binding) never imports, links or executes it, and
it shares no code with that path: the only common dependency is the seeded
input generator module ``synth``.

Contents (each function cites the passage of the paper it follows):

* ``lattice``   gamma matrices, Wilson hopping sum, D_W, the non-degenerate
                doublet D_ND, its site block A and closed-form inverse, the
                even-odd Schur complement S and Q = (Gamma5 x tau1) S.
* ``dense``     brute-force dense matrices assembled site by site (tiny lattices).
* ``solvers``   CG, multi-shift CG, Lagrange guesses, the difference-of-single-
                solves identity (case C), GMRES.
* ``mg``        aggregation prolongator, restriction/prolongation, Galerkin
                coarse operator, the odd-site shift term on the coarse grid.
* ``smoothers`` the cycle's post-smoothers: minimal-residual steps on the whole
                lattice, and the Schwarz alternating procedure (SAP) over two colours
                of blocks with minimal-residual block solves.
* ``mlp``       FP64 forward/backward/Adam for the guess-proposer network and
                its Gram-form loss.
* ``fp16``      half-precision storage codec with per-site scale.
"""
