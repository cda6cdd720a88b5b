"""CPU FP64 oracle for the Laplace-Beltrami double-layer solver.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The GPU library never
calls it and shares no code with it.

It is the plain definition of what the method computes, written from
Kropinski & Nigam, "Fast integral equation methods for the Laplace-Beltrami
equation on the sphere":

* geometry.py -- island curves on the sphere and their stereographic images
  (Section 3) with the analytic parameter derivatives the Nystrom rule needs
  (Section 5).
* nystrom.py  -- the dense Nystrom system of eq. matrix_eqns (Section 5):
  the double-layer operator I + K of eq. disc_sphere, the log-source block E,
  the constraint rows F and D; LU solve; a row-blocked direct O(N^2) matvec;
  the same kernel in its sphere form (Appendix A, eq. kern1) as a cross-check.
* gmres.py    -- GMRES(m) on the left-preconditioned system of
  eq. matrix_eqns_c with the Schur-complement block preconditioner.
* evaluate.py -- the representation of eq. eqn:u_multi at sphere targets.
* adjoint.py  -- gradients of a target misfit by the dense adjoint.

Readings of the paper where it is silent, ambiguous or garbled (each is
pinned by a test in tests/test_oracle_pins.py):

* Correction-term sign: the planar kernel's correction enters with "+",
  Re{(1/2 pi i) sigma [1/(xi - xi') + conj(xi')/(1 + |xi'|^2)] dxi'}, which is
  what differentiating eq. fundC gives; the printed "-" (eqs. dlpC,
  stereo:simple, disc_sphere) is a typo.
* Kernel scale: the per-parameter kernel carries 1/(2 pi) and the equation
  keeps the factor 2h of eq. disc_sphere.
* Diagonal: the exact limit of the off-diagonal Cauchy term,
  -Im(xi''/(2 xi')), so no curvature sign convention is needed.
* Orientation: each curve's sign s_k is +1 when its island lies to the left
  of the planar traversal.
* Inverse projection: x3 = (|xi|^2 - 1)/(|xi|^2 + 1) (the printed sign
  contradicts the forward map); the oracle never inverts the projection.
* Back-substitution of the block preconditioner: z_sigma = r_sigma - E z_a.
* Island 0 is the one without a constraint row; row 0 of the a-block is
  sum(A) = 0; constraint weights are 1 per node; nodes are t_j = 2 pi j / N_k,
  j = 0..N_k-1.
"""
