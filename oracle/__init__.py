"""CPU FP64 oracle for the block-acoustic preconditioned elastic Helmholtz solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links this package: only the tests, the smoke check and the benchmark's CPU
baseline leg may use it.  It shares no code with the GPU library; the two
meet only in the seeded input generators of the ``workloads`` module.

The oracle is plain, slow and meant to be checked by eye against the paper
(Yovel & Treister, "A block-acoustic preconditioner for the elastic Helmholtz
equation"):

* ``elastic``   -- the MAC discretisation of the mixed displacement-pressure
  system H = [A B^T; B -C] (Section 2.1, eq. mixed-discretized), the shear
  and pressure acoustic operators A_p and H_p (eqs. Ap, Hp), the complex shift
  (eq. shift) and the absorbing layer (Section 4).
* ``multigrid`` -- full-weighting restriction and bilinear/trilinear
  prolongation (eqs. Ru1, Rp), Galerkin coarsening (eq. galerkin), damped
  Jacobi, V- and W-cycles (Algorithm TwoCycle) and the coarsest direct solve.
* ``precond``   -- the distributor and the block-triangular preconditioner
  (eqs. mixed-distributor, mixed-distributed, prec).
* ``fgmres``    -- right-preconditioned flexible GMRES(m) (Saad 1993).
* ``analysis``  -- the commutator (eq. commutator) and the matrices of
  Theorem 3.1 (eqs. Z, precond_system, error_iter_mat).
* ``fwi``       -- least-squares misfit and its gradient with respect to
  per-cell vp, vs, rho through an adjoint solve.

Every function is pinned by a test in ``tests/test_oracle_*.py`` against
something other than itself (printed tables of the paper, closed forms,
exact identities, brute force).  A function without such a pin says
"parity unpinned" in its docstring.
"""
