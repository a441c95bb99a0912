"""Plain FP64 CPU oracle for the proxy-surface fast direct solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute anything in this package; only the test-suite, the smoke
check and the CPU-baseline leg of the benchmark use it.  It shares no code
with the GPU implementation: the only common dependency is the seeded input
generator in ``synthetic`` (vertex coordinates and incidence angles).

Contents (each function cites the passage of the paper it follows):

* ``special``   Hankel functions (library routine) and the ascending series of
                the two cancelling combinations that enter the elastodynamic
                fundamental solution (equation of the fundamental solution).
* ``kernels``   per-point integrands of the regularised Galerkin form of the
                Burton-Miller operator D + alpha N (Sections 3 and 5.2).
* ``quadrature``  the element-pair quadrature rules that define the discrete
                operator.
* ``galerkin``  entries of the 2N x 2N Galerkin matrix for arbitrary row and
                column DOF lists, load vectors (Section 5.2).
* ``dense``     the conventional dense BEM ("Conv" in Section 8): assemble
                and LU-solve.
* ``series``    closed-form series for plane-P scattering by a circular cavity.
* ``fds``       the fast direct solver, step by step (Sections 6, 7.1-7.3).
"""
