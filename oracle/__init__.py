"""FP64 CPU oracle for the batched SQP-ADMM optimal-control solver.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The product path
(the HIP library and its Python binding) never calls it and has no CPU
fallback.

Everything here is plain NumPy/SciPy in double precision, one instance at a
time, written from the paper's definitions:

* ``qp``       - OCP -> QP assembly (Appendix "QP Approximation").
* ``models``   - LTI and kinematic-bicycle OCP functions (cost, dynamics,
                 inequalities) with analytic derivatives.
* ``admm``     - the QP solver of Algorithm 3 (OSQP splitting with the
                 smoothed slack projection), Schur step by a library banded
                 Cholesky.
* ``sqp``      - Algorithm 1 with the backtracking line search
                 (Appendix "Line search").
* ``adjoint``  - active-set identification and the implicit-differentiation
                 VJP of Algorithm 2 / Appendix "Backward Pass", by a dense
                 direct solve of the active-set KKT system, plus the
                 regularised iterative-refinement variant.
* ``polish``   - active-set polish of an ADMM solution into an exact KKT point.

Parity status of each function is listed in its docstring.
"""
