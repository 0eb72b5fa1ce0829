"""Pins for the implicit-differentiation VJP (Algorithm 2; Appendix
"Backward Pass").

* Central finite differences (h = 1e-6) of exactly solved (polished) QPs.
* Closed form: with no inequality active, x_N = Phi x0 and u_0 = -K_0 x0
  (LQR), so dL/dx0 = 2 (K_0'K_0 + Phi'Phi) x0 for L = ||u_0||^2 + ||x_N||^2.
* The regularised iterative-refinement adjoint equals the dense solve.
"""
import numpy as np

from oracle.adjoint import adjoint_dense, adjoint_refined
from oracle.lti import (fd_theta_grad, implicit_theta_grad, loss_and_grad_x, qp_of_theta,
                        theta_of)
from workloads import random_lti


def test_implicit_gradient_matches_central_fd():
    b = random_lti(2, N=16, seed=4)
    for i in range(2):
        L, g, sol = implicit_theta_grad(b, i)
        assert sol["lower"].sum() + sol["upper"].sum() > 0  # constraints are active
        fd = fd_theta_grad(b, i, sol=sol)
        np.testing.assert_allclose(g, fd, rtol=1e-5, atol=1e-6 * max(1.0, np.abs(fd).max()))


def test_gradient_wrt_x0_is_lqr_closed_form():
    b = random_lti(2, N=12, seed=43, x_bound=1e4, u_bound=1e4)
    nx, nu, N = b.nx, b.nu, b.N
    for i in range(2):
        L, g, sol = implicit_theta_grad(b, i)
        assert sol["lower"].sum() + sol["upper"].sum() == 0
        A, B, Q, R = b.A[i], b.B[i], np.diag(b.Qd[i]), np.diag(b.Rd[i])
        P = np.diag(b.Qfd[i])
        Ks = []
        for t in range(N - 1, -1, -1):
            K = np.linalg.solve(R + B.T @ P @ B, B.T @ P @ A)
            P = Q + A.T @ P @ (A - B @ K)
            Ks.insert(0, K)
        Phi = np.eye(nx)
        for t in range(N):
            Phi = (A - B @ Ks[t]) @ Phi
        x0 = b.x0[i]
        expect = 2.0 * (Ks[0].T @ Ks[0] + Phi.T @ Phi) @ x0
        np.testing.assert_allclose(g[nx + nu: 2 * nx + nu], expect, rtol=1e-7, atol=1e-9)


def test_refinement_equals_dense_adjoint():
    b = random_lti(1, N=20, seed=44)
    L, g, sol = implicit_theta_grad(b, 0)
    qp = qp_of_theta(b, 0, theta_of(b, 0))
    _, gx = loss_and_grad_x(qp, sol["x"])
    e1 = adjoint_dense(qp, sol["x"], gx, sol["lower"], sol["upper"])
    e2 = adjoint_refined(qp, sol["x"], gx, sol["lower"], sol["upper"], sweeps=6)
    for a, c in zip(e1, e2):
        np.testing.assert_allclose(c, a, rtol=1e-10, atol=1e-12 * max(1.0, np.abs(a).max()))
