"""Pins for the QP assembly (Appendix "QP Approximation") and the Schur step
(Appendix "ADMM", eq. KKT and the Schur complement system).

* The assembled P, q, C, c, G are checked by evaluating the OCP directly
  (stage sums written independently here) at random points.
* The Schur solution equals the x-part of a dense LU solve of the full
  regularised KKT system [[P + sigma I, A'], [A, -rho^{-1} I]].
* The banded Cholesky used by the oracle equals numpy's dense Cholesky solve.
"""
import numpy as np
import scipy.linalg as sla

from oracle.admm import _QPMats
from oracle.qp import StageQP, lti_qp
from workloads import double_integrator, paper_point_mass_matrices, random_lti


def random_stage_qp(rng, nx=3, nu=2, ng=4, N=5):
    n = nx + nu
    D = np.stack([(lambda M: M @ M.T + 0.1 * np.eye(n))(rng.normal(size=(n, n))) for _ in range(N + 1)])
    E = 0.1 * rng.normal(size=(N, n, n))
    return StageQP(
        nx=nx, nu=nu, N=N, D=D, E=E, q=rng.normal(size=(N + 1, n)),
        Am=rng.normal(size=(N, nx, n)), Ap=rng.normal(size=(N, nx, n)), b=rng.normal(size=(N, nx)),
        x_init=rng.normal(size=nx), G=rng.normal(size=(N + 1, ng, n)),
        lo=-rng.uniform(0.5, 1.5, size=(N + 1, ng)), hi=rng.uniform(0.5, 1.5, size=(N + 1, ng)))


def test_cost_matches_stagewise_sum(rng):
    qp = random_stage_qp(rng)
    P, C, G, q, c, lo, hi = qp.matrices()
    for _ in range(5):
        xs = rng.normal(size=(qp.N + 1, qp.n))
        direct = 0.0
        for t in range(qp.N + 1):
            direct += 0.5 * xs[t] @ qp.D[t] @ xs[t] + qp.q[t] @ xs[t]
        for t in range(qp.N):
            direct += xs[t + 1] @ qp.E[t] @ xs[t]  # block (t+1, t) and its transpose
        x = xs.reshape(-1)
        assert np.isclose(0.5 * x @ (P @ x) + q @ x, direct, rtol=1e-12, atol=1e-12)


def test_constraints_match_stagewise_rows(rng):
    qp = random_stage_qp(rng)
    P, C, G, q, c, lo, hi = qp.matrices()
    xs = rng.normal(size=(qp.N + 1, qp.n))
    rows = [xs[0, : qp.nx] - qp.x_init]
    for t in range(qp.N):
        rows.append(qp.Am[t] @ xs[t] + qp.Ap[t] @ xs[t + 1] - qp.b[t])
    np.testing.assert_allclose(C @ xs.reshape(-1) - c, np.concatenate(rows), atol=1e-12)
    g = np.concatenate([qp.G[t] @ xs[t] for t in range(qp.N + 1)])
    np.testing.assert_allclose(G @ xs.reshape(-1), g, atol=1e-12)


def test_lti_qp_encodes_the_dynamics(rng):
    b = random_lti(2, N=6, seed=77)
    qp = lti_qp(b.A[1], b.B[1], b.Qd[1], b.Rd[1], b.Qfd[1], b.G, b.lo[1], b.hi[1], b.x0[1], b.N)
    P, C, G, q, c, lo, hi = qp.matrices()
    # roll the system forward with random controls: the trajectory satisfies Cx = c
    xs = np.zeros((b.N + 1, b.n))
    xs[0, : b.nx] = b.x0[1]
    for t in range(b.N + 1):
        xs[t, b.nx:] = rng.normal(size=b.nu)
        if t < b.N:
            xs[t + 1, : b.nx] = b.A[1] @ xs[t, : b.nx] + b.B[1] @ xs[t, b.nx:]
    np.testing.assert_allclose(C @ xs.reshape(-1), c, atol=1e-12)
    cost = sum(0.5 * (xs[t, :b.nx] @ (b.Qd[1] * xs[t, :b.nx]) + xs[t, b.nx:] @ (b.Rd[1] * xs[t, b.nx:]))
               for t in range(b.N)) + 0.5 * (xs[-1, :b.nx] @ (b.Qfd[1] * xs[-1, :b.nx]) + xs[-1, b.nx:] @ (b.Rd[1] * xs[-1, b.nx:]))
    x = xs.reshape(-1)
    assert np.isclose(0.5 * x @ (P @ x), cost)


def test_double_integrator_is_the_paper_euler_model():
    A, B = paper_point_mass_matrices(2, 0.1)
    b = double_integrator(1)
    np.testing.assert_array_equal(b.A[0], A)
    np.testing.assert_array_equal(b.B[0], B)


def test_schur_step_equals_full_kkt_solve(rng):
    qp = random_stage_qp(rng)
    M = _QPMats(qp)
    P, C, G = M.P.toarray(), M.C.toarray(), M.G.toarray()
    sigma, rho_f, rho_g = 1e-6, 100.0, 0.1
    A = np.vstack([C, G])
    rho = np.concatenate([np.full(C.shape[0], rho_f), np.full(G.shape[0], rho_g)])
    x = rng.normal(size=qp.nvar)
    z = rng.normal(size=A.shape[0])
    y = rng.normal(size=A.shape[0])
    # full KKT of the primal update (eq. KKT)
    K = np.block([[P + sigma * np.eye(qp.nvar), A.T], [A, -np.diag(1.0 / rho)]])
    rhs = np.concatenate([sigma * x - M.q, z - y / rho])
    full = np.linalg.solve(K, rhs)[: qp.nvar]
    # the oracle's Schur route: S x~ = eta, banded Cholesky
    eta = sigma * x - M.q + A.T @ (rho * z - y)
    cf = M.factor(sigma, rho_f, rho_g)
    xt = sla.cho_solve_banded((cf, True), eta)
    np.testing.assert_allclose(xt, full, rtol=1e-9, atol=1e-11)


def test_banded_cholesky_equals_dense(rng):
    qp = random_stage_qp(rng, nx=4, nu=2, ng=3, N=9)
    M = _QPMats(qp)
    S = M.schur(1e-6, 30.0, 0.7).toarray()
    eta = rng.normal(size=S.shape[0])
    cf = M.factor(1e-6, 30.0, 0.7)
    np.testing.assert_allclose(sla.cho_solve_banded((cf, True), eta), np.linalg.solve(S, eta), rtol=1e-10)
    L = np.linalg.cholesky(S)
    np.testing.assert_allclose(cf[0], np.diag(L), rtol=1e-12)
