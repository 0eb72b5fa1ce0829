"""Pins for the oracle's Algorithm 3 (ADMM QP solve).

* KKT certificate: the polished active-set solution is primal feasible, has
  correctly signed multipliers and zero KKT residuals; ADMM converges to it.
* Brute force: on a tiny problem every one of the 3^m active patterns is
  solved as an equality-constrained QP; the feasible, correctly-signed one is
  the optimum and matches ADMM.
* Closed form: with no inequality active the solution is the finite-horizon
  LQR solution (Riccati recursion), including the dynamics multipliers
  y_dyn_t = P_{t+1} x_{t+1} and y_init = -P_0 x_0.
* Soft rows: L1 and L2 slack QPs match an independent SLSQP solve of the
  slack-variable formulation.
* Iterate invariants: nonzero multipliers only on rows whose z sits on the
  matching bound; residuals decrease to the tolerance.
"""
import itertools

import numpy as np
import pytest
from scipy.optimize import minimize

from oracle.adjoint import polish
from oracle.admm import ADMMSettings, admm_solve, kkt_residuals
from oracle.qp import SOFT_L1, SOFT_L2, StageQP, lti_qp
from workloads import double_integrator, random_lti

TIGHT = ADMMSettings(eps_abs=1e-11, eps_rel=1e-11, max_iter=50000)


def tiny_qp(rng, soft=None):
    nx, nu, N = 2, 1, 2
    A = np.array([[1.0, 0.2], [-0.1, 1.05]])
    B = np.array([[0.0], [0.3]])
    G = np.array([[1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])  # x[0] and u boxed
    qp = lti_qp(A, B, np.array([1.0, 0.5]), np.array([0.2]), np.array([3.0, 3.0]), G,
                np.array([-0.6, -0.5]), np.array([0.6, 0.5]), np.array([0.5, -0.8]), N)
    qp.q[:] = rng.normal(scale=0.5, size=qp.q.shape)
    if soft is not None:
        qp.soft = np.array(soft)
        qp.gamma1 = 0.7
        qp.gamma2 = 2.0
    return qp


def brute_force(qp):
    P, C, G, q, c, lo, hi = (m.toarray() if hasattr(m, "toarray") else m for m in qp.matrices())
    m = G.shape[0]
    best = None
    nv, ne = qp.nvar, qp.neq
    for pat in itertools.product((-1, 0, 1), repeat=m):
        pat = np.array(pat)
        act = pat != 0
        GA = G[act]
        bA = np.where(pat < 0, lo, hi)[act]
        K = np.block([[P, C.T, GA.T], [C, np.zeros((ne, ne)), np.zeros((ne, GA.shape[0]))],
                      [GA, np.zeros((GA.shape[0], ne)), np.zeros((GA.shape[0], GA.shape[0]))]])
        if np.linalg.matrix_rank(K) < K.shape[0]:
            continue  # active rows dependent on the equality rows: no unique multipliers
        sol = np.linalg.solve(K, np.concatenate([-q, c, bA]))
        x = sol[:nv]
        assert np.allclose(C @ x, c, atol=1e-9)
        yA = sol[nv + ne:]
        g = G @ x
        feas = np.all(g >= lo - 1e-10) and np.all(g <= hi + 1e-10)
        sign_ok = np.all(yA[pat[act] < 0] <= 1e-10) and np.all(yA[pat[act] > 0] >= -1e-10)
        if feas and sign_ok:
            obj = 0.5 * x @ P @ x + q @ x
            if best is None or obj < best[0] - 1e-12:
                best = (obj, x)
    return best


def test_admm_matches_brute_force_enumeration(rng):
    for _ in range(4):
        qp = tiny_qp(rng)
        best = brute_force(qp)
        r = admm_solve(qp, TIGHT)
        assert r.status == 0
        np.testing.assert_allclose(r.x, best[1], atol=1e-7)


def test_kkt_certificate_on_random_lti():
    b = random_lti(3, N=20, seed=31)
    for i in range(3):
        qp = lti_qp(b.A[i], b.B[i], b.Qd[i], b.Rd[i], b.Qfd[i], b.G, b.lo[i], b.hi[i], b.x0[i], b.N)
        r = admm_solve(qp, TIGHT)
        assert r.status == 0
        ok, sol = polish(qp, r.x, r.y_g, eps_solve=1e-8)
        assert ok
        np.testing.assert_allclose(r.x, sol["x"], atol=1e-7)
        rp, rd, _, _ = kkt_residuals(qp, sol["x"], sol["z_g"], sol["xi"], sol["y_f"], sol["y_g"])
        assert rp < 1e-10 and rd < 1e-9


def _lqr(A, B, Q, R, Qf, x0, N):
    P = [None] * (N + 1)
    K = [None] * N
    P[N] = Qf
    for t in range(N - 1, -1, -1):
        K[t] = np.linalg.solve(R + B.T @ P[t + 1] @ B, B.T @ P[t + 1] @ A)
        P[t] = Q + A.T @ P[t + 1] @ (A - B @ K[t])
    xs, us = [x0], []
    for t in range(N):
        us.append(-K[t] @ xs[-1])
        xs.append(A @ xs[-1] + B @ us[-1])
    return np.array(xs), np.array(us), P


def test_unconstrained_case_is_lqr():
    b = random_lti(2, N=15, seed=41, x_bound=1e4, u_bound=1e4)
    for i in range(2):
        qp = lti_qp(b.A[i], b.B[i], b.Qd[i], b.Rd[i], b.Qfd[i], b.G, b.lo[i], b.hi[i], b.x0[i], b.N)
        r = admm_solve(qp, TIGHT)
        xs, us, Pr = _lqr(b.A[i], b.B[i], np.diag(b.Qd[i]), np.diag(b.Rd[i]), np.diag(b.Qfd[i]), b.x0[i], b.N)
        z = r.x.reshape(b.N + 1, b.n)
        np.testing.assert_allclose(z[:, : b.nx], xs, atol=1e-7)
        np.testing.assert_allclose(z[: b.N, b.nx:], us, atol=1e-7)
        np.testing.assert_allclose(z[b.N, b.nx:], 0.0, atol=1e-8)
        y = r.y_f.reshape(b.N + 1, b.nx)
        np.testing.assert_allclose(y[0], -Pr[0] @ xs[0], atol=1e-6)
        for t in range(b.N):
            np.testing.assert_allclose(y[t + 1], Pr[t + 1] @ xs[t + 1], atol=1e-6)


@pytest.mark.parametrize("kind", [SOFT_L1, SOFT_L2])
def test_soft_rows_match_slsqp(rng, kind):
    for _ in range(2):
        qp = tiny_qp(rng, soft=[kind, 0])
        qp.lo[:, 0] = -0.2  # make the soft row bind
        qp.hi[:, 0] = 0.2
        P, C, G, q, c, lo, hi = (m.toarray() if hasattr(m, "toarray") else m for m in qp.matrices())
        nv = qp.nvar
        soft = qp.soft_rows() == kind
        ns = int(soft.sum())
        S = np.zeros((G.shape[0], ns))
        S[np.flatnonzero(soft), np.arange(ns)] = 1.0

        # variables (x, s_plus, s_minus); xi = s_plus - s_minus on soft rows
        def obj(v):
            x, sp_, sm = v[:nv], v[nv:nv + ns], v[nv + ns:]
            pen = qp.gamma1 * np.sum(sp_ + sm) if kind == SOFT_L1 else 0.5 * qp.gamma2 * np.sum((sp_ - sm) ** 2)
            return 0.5 * x @ P @ x + q @ x + pen

        cons = [{"type": "eq", "fun": lambda v: C @ v[:nv] - c},
                {"type": "ineq", "fun": lambda v: (G @ v[:nv] + S @ (v[nv:nv + ns] - v[nv + ns:])) - lo},
                {"type": "ineq", "fun": lambda v: hi - (G @ v[:nv] + S @ (v[nv:nv + ns] - v[nv + ns:]))}]
        bounds = [(None, None)] * nv + [(0, None)] * (2 * ns)
        ref = minimize(obj, np.zeros(nv + 2 * ns), method="SLSQP", constraints=cons, bounds=bounds,
                       options={"ftol": 1e-15, "maxiter": 2000})
        assert ref.success
        r = admm_solve(qp, TIGHT)
        assert r.status == 0
        np.testing.assert_allclose(r.x, ref.x[:nv], atol=2e-5)
        assert np.any(np.abs(r.xi) > 1e-3)  # the slack is in use


def test_iterate_invariants_and_residual_decrease():
    b = double_integrator(1)
    qp = lti_qp(b.A[0], b.B[0], b.Qd[0], b.Rd[0], b.Qfd[0], b.G, b.lo[0], b.hi[0], b.x0[0], b.N)
    r = admm_solve(qp, ADMMSettings(max_iter=200, k_check=0, adapt_rho=False), record=True)
    lo, hi = qp.lo.reshape(-1), qp.hi.reshape(-1)
    for (x, z, xi, yf, yg) in r.history:
        assert np.all(z >= lo - 1e-15) and np.all(z <= hi + 1e-15)
        assert np.all(z[yg > 1e-12] == hi[yg > 1e-12])
        assert np.all(z[yg < -1e-12] == lo[yg < -1e-12])
        assert np.all(xi == 0.0)
    res = [kkt_residuals(qp, *h)[:2] for h in r.history[::20]]
    assert res[-1][0] < 1e-1 * res[0][0] and res[-1][1] < 1e-1 * res[0][1]
