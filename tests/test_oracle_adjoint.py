"""Pins for the implicit-differentiation VJP (Algorithm 2; Appendix
"Backward Pass").

* Central finite differences (h = 1e-6) of exactly solved (polished) QPs.
* Closed form: with no inequality active, x_N = Phi x0 and u_0 = -K_0 x0
  (LQR), so dL/dx0 = 2 (K_0'K_0 + Phi'Phi) x0 for L = ||u_0||^2 + ||x_N||^2.
* The regularised iterative-refinement adjoint equals the dense solve.
"""
import numpy as np
import pytest

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


def _l2_slack_qp():
    """Double integrator whose position rows carry an L2 slack and bind: the
    start lies outside the tightened position box, so the first stages hold
    nonzero slack."""
    from oracle.qp import SOFT_L2, lti_batch_qp
    from workloads import double_integrator

    b = double_integrator(1, N=12, seed=3)
    b.x0[0, :2] = [1.8, -1.6]
    qp = lti_batch_qp(b, 0)
    kinds = np.zeros(qp.ng, dtype=np.int64)
    kinds[:2] = SOFT_L2
    qp.soft = kinds
    qp.gamma2 = 4.0
    qp.lo[:, :2] = -1.0
    qp.hi[:, :2] = 1.0
    return qp


def _admm_exact(qp, warm=None):
    from oracle.admm import ADMMSettings, admm_solve

    return admm_solve(qp, ADMMSettings(eps_abs=1e-13, eps_rel=1e-13, max_iter=400000), warm=warm)


def test_l2_slack_adjoint_matches_central_fd_of_admm_solutions():
    """eq. bwd:slack_reduced_system: eta on a QP with active L2-slack rows,
    against central differences of the ADMM solutions (the smoothed slack
    projection, an independent route to the optimum), h = 1e-5."""
    from oracle.adjoint import polish, qp_vjp
    from oracle.qp import SOFT_L2

    qp = _l2_slack_qp()
    r = _admm_exact(qp)
    ok, sol = polish(qp, r.x, r.y_g, xi=r.xi, eps_solve=1e-8)
    assert ok
    lower, upper = sol["lower"], sol["upper"]
    l2 = (lower | upper) & (qp.soft_rows() == SOFT_L2)
    assert l2.sum() >= 2 and np.all(np.abs(sol["xi"][l2]) > 1e-3)
    np.testing.assert_allclose(sol["xi"], r.xi, atol=1e-8)
    g = np.random.default_rng(5).standard_normal(qp.nvar)
    ex, ef, eg = adjoint_dense(qp, sol["x"], g, lower, upper)
    grads = qp_vjp(qp, sol["x"], ex, ef, eg, lower, upper, xi=sol["xi"])
    warm = {"x": r.x, "z_g": r.z_g, "y_f": r.y_f, "y_g": r.y_g, "rho_bar": r.rho_bar}
    h = 1e-5

    def fd(field, idx):
        vals = []
        for sgn in (1.0, -1.0):
            arr = getattr(qp, field)
            old = arr[idx]
            arr[idx] = old + sgn * h
            vals.append(g @ _admm_exact(qp, warm).x)
            arr[idx] = old
        return (vals[0] - vals[1]) / (2 * h)

    rows = np.flatnonzero(l2)
    t0, r0 = divmod(int(rows[0]), qp.ng)
    checks = [("q", (0, 4), grads["d_q"][0, 4]), ("q", (5, 1), grads["d_q"][5, 1]),
              ("x_init", (0,), grads["d_x_init"][0]), ("x_init", (3,), grads["d_x_init"][3])]
    bound = "lo" if lower[rows[0]] else "hi"
    checks.append((bound, (t0, r0), grads["d_" + bound][t0, r0]))
    for field, idx, want in checks:
        got = fd(field, idx)
        assert abs(got - want) <= 1e-4 * max(1.0, abs(want)), (field, idx, got, want)
    # the slack weight itself (Sec. "Backward pass", slack variables)
    vals = []
    for sgn in (1.0, -1.0):
        qp.gamma2 = 4.0 + sgn * h
        vals.append(g @ _admm_exact(qp, warm).x)
    qp.gamma2 = 4.0
    got = (vals[0] - vals[1]) / (2 * h)
    assert abs(got - grads["d_gamma2"]) <= 1e-4 * max(1.0, abs(got)), (got, grads["d_gamma2"])
    assert abs(grads["d_gamma2"]) > 1e-4
    # the slack rows' adjoint multipliers satisfy their row of the dense
    # system, G_S eta_x - eta_y / gamma2 = 0, and are not all zero
    G = qp.matrices()[2]
    np.testing.assert_allclose(eg[l2], qp.gamma2 * (G @ ex)[l2], atol=1e-10)
    assert np.any(np.abs(eg[l2]) > 1e-3)


def test_l2_slack_refinement_equals_dense_adjoint():
    """The reduced system of the GPU scheme (slack rows in H, eta_y recovered)
    equals the full active-set KKT solve with its -1/gamma2 slack diagonal."""
    from oracle.adjoint import polish

    qp = _l2_slack_qp()
    r = _admm_exact(qp)
    ok, sol = polish(qp, r.x, r.y_g, xi=r.xi, eps_solve=1e-8)
    assert ok
    g = np.random.default_rng(6).standard_normal(qp.nvar)
    e1 = adjoint_dense(qp, sol["x"], g, sol["lower"], sol["upper"])
    e2 = adjoint_refined(qp, sol["x"], g, sol["lower"], sol["upper"], sweeps=6)
    for a, c in zip(e1, e2):
        np.testing.assert_allclose(c, a, rtol=1e-9, atol=1e-11 * max(1.0, np.abs(a).max()))


def _dependent_active_set():
    """Random LTI QP solved exactly, with the stage-0 state rows added to the
    active set: x_0 is already fixed by the initial-state rows, so each added
    row duplicates one of them (LICQ fails, K is singular)."""
    b = random_lti(1, N=8, seed=45)
    L, g, sol = implicit_theta_grad(b, 0)
    qp = qp_of_theta(b, 0, theta_of(b, 0))
    _, gx = loss_and_grad_x(qp, sol["x"])
    lower, upper = sol["lower"].copy(), sol["upper"].copy()
    ng = qp.ng
    extra = np.zeros_like(lower)
    extra[:b.nx] = True  # rows 0..nx-1 of stage 0 select x_0 (G = I on the box rows)
    assert not np.any((lower | upper) & extra)
    return qp, sol, gx, lower, upper, lower | extra


def test_dependent_active_rows_give_the_minimum_norm_adjoint():
    from oracle.adjoint import independent_rows

    qp, sol, gx, lower, upper, lower_dep = _dependent_active_set()
    assert independent_rows(qp, lower, upper)
    assert not independent_rows(qp, lower_dep, upper)
    ex0, ef0, eg0 = adjoint_dense(qp, sol["x"], gx, lower, upper)
    ex, ef, eg = adjoint_dense(qp, sol["x"], gx, lower_dep, upper)
    nx = qp.nx
    # eta_x is unique: a duplicated row changes nothing
    np.testing.assert_allclose(ex, ex0, rtol=1e-9, atol=1e-11)
    # two identical rows share the multiplier evenly in the minimum-norm
    # solution: each gets half of what the single row carried
    np.testing.assert_allclose(ef[:nx], 0.5 * ef0[:nx], rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(eg[:nx], 0.5 * ef0[:nx], rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(ef[nx:], ef0[nx:], rtol=1e-9, atol=1e-11)
    # and the regularised refinement from zero (the GPU scheme) reaches it
    rx, rf, rg = adjoint_refined(qp, sol["x"], gx, lower_dep, upper, sweeps=8)
    for a, c in ((ex, rx), (ef, rf), (eg, rg)):
        np.testing.assert_allclose(c, a, rtol=1e-7, atol=1e-9 * max(1.0, np.abs(a).max()))


def test_proximity_tolerance_does_not_scale_with_the_multipliers():
    """Appendix "Active constraints identification": closeness to a bound is
    measured relative to the bound.  With ||y_g||_inf = 1e4 the dual threshold
    is 10 * 1e-4 * 1e4 = 10, but a row with y = 0 sitting 5 below its upper
    bound 10 is not near it (proximity tolerance 10 * 1e-4 * 10 = 1e-2)."""
    from oracle.adjoint import active_set

    b = random_lti(1, N=2, seed=46)
    qp = qp_of_theta(b, 0, theta_of(b, 0))
    x = np.zeros(qp.nvar)
    n = qp.n
    x[n + 0] = 5.0          # stage 1, state 0: 5 from the bound 10
    x[n + 1] = 10.0 - 5e-3  # stage 1, state 1: within 1e-2 of the bound
    y = np.zeros(qp.nineq)
    y[2 * qp.ng + 3] = 1e4  # a large multiplier elsewhere
    lower, upper = active_set(qp, x, y, eps_solve=1e-4)
    assert not upper[qp.ng + 0] and upper[qp.ng + 1]
    assert upper[2 * qp.ng + 3] and not lower[2 * qp.ng + 3]


def test_singularity_detection_agrees_with_the_rank_test():
    """adjoint_dense switches to the minimum-norm solve exactly when the
    active rows are dependent: on the converged C2-shaped instances of the
    sample (independent rows) the sparse LU result is kept, on the
    constructed dependent set the minimum-norm one is returned."""
    import scipy.linalg as sla

    from oracle.adjoint import _kkt, independent_rows

    qp, sol, gx, lower, upper, lower_dep = _dependent_active_set()
    for lo_, dep in ((lower, False), (lower_dep, True)):
        assert independent_rows(qp, lo_, upper) == (not dep)
        K = _kkt(qp, lo_, upper)[0]
        rhs = np.concatenate([gx, np.zeros(K.shape[0] - gx.size)])
        ex, ef, eg = adjoint_dense(qp, sol["x"], gx, lo_, upper)
        mn = sla.lstsq(K.toarray(), rhs, cond=1e-12)[0]
        np.testing.assert_allclose(np.concatenate([ex, ef]), mn[:ex.size + ef.size], rtol=1e-8, atol=1e-10)


def _slack_qp(kind, gamma):
    """Double integrator with slack position rows (L2 or L1) and a start
    outside the tightened box: the first stages hold nonzero slack."""
    from workloads import double_integrator
    from oracle.qp import lti_batch_qp

    b = double_integrator(1, N=12, seed=3)
    b.x0[0, :2] = [1.8, -1.6]
    qp = lti_batch_qp(b, 0)
    kinds = np.zeros(qp.ng, dtype=np.int64)
    kinds[:2] = kind
    qp.soft = kinds
    if kind == 1:
        qp.gamma2 = gamma
    else:
        qp.gamma1 = gamma
    qp.lo[:, :2] = -1.0
    qp.hi[:, :2] = 1.0
    return qp


@pytest.mark.parametrize("kind,gamma", [(1, 4.0), (2, 0.7)], ids=["L2", "L1"])
def test_slack_loss_gradients_match_central_fd(kind, gamma):
    """A loss on the slacks, L = g'x + h'xi (eq. loss_gradient with the
    slack block of eq. bwd:slack_adjoint): the VJP w.r.t. q, x_init, the
    bound of a slacked row and the slack weight against central differences
    (h = 1e-5) of ADMM solutions; the refinement form gives the dense one."""
    from oracle.adjoint import adjoint_refined, polish, qp_vjp

    qp = _slack_qp(kind, gamma)
    r = _admm_exact(qp)
    ok, sol = polish(qp, r.x, r.y_g, xi=r.xi, eps_solve=1e-8)
    assert ok
    xi0 = sol["xi"] if kind == 1 else r.xi
    lower, upper = sol["lower"], sol["upper"]
    rng = np.random.default_rng(8)
    g = rng.standard_normal(qp.nvar)
    hx = np.zeros(qp.nineq)
    slack = np.flatnonzero(np.abs(xi0) > 1e-3)
    assert slack.size >= 2
    hx[slack] = rng.standard_normal(slack.size)
    ex, ef, eg = adjoint_dense(qp, sol["x"], g, lower, upper, dL_dxi=hx, xi=xi0)
    e2 = adjoint_refined(qp, sol["x"], g, lower, upper, sweeps=8, dL_dxi=hx, xi=xi0)
    for a, c in zip((ex, ef, eg), e2):
        np.testing.assert_allclose(c, a, rtol=1e-8, atol=1e-10 * max(1.0, np.abs(a).max()))
    gr = qp_vjp(qp, sol["x"], ex, ef, eg, lower, upper, xi=xi0, dL_dxi=hx)
    warm = {"x": r.x, "z_g": r.z_g, "y_f": r.y_f, "y_g": r.y_g, "rho_bar": r.rho_bar}
    h = 1e-5

    def loss(res):
        return g @ res.x + hx @ res.xi

    def fd(set_, base):
        vals = []
        for sgn in (1.0, -1.0):
            set_(base + sgn * h)
            vals.append(loss(_admm_exact(qp, warm)))
        set_(base)
        return (vals[0] - vals[1]) / (2 * h)

    def setter(arr, idx):
        def f(v):
            arr[idx] = v
        return f

    t0, r0 = divmod(int(slack[0]), qp.ng)
    side = "lo" if xi0[slack[0]] > 0 else "hi"
    if kind == 1:
        side = "lo" if lower[slack[0]] else "hi"
    checks = [("q", (0, 4), gr["d_q"][0, 4]), ("q", (5, 1), gr["d_q"][5, 1]),
              ("x_init", (0,), gr["d_x_init"][0]), (side, (t0, r0), gr["d_" + side][t0, r0])]
    for field, idx, want in checks:
        arr = getattr(qp, field)
        got = fd(setter(arr, idx), arr[idx])
        assert abs(got - want) <= 1e-4 * max(1.0, abs(want)), (field, idx, got, want)
    wname = "gamma2" if kind == 1 else "gamma1"
    got = fd(lambda v: setattr(qp, wname, v), gamma)
    want = gr["d_" + wname]
    assert abs(got - want) <= 1e-4 * max(1.0, abs(got)), (wname, got, want)
    assert abs(want) > 1e-4
    # eta_xi = -G eta_x on the slacked rows (eq. bwd:slack:eta_xi_yg)
    G = qp.matrices()[2]
    np.testing.assert_allclose(gr["eta_xi"].reshape(-1)[slack], -(G @ ex)[slack], atol=1e-12)
