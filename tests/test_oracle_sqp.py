"""Pins for the SQP path (Algorithm 1) and the bicycle model.

* Dynamics Jacobians A^-, A^+ against central differences of the residual.
* Convexification: the QP cost equals the OCP cost up to a constant (the cost
  is quadratic), C x - c equals the linearised residual f(xbar) + J (x - xbar),
  and G x lies in the shifted bounds exactly when g(x) lies in [g_lo, g_hi].
* Implicit midpoint: exact for straight-line constant-acceleration motion
  (closed form x(t) = x0 + (v0 t + a t^2 / 2) (cos yaw, sin yaw)); second-order
  accurate on a constant-steer circle against the exact arc.
* A linear problem converges in one SQP step.
* At SQP convergence the NLP stopping quantities (eq. sqp_stop) are small.
"""
import numpy as np
import pytest

from oracle.admm import ADMMSettings
from oracle.models import (BicycleOCP, midpoint_jacobians, midpoint_residual, trapezoid_jacobians,
                           trapezoid_residual)
from oracle.sqp import SQPSettings, line_search, sqp_solve, stop_test
from workloads import bicycle_batch


def _newton_step(xt, ut, dt, L, res=midpoint_residual):
    xn = xt.copy()
    for _ in range(50):
        r = res(xt, ut, xn, dt, L)
        J = np.zeros((4, 4))
        for k in range(4):
            e = np.zeros(4)
            e[k] = 1e-7
            J[:, k] = (res(xt, ut, xn + e, dt, L) - res(xt, ut, xn - e, dt, L)) / 2e-7
        xn = xn - np.linalg.solve(J, r)
        if np.max(np.abs(r)) < 1e-15:
            break
    return xn


@pytest.mark.parametrize("rule", ["midpoint", "trapezoid"])
def test_jacobians_match_central_differences(rng, rule):
    res, jac = ((midpoint_residual, midpoint_jacobians) if rule == "midpoint"
                else (trapezoid_residual, trapezoid_jacobians))
    for _ in range(20):
        xt = rng.normal(size=4) + np.array([0, 0, 0, 6.0])
        xn = xt + 0.1 * rng.normal(size=4)
        ut = rng.uniform(-0.3, 0.3, size=2)
        Am, Ap = jac(xt, ut, xn, 0.05, 2.5)
        h = 1e-6
        for k in range(6):
            e = np.zeros(6)
            e[k] = h
            zp, zm = np.concatenate([xt, ut]) + e, np.concatenate([xt, ut]) - e
            d = (res(zp[:4], zp[4:], xn, 0.05, 2.5) - res(zm[:4], zm[4:], xn, 0.05, 2.5)) / (2 * h)
            np.testing.assert_allclose(Am[:, k], d, atol=1e-8)
        for k in range(4):
            e = np.zeros(4)
            e[k] = h
            d = (res(xt, ut, xn + e, 0.05, 2.5) - res(xt, ut, xn - e, 0.05, 2.5)) / (2 * h)
            np.testing.assert_allclose(Ap[:, k], d, atol=1e-8)
        np.testing.assert_allclose(Ap[:, 4:], 0.0)


def test_trapezoid_exact_for_constant_acceleration_line_and_second_order_on_circle():
    """The trapezoidal rule integrates v' = a exactly along a straight line
    (the position is quadratic in time) and is second-order on a circle;
    it differs from the midpoint rule once the heading turns."""
    dt, L, yaw, v0, a = 0.05, 2.5, 0.3, 5.0, 1.7
    x = np.array([1.0, -2.0, yaw, v0])
    for t in range(1, 40):
        x = _newton_step(x, np.array([a, 0.0]), dt, L, trapezoid_residual)
        tt = t * dt
        s = v0 * tt + 0.5 * a * tt ** 2
        np.testing.assert_allclose(x, [1.0 + s * np.cos(yaw), -2.0 + s * np.sin(yaw), yaw, v0 + a * tt], atol=1e-11)
    Lw, v, d = 2.5, 8.0, 0.2
    w = v * np.tan(d) / Lw
    errs, last = [], None
    for dt in (0.05, 0.025):
        x = np.array([0.0, 0.0, 0.0, v])
        T = 2.0
        for _ in range(int(round(T / dt))):
            x = _newton_step(x, np.array([0.0, d]), dt, Lw, trapezoid_residual)
        exact = np.array([v / w * np.sin(w * T), v / w * (1 - np.cos(w * T)), w * T, v])
        errs.append(np.max(np.abs(x - exact)))
        last = x
    assert errs[0] < 1e-2 and 3.5 < errs[0] / errs[1] < 4.5
    xm = np.array([0.0, 0.0, 0.0, v])
    for _ in range(80):
        xm = _newton_step(xm, np.array([0.0, d]), 0.025, Lw)
    assert np.max(np.abs(xm - last)) > 1e-6


def test_midpoint_exact_for_constant_acceleration_line():
    dt, L, yaw, v0, a = 0.05, 2.5, 0.3, 5.0, 1.7
    x = np.array([1.0, -2.0, yaw, v0])
    for t in range(1, 40):
        x = _newton_step(x, np.array([a, 0.0]), dt, L)
        tt = t * dt
        s = v0 * tt + 0.5 * a * tt ** 2
        np.testing.assert_allclose(x, [1.0 + s * np.cos(yaw), -2.0 + s * np.sin(yaw), yaw, v0 + a * tt], atol=1e-11)


def test_midpoint_second_order_on_circle():
    L, v, d = 2.5, 8.0, 0.2
    w = v * np.tan(d) / L
    errs = []
    for dt in (0.05, 0.025):
        x = np.array([0.0, 0.0, 0.0, v])
        T = 2.0
        for _ in range(int(round(T / dt))):
            x = _newton_step(x, np.array([0.0, d]), dt, L)
        exact = np.array([v / w * np.sin(w * T), v / w * (1 - np.cos(w * T)), w * T, v])
        errs.append(np.max(np.abs(x - exact)))
    assert errs[0] < 1e-2 and 3.5 < errs[0] / errs[1] < 4.5


@pytest.mark.parametrize("racing", [False, True], ids=["tracking", "rate_cost_and_u_init"])
def test_convexification_pins(rng, racing):
    """racing: the control-rate cost (cross-stage E_t) and u_0 = u_init."""
    b = bicycle_batch(2, N=12, seed=91)
    if racing:
        b.Wd = np.array([3.0, 40.0])
        b.u_init = np.array([[0.4, -0.05], [-0.7, 0.1]])
    ocp = BicycleOCP(b, 1)
    zbar = ocp.initial_guess() + 0.05 * rng.normal(size=(ocp.N + 1, 6))
    qp = ocp.convexify(zbar)
    P, C, G, q, c, lo, hi = qp.matrices()
    # cost: QP objective and OCP cost differ by a constant
    consts = []
    for _ in range(4):
        z = zbar + 0.3 * rng.normal(size=zbar.shape)
        x = z.reshape(-1)
        consts.append(ocp.cost(z) - (0.5 * x @ (P @ x) + q @ x))
    assert np.ptp(consts) < 1e-9
    # equality rows: C x - c = f(zbar) + J (x - zbar), J by central differences
    dz = 1e-3 * rng.normal(size=zbar.shape)
    lin = C @ (zbar + dz).reshape(-1) - c
    f0 = ocp.eq_residual(zbar)
    h = 1e-6
    jd = (ocp.eq_residual(zbar + h * dz) - ocp.eq_residual(zbar - h * dz)) / (2 * h)
    np.testing.assert_allclose(lin, f0 + jd, atol=1e-9)
    # inequality rows: linear g, so the shifted bounds are exact
    z = zbar + rng.normal(size=zbar.shape)
    g = ocp.ineq(z).reshape(-1)
    Gx = G @ z.reshape(-1)
    np.testing.assert_allclose(Gx - lo, g - ocp.g_lo.reshape(-1), atol=1e-12)
    np.testing.assert_allclose(hi - Gx, ocp.g_hi.reshape(-1) - g, atol=1e-12)
    if racing:
        # the two control rows of stage 0 are the equality u_0 = u_init
        np.testing.assert_array_equal(lo[:2], b.u_init[1])
        np.testing.assert_array_equal(hi[:2], b.u_init[1])


class _LinearOCP:
    """A linear-quadratic OCP exposed through the same interface the SQP uses."""

    def __init__(self, N=15, seed=7):
        rng = np.random.default_rng(seed)
        self.N, self.nx, self.nu, self.ng = N, 3, 2, 2
        self.A = np.eye(3) + 0.1 * rng.normal(size=(3, 3))
        self.B = rng.normal(size=(3, 2))
        self.x_init = rng.normal(size=3)
        self.ref = rng.normal(size=(N + 1, 5))
        self.W = np.diag([1.0, 2.0, 0.5, 0.3, 0.3])
        self.g_lo = np.array([-0.2, -0.3])
        self.g_hi = np.array([0.25, 0.3])
        self.soft = np.array([0, 0])
        self.gamma1 = 1.0

    def initial_guess(self):
        # a feasible rollout with zero controls: with the paper's penalty rule
        # (no curvature term in mu) a unit step from an infeasible start can be
        # rejected, so one-step convergence is stated from a feasible start
        z = np.zeros((self.N + 1, 5))
        z[0, :3] = self.x_init
        for t in range(self.N):
            z[t + 1, :3] = self.A @ z[t, :3]
        return z

    def cost(self, z):
        e = z - self.ref
        return 0.5 * np.einsum("ti,ij,tj->", e, self.W, e)

    def cost_grad(self, z):
        return (z - self.ref) @ self.W

    def eq_residual(self, z):
        r = [z[0, :3] - self.x_init]
        for t in range(self.N):
            r.append(self.A @ z[t, :3] + self.B @ z[t, 3:] - z[t + 1, :3])
        return np.concatenate(r)

    def eq_jac_T_times(self, z, y):
        out = np.zeros_like(z)
        out[0, :3] += y[:3]
        for t in range(self.N):
            yt = y[3 + 3 * t: 6 + 3 * t]
            out[t, :3] += self.A.T @ yt
            out[t, 3:] += self.B.T @ yt
            out[t + 1, :3] -= yt
        return out

    def G_block(self, t):
        return np.array([[0, 0, 0, 1.0, 0], [0, 0, 0, 0, 1.0]])

    def g_const(self, t):
        return np.zeros(2)

    def ineq(self, z):
        return z[:, 3:].copy()

    def convexify(self, z):
        from oracle.qp import StageQP
        N = self.N
        Am = np.tile(np.hstack([self.A, self.B]), (N, 1, 1))
        Ap = np.tile(np.hstack([-np.eye(3), np.zeros((3, 2))]), (N, 1, 1))
        return StageQP(nx=3, nu=2, N=N, D=np.tile(self.W, (N + 1, 1, 1)), E=np.zeros((N, 5, 5)),
                       q=-(self.ref @ self.W), Am=Am, Ap=Ap, b=np.zeros((N, 3)), x_init=self.x_init,
                       G=np.tile(self.G_block(0), (N + 1, 1, 1)), lo=np.tile(self.g_lo, (N + 1, 1)),
                       hi=np.tile(self.g_hi, (N + 1, 1)))


def test_linear_problem_converges_in_one_sqp_step():
    ocp = _LinearOCP()
    tight = ADMMSettings(eps_abs=1e-11, eps_rel=1e-11, max_iter=20000)
    r = sqp_solve(ocp, SQPSettings(max_sqp=5, fixed_iters=False, eps_c=1e-8), admm=tight)
    assert r.converged and r.sqp_iters == 1 and r.alphas == [1.0]
    assert np.any(np.abs(r.z[:, 3:]) >= 0.2 - 1e-9)  # bounds are active


@pytest.mark.parametrize("integrator", [0, 1], ids=["midpoint", "trapezoid"])
def test_bicycle_sqp_reaches_nlp_kkt_point(integrator):
    b = bicycle_batch(1, N=20, seed=92)
    b.integrator = integrator
    ocp = BicycleOCP(b, 0)
    tight = ADMMSettings(eps_abs=1e-11, eps_rel=1e-11, max_iter=20000)
    r = sqp_solve(ocp, SQPSettings(max_sqp=25, fixed_iters=False, eps_c=1e-7), admm=tight)
    assert r.converged
    s = stop_test(ocp, r.z, r.xi, r.y_f, r.y_g)
    assert max(s.values()) < 1e-7
    # started at the converged point, one more iteration stays there
    r2 = sqp_solve(ocp, SQPSettings(max_sqp=1, fixed_iters=True), admm=tight, z0=r.z)
    np.testing.assert_allclose(r2.z, r.z, atol=1e-6)


def test_line_search_unit_step_and_fallback():
    """Along the QP step from a feasible point the unit step passes the Armijo
    test; along the reversed step every candidate increases the merit, so the
    fallback returns the candidate with the smallest merit (the shortest)."""
    ocp = _LinearOCP()
    z0 = ocp.initial_guess()
    xi = np.zeros((ocp.N + 1, ocp.ng))
    tight = ADMMSettings(eps_abs=1e-11, eps_rel=1e-11, max_iter=20000)
    r = sqp_solve(ocp, SQPSettings(max_sqp=1), admm=tight)
    dz = r.z - z0
    a, mu = line_search(ocp, z0, xi, dz, xi, 0.0, SQPSettings())
    assert a == 1.0 and mu >= 1.0
    a_bad, _ = line_search(ocp, z0, xi, -dz, xi, 0.0, SQPSettings())
    assert a_bad == 2.0 ** -7
