"""Pins for the racing features of the bicycle OCP (Sec. "Hardware
Deployment: Autonomous Racing"): the control-rate cost of eq. cost and the
fixed first control (x_0, u_0) = (x_init, u_init).

* The rate term's value on step-shaped control sequences (closed form).
* A converged SQP solution keeps u_0 = u_init and meets the SQP stop test
  (its stationarity includes the rate gradient).
* A very large rate weight freezes the controls at u_init; without u_init
  and without rate cost the first control moves.
* The implicit SQP derivative with both features matches central
  differences of converged SQP solves (the cost's cross-stage Hessian blocks
  add to the dynamics curvature).
"""
import numpy as np
import pytest

from oracle.admm import ADMMSettings
from oracle.models import BicycleOCP
from oracle.sqp import SQPSettings, sqp_solve
from oracle.sqp_adjoint import sqp_param_grads
from workloads import bicycle_batch

TIGHT_SQP = SQPSettings(max_sqp=60, eps_c=1e-9, fixed_iters=False)
TIGHT_ADMM = ADMMSettings(eps_abs=1e-12, eps_rel=1e-12, max_iter=100000, k_check=25)


def _racing_batch(Wd=(2.0, 30.0), seed=3, N=12):
    b = bicycle_batch(3, N=N, seed=seed)
    b.Wd = np.array(Wd, dtype=float)
    b.u_init = np.array([[0.3, 0.02], [-0.5, -0.04], [0.8, 0.05]])
    return b


def test_rate_cost_closed_form():
    b = _racing_batch(Wd=(2.0, 30.0))
    ocp = BicycleOCP(b, 0)
    z = ocp.initial_guess()
    z[:, 4:] = 0.0
    base = ocp.cost(z)  # tracking part only (controls zero, reference states)
    s = 0.7
    for k, j, diffs in ((0, 0, 1), (5, 1, 2), (ocp.N, 1, 1)):
        zz = z.copy()
        zz[k, 4 + j] = s
        rate = 0.5 * b.Wd[j] * s * s * diffs
        tracking = 0.5 * b.Rd[j] * s * s
        assert ocp.cost(zz) - base == pytest.approx(rate + tracking, rel=1e-14)
    # a constant control sequence has no rate cost
    zz = z.copy()
    zz[:, 4:] = [0.2, -0.1]
    assert ocp.cost(zz) - base == pytest.approx((ocp.N + 1) * 0.5 * (b.Rd[0] * 0.04 + b.Rd[1] * 0.01), rel=1e-13)


def test_converged_sqp_keeps_the_first_control():
    b = _racing_batch()
    for i in range(b.batch):
        ocp = BicycleOCP(b, i)
        r = sqp_solve(ocp, SQPSettings(max_sqp=40, eps_c=1e-7), admm=TIGHT_ADMM)
        assert max(r.stop.values()) < 1e-5, r.stop
        np.testing.assert_allclose(r.z[0, 4:], b.u_init[i], atol=1e-7)


def test_large_rate_weight_freezes_the_controls():
    loose = ADMMSettings(eps_abs=1e-8, eps_rel=1e-8, max_iter=20000, k_check=25)
    b = _racing_batch(Wd=(1e4, 1e4))
    ocp = BicycleOCP(b, 0)
    r = sqp_solve(ocp, SQPSettings(max_sqp=30, eps_c=1e-6), admm=loose)
    assert r.converged
    assert np.max(np.abs(r.z[:, 4:] - b.u_init[0])) < 2e-3
    free = bicycle_batch(3, N=12, seed=3)
    rf = sqp_solve(BicycleOCP(free, 0), SQPSettings(max_sqp=30, eps_c=1e-6), admm=loose)
    assert np.max(np.abs(rf.z[0, 4:] - b.u_init[0])) > 1e-2


def test_sqp_derivative_with_rate_cost_matches_central_fd():
    b = _racing_batch()
    ocp = BicycleOCP(b, 1)

    def solve():
        r = sqp_solve(ocp, TIGHT_SQP, admm=TIGHT_ADMM)
        assert r.converged
        return r

    r = solve()
    c = np.random.default_rng(4).standard_normal((ocp.N + 1, 6))
    g = sqp_param_grads(ocp, r.z, r.xi, r.y_f, r.y_g, c, exact=True)
    h = 1e-5

    def fd(arr, idx):
        base = arr[idx]
        vals = []
        for sgn in (1.0, -1.0):
            arr[idx] = base + sgn * h
            vals.append(float(np.sum(c * solve().z)))
        arr[idx] = base
        return (vals[0] - vals[1]) / (2 * h)

    for name, arr, idx, want in (("x0", ocp.x_init, 1, g["x0"][1]), ("Q", ocp.Q, (2, 2), g["Qd"][2]),
                                 ("R", ocp.R, (0, 0), g["Rd"][0]), ("ref", ocp.ref, (6, 0), g["ref"][6, 0])):
        got = fd(arr, idx)
        assert abs(got - want) <= 1e-4 * max(1.0, abs(got)), (name, got, want)
