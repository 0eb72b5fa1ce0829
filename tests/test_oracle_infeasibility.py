"""Pins for the primal-infeasibility status (OCP_INFEASIBLE = 4).

A scalar system x_{t+1} = x_t + u_t from x_0 = 0 with |u_t| <= 1 reaches at
most 2 by t = 2; asking x_2 >= 5 makes the constraint set empty.  Hand
derivation of a Farkas certificate (variables (x_t, u_t), rows: initial state,
dynamics x_t + u_t - x_{t+1} = 0 for t = 0, 1, and the box rows x_t, u_t):
dy_g(u_0) = dy_g(u_1) = 1, dy_g(x_2) = -1, dy_dyn = (-1, -1), dy_init = 1
gives A'dy = 0 and the support value hi(u_0) + hi(u_1) - lo(x_2) = 1 + 1 - 5
= -3 < 0.  With lo(x_2) = 1.5 (reachable) the same dy has support 0.5 > 0.
"""
import numpy as np

from oracle.admm import PRIMAL_INFEASIBLE, ADMMSettings, _QPMats, admm_solve, infeasibility_certificate
from oracle.qp import lti_qp
from oracle.scaling import box_scaling
from workloads import random_lti
from oracle.qp import lti_batch_qp


def _scalar_qp(lo_x2):
    qp = lti_qp(np.array([[1.0]]), np.array([[1.0]]), np.array([1.0]), np.array([0.1]), np.array([1.0]),
                np.eye(2), np.array([-100.0, -1.0]), np.array([100.0, 1.0]), np.array([0.0]), 2)
    qp.lo[2, 0] = lo_x2
    return qp


def _hand_certificate():
    dy_f = np.array([1.0, -1.0, -1.0])  # initial row, dynamics rows 0 and 1
    dy_g = np.array([0.0, 1.0, 0.0, 1.0, -1.0, 0.0])  # (x0, u0, x1, u1, x2, u2)
    return dy_f, dy_g


def test_hand_certificate():
    dy_f, dy_g = _hand_certificate()
    M = _QPMats(_scalar_qp(5.0))
    np.testing.assert_array_equal(M.C.T @ dy_f + M.G.T @ dy_g, np.zeros(6))
    assert infeasibility_certificate(M, dy_f, dy_g, 1e-4)
    assert infeasibility_certificate(M, 7.5 * dy_f, 7.5 * dy_g, 1e-4)  # any positive multiple
    assert not infeasibility_certificate(_QPMats(_scalar_qp(1.5)), dy_f, dy_g, 1e-4)
    assert not infeasibility_certificate(M, -dy_f, -dy_g, 1e-4)  # support +3
    assert not infeasibility_certificate(M, np.zeros(3), np.zeros(6), 1e-4)


def test_admm_reports_the_infeasible_problem():
    st = ADMMSettings(eps_abs=1e-6, eps_rel=1e-6, max_iter=5000)
    r = admm_solve(_scalar_qp(5.0), st)
    assert r.status == PRIMAL_INFEASIBLE and r.iters < 5000
    r = admm_solve(_scalar_qp(5.0), st, scaling=box_scaling(_scalar_qp(5.0), 0.6))
    assert r.status == PRIMAL_INFEASIBLE
    assert admm_solve(_scalar_qp(1.5), st).status == 0


def test_feasible_instances_are_never_flagged():
    b = random_lti(24, N=30, seed=2, x_bound=1e3)  # loose state boxes: feasible
    st = ADMMSettings(eps_abs=1e-4, eps_rel=1e-4, max_iter=1000)
    for i in range(b.batch):
        assert admm_solve(lti_batch_qp(b, i), st).status != PRIMAL_INFEASIBLE
