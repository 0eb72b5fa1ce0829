"""Pins for the rescaled ADMM solve (Remark 4, "Rescaling").

* The rescaled data: cost and constraints of the scaled QP at xh = x / d equal
  c times the original cost and the row-scaled original constraints, at random
  points (a dropped factor, a transposed scaling or a wrong row factor fails).
* The identity scaling reproduces the unscaled iterates bit for bit.
* The scaled solve converges to the polished optimum of the original problem
  and its multipliers, mapped back, satisfy the original KKT stationarity.
* The point maps are inverse to each other and carry the scaled problem's
  KKT residuals to c diag(d) times the original ones.
* The box normalisation of the random-LTI workload has the closed form
  d = (half width)^p, e_g = 1/d, c = 1/max_j d_j^2 P_jj.
* The stopping test and the reported residuals are those of the original
  problem.
"""
import numpy as np
import pytest

from oracle.adjoint import polish
from oracle.admm import ADMMSettings, _QPMats, admm_solve, kkt_residuals
from oracle.qp import lti_batch_qp
from oracle.scaling import Scaling, box_scaling, identity_scaling, scale_qp, to_scaled, to_unscaled
from workloads import double_integrator, random_lti


def _qp(i=0, N=12):
    return lti_batch_qp(random_lti(4, N=N, seed=2), i)


def _random_scaling(qp, rng):
    return Scaling(rng.uniform(0.2, 5.0, qp.n), rng.uniform(0.2, 5.0, qp.ng), float(rng.uniform(0.01, 10.0)))


def test_scaled_data_at_corresponding_points(rng):
    qp = _qp()
    qp.q[:] = rng.normal(size=qp.q.shape)
    qp.b[:] = rng.normal(size=qp.b.shape)
    qp.E[:] = 0.1 * rng.normal(size=qp.E.shape)
    sc = _random_scaling(qp, rng)
    qs = scale_qp(qp, sc)
    P, C, G, q, c, lo, hi = qp.matrices()
    Ps, Cs, Gs, qs_, cs, los, his = qs.matrices()
    N1 = qp.N + 1
    dv = np.tile(sc.d, N1)
    ef = np.tile(1.0 / sc.d[:qp.nx], N1)
    eg = np.tile(sc.e_g, N1)
    for _ in range(3):
        x = rng.normal(size=qp.nvar)
        xh = x / dv
        f = 0.5 * x @ (P @ x) + q @ x
        fh = 0.5 * xh @ (Ps @ xh) + qs_ @ xh
        assert fh == pytest.approx(sc.c * f, rel=1e-12)
        np.testing.assert_allclose(Cs @ xh - cs, ef * (C @ x - c), rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(Gs @ xh, eg * (G @ x), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(los, eg * lo)
    np.testing.assert_allclose(his, eg * hi)
    # the structure the kernels rely on survives: A+ = [-I 0] and A_init = [I 0]
    np.testing.assert_array_equal(qs.Ap, qp.Ap)
    assert np.array_equal(Cs[:qp.nx, :qp.n].toarray(), C[:qp.nx, :qp.n].toarray())


def test_identity_scaling_gives_the_same_iterates():
    qp = _qp()
    st = ADMMSettings(max_iter=80, k_check=0)
    a = admm_solve(qp, st, record=True)
    b = admm_solve(qp, st, record=True, scaling=identity_scaling(qp))
    for u, v in zip(a.history, b.history):
        for p, r in zip(u, v):
            np.testing.assert_array_equal(p, r)
    assert a.rho_changes == b.rho_changes


def test_scaled_solve_reaches_the_original_optimum(rng):
    tight = ADMMSettings(eps_abs=1e-11, eps_rel=1e-11, max_iter=50000)
    for i in range(2):
        qp = _qp(i)
        ok, ref = polish(qp, *(lambda r: (r.x, r.y_g))(admm_solve(qp, tight)), eps_solve=1e-8)
        assert ok
        for sc in (box_scaling(qp, 0.6), _random_scaling(qp, rng)):
            r = admm_solve(qp, tight, scaling=sc)
            assert r.status == 0
            assert np.max(np.abs(r.x - ref["x"])) < 1e-8 * max(1.0, np.max(np.abs(ref["x"])))
            # mapped-back multipliers satisfy the original KKT stationarity
            P, C, G, q, c, lo, hi = qp.matrices()
            stat = P @ r.x + q + C.T @ r.y_f + G.T @ r.y_g
            assert np.max(np.abs(stat)) < 1e-8 * max(1.0, np.max(np.abs(q)), np.max(np.abs(r.y_f)))
            np.testing.assert_allclose(r.y_f, ref["y_f"], atol=1e-6 * max(1.0, np.max(np.abs(ref["y_f"]))))


def test_point_maps_are_inverse_and_carry_the_kkt_residuals(rng):
    qp = _qp()
    qp.q[:] = rng.normal(size=qp.q.shape)
    sc = _random_scaling(qp, rng)
    qs = scale_qp(qp, sc)
    v = (rng.normal(size=qp.nvar), rng.normal(size=qp.nineq), np.zeros(qp.nineq), rng.normal(size=qp.neq),
         rng.normal(size=qp.nineq))
    back = to_unscaled(qp, sc, *to_scaled(qp, sc, *v))
    for a, b in zip(v, back):
        np.testing.assert_allclose(b, a, rtol=1e-13, atol=1e-13)
    P, C, G, q, c, lo, hi = qp.matrices()
    Ps, Cs, Gs, qs_, cs, los, his = qs.matrices()
    x, zg, xi, yf, yg = v
    xh, zh, xih, yfh, ygh = to_scaled(qp, sc, *v)
    dv = np.tile(sc.d, qp.N + 1)
    stat = P @ x + q + C.T @ yf + G.T @ yg
    stat_h = Ps @ xh + qs_ + Cs.T @ yfh + Gs.T @ ygh
    np.testing.assert_allclose(stat_h, sc.c * dv * stat, rtol=1e-11, atol=1e-11)


def test_box_scaling_closed_form():
    """Random LTI: x in [-10, 10], u in [-1, 1], Q = diag(U[0.5, 2]), R = 0.1 I:
    10^0.6 = 3.98 rounds to d_x = 4, 1^0.6 = 1 gives d_u = 1; the largest
    diagonal entry of diag(d) D diag(d) is 16 max Q_jj in [8, 32], so c is
    1/8, 1/16 or 1/32 by where 16 max Q_jj falls against 8 sqrt 2 and 16 sqrt 2."""
    b = random_lti(2, N=5, seed=2)
    for i in range(2):
        qp = lti_batch_qp(b, i)
        sc = box_scaling(qp, 0.6)
        np.testing.assert_array_equal(sc.d, np.concatenate([np.full(b.nx, 4.0), np.ones(b.nu)]))
        np.testing.assert_array_equal(sc.e_g, 1.0 / sc.d)
        m = 16.0 * max(np.max(b.Qd[i]), np.max(b.Qfd[i]))
        expect = 1 / 8 if m < 8 * np.sqrt(2) else (1 / 16 if m < 16 * np.sqrt(2) else 1 / 32)
        assert sc.c == expect


def test_stopping_test_and_residuals_are_the_original_problems():
    qp = lti_batch_qp(double_integrator(1, N=20, seed=1), 0)
    st = ADMMSettings(eps_abs=1e-6, eps_rel=1e-6, max_iter=5000)
    r = admm_solve(qp, st, scaling=box_scaling(qp, 0.6))
    assert r.status == 0
    rp, rd, ps, ds = kkt_residuals(qp, r.x, r.z_g, r.xi, r.y_f, r.y_g)
    assert r.r_prim == pytest.approx(rp, rel=1e-12, abs=1e-15)
    assert r.r_dual == pytest.approx(rd, rel=1e-12, abs=1e-15)
    assert rp <= 1e-6 + 1e-6 * ps and rd <= 1e-6 + 1e-6 * ds
