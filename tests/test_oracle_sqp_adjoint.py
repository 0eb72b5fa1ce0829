"""Pins for the implicit derivative of the SQP solution (oracle.sqp_adjoint).

* The dynamics Hessian sum_t y_t' grad^2 f_t equals central differences of
  the Lagrangian gradient grad l(z) + grad f(z)' y (both integrators).
* Parameter gradients of a loss of the converged SQP solution (exact
  Lagrangian Hessian) equal central differences of tightly converged oracle
  SQP solves, for x0, the cost weights, a reference point and the bounds.
"""
import numpy as np
import pytest

from oracle.admm import ADMMSettings
from oracle.models import BicycleOCP
from oracle.sqp import SQPSettings, sqp_solve
from oracle.sqp_adjoint import dynamics_hessian, sqp_param_grads
from workloads import bicycle_batch


def _lagrangian_grad(ocp, z, y):
    return (ocp.cost_grad(z) + ocp.eq_jac_T_times(z, y)).reshape(-1)


@pytest.mark.parametrize("integrator", [0, 1], ids=["midpoint", "trapezoid"])
def test_dynamics_hessian_matches_fd_of_the_lagrangian_gradient(integrator):
    b = bicycle_batch(1, N=6, seed=3)
    b.integrator = integrator
    ocp = BicycleOCP(b, 0)
    rng = np.random.default_rng(1)
    z = ocp.initial_guess() + 0.2 * rng.standard_normal((ocp.N + 1, 6))
    y = rng.standard_normal(4 * (ocp.N + 1))
    Hd, He = dynamics_hessian(ocp, z, y[4:].reshape(ocp.N, 4), trapezoid=integrator == 1)
    n = 6
    H = np.zeros(((ocp.N + 1) * n,) * 2)
    for t in range(ocp.N + 1):
        H[t * n:(t + 1) * n, t * n:(t + 1) * n] = Hd[t] + ocp.stage_weights(t)
    for t in range(ocp.N):
        H[(t + 1) * n:(t + 2) * n, t * n:(t + 1) * n] = He[t]
        H[t * n:(t + 1) * n, (t + 1) * n:(t + 2) * n] = He[t].T
    h = 1e-6
    fd = np.zeros_like(H)
    zf = z.reshape(-1)
    for k in range(zf.size):
        zp, zm = zf.copy(), zf.copy()
        zp[k] += h
        zm[k] -= h
        fd[:, k] = (_lagrangian_grad(ocp, zp.reshape(z.shape), y) - _lagrangian_grad(ocp, zm.reshape(z.shape), y)) / (2 * h)
    np.testing.assert_allclose(H, fd, atol=1e-7)


TIGHT_SQP = SQPSettings(max_sqp=60, eps_c=1e-10, fixed_iters=False)
TIGHT_ADMM = ADMMSettings(eps_abs=1e-12, eps_rel=1e-12, max_iter=100000, k_check=25)


def _solve(ocp, z0=None):
    r = sqp_solve(ocp, TIGHT_SQP, admm=TIGHT_ADMM, z0=z0)
    assert r.converged
    return r


def test_sqp_parameter_gradients_match_central_fd():
    b = bicycle_batch(3, N=12, seed=3)
    ocp = BicycleOCP(b, 1)
    r = _solve(ocp)
    rng = np.random.default_rng(4)
    c = rng.standard_normal((ocp.N + 1, 6))
    g = sqp_param_grads(ocp, r.z, r.xi, r.y_f, r.y_g, c, exact=True)
    gn = sqp_param_grads(ocp, r.z, r.xi, r.y_f, r.y_g, c, exact=False)
    h = 1e-5

    def fd(get, put):
        base = get()
        vals = []
        for s in (1.0, -1.0):
            put(base + s * h)
            vals.append(float(np.sum(c * _solve(ocp).z)))
        put(base)
        return (vals[0] - vals[1]) / (2 * h)

    def arr_item(obj, name, idx):
        arr = getattr(obj, name)
        return (lambda: arr[idx]), (lambda v: arr.__setitem__(idx, v))

    checks = []
    for j in (0, 3):
        checks.append(("x0", j, *arr_item(ocp, "x_init", j), g["x0"][j]))
    checks.append(("Q", 1, *arr_item(ocp, "Q", (1, 1)), g["Qd"][1]))
    checks.append(("Q", 2, *arr_item(ocp, "Q", (2, 2)), g["Qd"][2]))
    checks.append(("R", 1, *arr_item(ocp, "R", (1, 1)), g["Rd"][1]))
    checks.append(("Qf", 0, *arr_item(ocp, "Qf", (0, 0)), g["Qfd"][0]))
    checks.append(("ref", (5, 1), *arr_item(ocp, "ref", (5, 1)), g["ref"][5, 1]))
    checks.append(("ref", (8, 2), *arr_item(ocp, "ref", (8, 2)), g["ref"][8, 2]))
    worst_gn = 0.0
    for name, idx, get, put, want in checks:
        got = fd(get, put)
        assert abs(got - want) <= 1e-4 * max(1.0, abs(got)), (name, idx, got, want)
    # the Gauss-Newton form drops the dynamics curvature: visibly different here
    worst_gn = max(abs(g[k] - gn[k]).max() for k in ("x0", "Qd", "Rd"))
    assert worst_gn > 1e-6
